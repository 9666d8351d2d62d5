// Per-node device operations shared by the one-launch-per-step kernels
// (kernels.hip) and the cooperative coarse-level V-cycle (coarse.hip).
#pragma once

#include "hexmg_impl.h"

namespace hexmg {

__device__ inline void node_coords(const Level& L, int n, int& i, int& j, int& k) {
  i = n % L.nxn;
  const int t = n / L.nxn;
  j = t % L.nyn;
  k = t / L.nyn;
}

// Matrix-free K u (Sec. 4.2.1) at node n: the node gathers the rows of its
// <= 8 adjacent elements, y_n = sum_e E_e K0[a_e(n), :] u_e, so no global
// matrix and no scatter conflicts.  Supports: u is read as M u; fixed DOFs
// return u.  MODE 0: y = A u;  1: y = u + wdinv (f - A u) (damped Jacobi,
// Eq. 21);  2: y = f - A u (residual, Eq. 19).  Vectors of one right-hand side.
// TU: the type u is stored in (T, or binary32 read into binary64 arithmetic).
template <typename T, int MODE, typename TU = T>
__device__ inline void gather_node(const Level& L, const T* __restrict__ Ke, const T* __restrict__ E,
                                   const TU* __restrict__ u, const T* __restrict__ f, const T* __restrict__ wdinv,
                                   T* __restrict__ y, int n) {
  int i, j, k;
  node_coords(L, n, i, j, k);
  T un[27][3];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int o = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        T v0 = 0, v1 = 0, v2 = 0;
        if (ii >= 0 && ii < L.nxn && jj >= 0 && jj < L.nyn && kk >= 0 && kk < L.nzn) {
          const int m = n + dx + L.nxn * (dy + L.nyn * dz);
          const int mk = L.mask[m];
          const TU* um = u + 3ll * m;
          v0 = (mk & 1) ? T(0) : T(um[0]);
          v1 = (mk & 2) ? T(0) : T(um[1]);
          v2 = (mk & 4) ? T(0) : T(um[2]);
        }
        un[o][0] = v0;
        un[o][1] = v1;
        un[o][2] = v2;
      }
  T acc0 = 0, acc1 = 0, acc2 = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const int ei = i - ax, ej = j - ay, ek = k - az;
    if (ei < 0 || ei >= L.nx || ej < 0 || ej >= L.ny || ek < 0 || ek >= L.nz) continue;
    const T Ee = E[ei + L.nx * (ej + L.ny * ek)];
    T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
      const int o = (bz - az + 1) * 9 + (by - ay + 1) * 3 + (bx - ax + 1);
      const T* kr = Ke + (3 * a) * 24 + 3 * b;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        s0 += kr[d] * un[o][d];
        s1 += kr[24 + d] * un[o][d];
        s2 += kr[48 + d] * un[o][d];
      }
    }
    acc0 += Ee * s0;
    acc1 += Ee * s1;
    acc2 += Ee * s2;
  }
  const int mk = L.mask[n];
  const long long b = 3ll * n;
  const T Au0 = (mk & 1) ? u[b] : acc0;
  const T Au1 = (mk & 2) ? u[b + 1] : acc1;
  const T Au2 = (mk & 4) ? u[b + 2] : acc2;
  if (MODE == kApply) {
    y[b] = Au0;
    y[b + 1] = Au1;
    y[b + 2] = Au2;
  } else if (MODE == kSmooth) {
    y[b] = u[b] + wdinv[b] * (f[b] - Au0);
    y[b + 1] = u[b + 1] + wdinv[b + 1] * (f[b + 1] - Au1);
    y[b + 2] = u[b + 2] + wdinv[b + 2] * (f[b + 2] - Au2);
  } else {
    y[b] = f[b] - Au0;
    y[b + 1] = f[b + 1] - Au1;
    y[b + 2] = f[b + 2] - Au2;
  }
}

// Coarse right-hand side at coarse node m: f_c = M_c P^T r with trilinear
// weights 1, 1/2 per axis.  With wdc set, also the coarse level's first Jacobi
// sweep from zero, tc = wdc * f_c.  Vectors of one right-hand side.
template <typename T>
__device__ inline void restrict_node(const Level& F, const Level& C, const T* __restrict__ r, T* __restrict__ fc,
                                     const T* __restrict__ wdc, T* __restrict__ tc, int m) {
  int I, J, K;
  node_coords(C, m, I, J, K);
  // all 27 neighbours are requested at once: out-of-range ones read a clamped
  // in-range node with weight 0
  T v[27][3], w[27];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int q = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        const int ii = 2 * I + dx, jj = 2 * J + dy, kk = 2 * K + dz;
        const bool in = ii >= 0 && ii < F.nxn && jj >= 0 && jj < F.nyn && kk >= 0 && kk < F.nzn;
        const int ic = min(max(ii, 0), F.nxn - 1), jc = min(max(jj, 0), F.nyn - 1), kc = min(max(kk, 0), F.nzn - 1);
        const T* rn = r + 3ll * (ic + F.nxn * (jc + F.nyn * kc));
        w[q] = in ? (dx ? T(0.5) : T(1)) * (dy ? T(0.5) : T(1)) * (dz ? T(0.5) : T(1)) : T(0);
        v[q][0] = rn[0];
        v[q][1] = rn[1];
        v[q][2] = rn[2];
      }
  T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    s0 += w[q] * v[q][0];
    s1 += w[q] * v[q][1];
    s2 += w[q] * v[q][2];
  }
  const int mk = C.mask[m];
  const T f0 = (mk & 1) ? T(0) : s0, f1 = (mk & 2) ? T(0) : s1, f2 = (mk & 4) ? T(0) : s2;
  fc[3ll * m] = f0;
  fc[3ll * m + 1] = f1;
  fc[3ll * m + 2] = f2;
  if (wdc) {
    tc[3ll * m] = wdc[3ll * m] * f0;
    tc[3ll * m + 1] = wdc[3ll * m + 1] * f1;
    tc[3ll * m + 2] = wdc[3ll * m + 2] * f2;
  }
}

// Fine correction at fine node n: u += M P e_c (trilinear interpolation),
// formed axis by axis: along x the mean of the two coarse neighbours (the same
// node twice where i is even), then halfway between coarse rows where j is
// odd and between coarse planes where k is odd (the row kernel k_prolong_add
// takes the same steps, so both round alike).
template <typename T>
__device__ inline void prolong_node(const Level& F, const Level& C, const T* __restrict__ ec, T* __restrict__ u,
                                    int n) {
  int i, j, k;
  node_coords(F, n, i, j, k);
  const int I0 = i >> 1, I1 = (i + 1) >> 1, J = j >> 1, K = k >> 1;
  auto xrow = [&](int Jc, int Kc, T (&v)[3]) {
    const T* a = ec + 3ll * (I0 + C.nxn * (Jc + C.nyn * Kc));
    const T* b = ec + 3ll * (I1 + C.nxn * (Jc + C.nyn * Kc));
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = T(0.5) * (a[c] + b[c]);
  };
  T s[3];
  xrow(J, K, s);
  if (j & 1) {
    T t[3];
    xrow(J + 1, K, t);
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = T(0.5) * (s[c] + t[c]);
  }
  if (k & 1) {
    T t[3];
    xrow(J, K + 1, t);
    if (j & 1) {
      T t2[3];
      xrow(J + 1, K + 1, t2);
#pragma unroll
      for (int c = 0; c < 3; ++c) t[c] = T(0.5) * (t[c] + t2[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = T(0.5) * (s[c] + t[c]);
  }
  const int mk = F.mask[n];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (!((mk >> c) & 1)) u[3ll * n + c] += s[c];
}

__device__ inline double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Row `row` of y = Ainv x by one wave (the coarsest solve); binary64 sum.
template <typename T>
__device__ inline void gemv_row(int n, const double* __restrict__ Ainv, const T* __restrict__ x, T* __restrict__ y,
                                int row, int lane) {
  double s = 0.0;
#pragma unroll 8
  for (int c = lane; c < n; c += 64) s += Ainv[(long long)row * n + c] * (double)x[c];
  s = wave_sum64(s);
  if (lane == 0) y[row] = (T)s;
}

}  // namespace hexmg
