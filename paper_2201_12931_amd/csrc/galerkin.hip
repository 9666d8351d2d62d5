// Galerkin coarse operators (Eq. 23): A_{l+1} = P~^T A_l P~ + (I - M_{l+1}),
// P~ = M_l P M_{l+1}, as an alternative to the re-discretized coarse levels.
//
// A Galerkin level is stored as its 27-point block stencil: for node n and
// neighbour offset o = (dz+1)*9 + (dy+1)*3 + (dx+1), the 3x3 block
// A(3n+ci, 3(n+o)+cj) at S[(9*o + 3*ci + cj) * nn + n] (coefficient-major, so
// a wave reading one coefficient of 64 consecutive nodes is coalesced).  The
// stencil already holds the supports: zero rows and columns at fixed DOFs and
// a unit diagonal there, so applying it needs no masking.
//
// Level 1 is built from the matrix-free level 0.  Every fine element lies in
// one coarse element and is one of its eight children c, so
//   P~^T (M K M) P~ = sum over coarse elements of sum_c E_c G_c,
// G_c = P_c^T K0 P_c (24x24, constant, computed on the host), except where a
// child touches a fixed fine DOF: there the masked product is formed on the
// fly.  Deeper levels take the triple product of the stencils.
//
// Storage of the binary32 V-cycle's stencils: binary32, or 16 bits per
// coefficient (half the bytes of the HBM-bound stencil sweep).  bfloat16 keeps
// binary32's exponent range; binary16 keeps 3 more significand bits but not the
// range (the coefficients span Emin..E0 times 2^l), so each node's 243
// coefficients are stored scaled by a power of two that brings the row's
// largest magnitude into [2^14, 2^15), and the sweep applies 2^-s to the row
// sums.  Both are rounded to nearest from the binary64 stencil (bfloat16
// through binary32).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "hexmg_impl.h"
#include "node_ops.h"

namespace hexmg {

namespace {

__device__ inline int off_dx(int o) { return o % 3 - 1; }
__device__ inline int off_dy(int o) { return (o / 3) % 3 - 1; }
__device__ inline int off_dz(int o) { return o / 9 - 1; }

// 1-D trilinear weight of coarse corner a (0/1) at fine offset t (0..2) inside a coarse element
__device__ inline double wt(int t, int a) {
  return a == 0 ? (t == 0 ? 1.0 : (t == 1 ? 0.5 : 0.0)) : (t == 2 ? 1.0 : (t == 1 ? 0.5 : 0.0));
}

// Writes the 3x3 block (m, m + o) with the coarse supports applied.
__device__ inline void store_block(const Level& C, int m, int m2, int o, const double (&blk)[9], double* S64,
                                   float* S32) {
  const int mk = C.mask[m], mk2 = m2 >= 0 ? C.mask[m2] : 7;
#pragma unroll
  for (int ci = 0; ci < 3; ++ci)
#pragma unroll
    for (int cj = 0; cj < 3; ++cj) {
      double v = (((mk >> ci) & 1) || ((mk2 >> cj) & 1)) ? 0.0 : blk[3 * ci + cj];
      if (o == 13 && ci == cj && ((mk >> ci) & 1)) v = 1.0;
      const long long idx = (long long)(9 * o + 3 * ci + cj) * C.nn + m;
      S64[idx] = v;
      if (S32) S32[idx] = (float)v;  // absent when the binary32 V-cycle reads 16-bit coefficients
    }
}

// grid (ceil(C.nn / kBlock), 27): block (m, m + o) of the level-1 operator.
__global__ void k_galerkin_first(Level F, Level C, const double* __restrict__ E, const double* __restrict__ G,
                                 const double* __restrict__ Ke, double* __restrict__ S64, float* __restrict__ S32) {
  const int m = blockIdx.x * kBlock + threadIdx.x, o = blockIdx.y;
  if (m >= C.nn) return;
  int I, J, K;
  node_coords(C, m, I, J, K);
  const int I2 = I + off_dx(o), J2 = J + off_dy(o), K2 = K + off_dz(o);
  double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const bool in = I2 >= 0 && I2 < C.nxn && J2 >= 0 && J2 < C.nyn && K2 >= 0 && K2 < C.nzn;
  const int m2 = in ? I2 + C.nxn * (J2 + C.nyn * K2) : -1;
  if (in) {
    // coarse elements holding both nodes
    for (int EK = (K < K2 ? K : K2) - (K == K2 ? 1 : 0); EK <= (K < K2 ? K : K2); ++EK) {
      if (EK < 0 || EK >= C.nz) continue;
      for (int EJ = (J < J2 ? J : J2) - (J == J2 ? 1 : 0); EJ <= (J < J2 ? J : J2); ++EJ) {
        if (EJ < 0 || EJ >= C.ny) continue;
        for (int EI = (I < I2 ? I : I2) - (I == I2 ? 1 : 0); EI <= (I < I2 ? I : I2); ++EI) {
          if (EI < 0 || EI >= C.nx) continue;
          const int ax = I - EI, ay = J - EJ, az = K - EK;  // corner of m in the coarse element
          const int bx = I2 - EI, by = J2 - EJ, bz = K2 - EK;
          const int a = ax + 2 * ay + 4 * az, b = bx + 2 * by + 4 * bz;
          for (int c = 0; c < 8; ++c) {
            const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
            const int fi = 2 * EI + cx, fj = 2 * EJ + cy, fk = 2 * EK + cz;  // fine element
            const double Ee = E[fi + F.nx * (fj + F.ny * fk)];
            int fixed = 0;
            for (int p = 0; p < 8; ++p)
              fixed |= F.mask[(fi + (p & 1)) + F.nxn * ((fj + ((p >> 1) & 1)) + F.nyn * (fk + (p >> 2)))];
            if (!fixed) {
              const double* Gc = G + c * 576 + (3 * a) * 24 + 3 * b;
#pragma unroll
              for (int ci = 0; ci < 3; ++ci)
#pragma unroll
                for (int cj = 0; cj < 3; ++cj) blk[3 * ci + cj] += Ee * Gc[ci * 24 + cj];
            } else {  // masked child: P_c^T (M K0 M) P_c restricted to corners a, b
              for (int p = 0; p < 8; ++p) {
                const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
                const double wa = wt(cx + px, ax) * wt(cy + py, ay) * wt(cz + pz, az);
                if (wa == 0.0) continue;
                const int mp = F.mask[(fi + px) + F.nxn * ((fj + py) + F.nyn * (fk + pz))];
                for (int q = 0; q < 8; ++q) {
                  const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
                  const double wb = wt(cx + qx, bx) * wt(cy + qy, by) * wt(cz + qz, bz);
                  if (wb == 0.0) continue;
                  const int mq = F.mask[(fi + qx) + F.nxn * ((fj + qy) + F.nyn * (fk + qz))];
                  for (int ci = 0; ci < 3; ++ci) {
                    if ((mp >> ci) & 1) continue;
                    for (int cj = 0; cj < 3; ++cj) {
                      if ((mq >> cj) & 1) continue;
                      blk[3 * ci + cj] += Ee * wa * wb * Ke[(3 * p + ci) * 24 + 3 * q + cj];
                    }
                  }
                }
              }
            }
          }
        }
      }
    }
  }
  store_block(C, m, m2, o, blk, S64, S32);
}

// grid (ceil(C.nn / kBlock), 27): block (m, m + o) of P~^T A_f P~ from the
// fine stencil.  Fine node i runs over the support of coarse node m (weight
// 1 or 1/2 per axis), j = i + o' over i's stencil, restricted to the support
// of m + o.
__global__ void k_galerkin_coarsen(Level F, Level C, const double* __restrict__ Sf, double* __restrict__ S64,
                                   float* __restrict__ S32) {
  const int m = blockIdx.x * kBlock + threadIdx.x, o = blockIdx.y;
  if (m >= C.nn) return;
  int I, J, K;
  node_coords(C, m, I, J, K);
  const int I2 = I + off_dx(o), J2 = J + off_dy(o), K2 = K + off_dz(o);
  double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const bool in = I2 >= 0 && I2 < C.nxn && J2 >= 0 && J2 < C.nyn && K2 >= 0 && K2 < C.nzn;
  const int m2 = in ? I2 + C.nxn * (J2 + C.nyn * K2) : -1;
  if (in) {
    for (int iz = -1; iz <= 1; ++iz) {
      const int fk = 2 * K + iz;
      if (fk < 0 || fk >= F.nzn) continue;
      for (int iy = -1; iy <= 1; ++iy) {
        const int fj = 2 * J + iy;
        if (fj < 0 || fj >= F.nyn) continue;
        for (int ix = -1; ix <= 1; ++ix) {
          const int fi = 2 * I + ix;
          if (fi < 0 || fi >= F.nxn) continue;
          const double wi = (ix ? 0.5 : 1.0) * (iy ? 0.5 : 1.0) * (iz ? 0.5 : 1.0);
          const int i = fi + F.nxn * (fj + F.nyn * fk);
          const int mi = F.mask[i];
          for (int o2 = 0; o2 < 27; ++o2) {
            const int gi = fi + off_dx(o2), gj = fj + off_dy(o2), gk = fk + off_dz(o2);
            const int ex = gi - 2 * I2, ey = gj - 2 * J2, ez = gk - 2 * K2;
            if (ex < -1 || ex > 1 || ey < -1 || ey > 1 || ez < -1 || ez > 1) continue;
            if (gi < 0 || gi >= F.nxn || gj < 0 || gj >= F.nyn || gk < 0 || gk >= F.nzn) continue;
            const double wj = (ex ? 0.5 : 1.0) * (ey ? 0.5 : 1.0) * (ez ? 0.5 : 1.0);
            const int j = gi + F.nxn * (gj + F.nyn * gk);
            const int mj = F.mask[j];
            const double w = wi * wj;
#pragma unroll
            for (int ci = 0; ci < 3; ++ci) {
              if ((mi >> ci) & 1) continue;
#pragma unroll
              for (int cj = 0; cj < 3; ++cj) {
                if ((mj >> cj) & 1) continue;
                blk[3 * ci + cj] += w * Sf[(long long)(9 * o2 + 3 * ci + cj) * F.nn + i];
              }
            }
          }
        }
      }
    }
  }
  store_block(C, m, m2, o, blk, S64, S32);
}

// One node's 243 binary64 coefficients to 16 bits: bfloat16 (STORE ==
// HEXMG_STENCIL_BF16) or binary16 scaled by 2^s[n] (HEXMG_STENCIL_F16).
template <int STORE>
__global__ void k_stencil_to16(Level L, const double* __restrict__ S64, uint16_t* __restrict__ S16,
                               int8_t* __restrict__ sexp) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= L.nn) return;
  if (STORE == HEXMG_STENCIL_BF16) {
    for (int q = 0; q < 243; ++q) {
      const long long idx = (long long)q * L.nn + n;
      S16[idx] = __bfloat16_as_ushort(__float2bfloat16((float)S64[idx]));
    }
    return;
  }
  double amax = 0.0;
  for (int q = 0; q < 243; ++q) amax = fmax(amax, fabs(S64[(long long)q * L.nn + n]));
  int e = 0;
  if (amax > 0.0) (void)frexp(amax, &e);  // amax in [2^(e-1), 2^e)
  const int sc = min(max(15 - e, -126), 126);  // amax * 2^sc in [2^14, 2^15)
  sexp[n] = (int8_t)max(min(sc, 127), -127);
  for (int q = 0; q < 243; ++q) {
    const long long idx = (long long)q * L.nn + n;
    const _Float16 h = (_Float16)ldexp(S64[idx], sexp[n]);
    S16[idx] = __builtin_bit_cast(uint16_t, h);
  }
}

__device__ inline float stencil_coef(const float* S, long long i) { return S[i]; }
__device__ inline double stencil_coef(const double* S, long long i) { return S[i]; }

// 16-bit coefficients (bfloat16 or binary16, by storage type tag)
struct Bf16Tag {};
struct F16Tag {};
template <typename Tag>
struct Stored16 {
  const uint16_t* p;
};
__device__ inline float stencil_coef(Stored16<Bf16Tag> S, long long i) {
  return __uint_as_float((unsigned)S.p[i] << 16);
}
__device__ inline float stencil_coef(Stored16<F16Tag> S, long long i) {
  return __half2float(__ushort_as_half(S.p[i]));
}

// y = A u from the stencil (MODE as the element kernels: 0 A u, 1 Jacobi
// sweep, 2 residual); grid (ceil(nn / kBlock), nrhs).  SP: the coefficient
// array (T*, or Stored16<tag> for the 16-bit storages); sexp: the binary16
// rows' scale exponents (null otherwise).
template <typename T, typename SP, int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil(Level L, SP S, const int8_t* __restrict__ sexp,
                                                    const T* __restrict__ u, const T* __restrict__ f,
                                                    const T* __restrict__ wdinv, T* __restrict__ y,
                                                    const int* __restrict__ act) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= L.nn || (act && !act[blockIdx.y])) return;
  const long long off = 3ll * L.nn * blockIdx.y;
  u += off;
  y += off;
  if (MODE != kApply) f += off;
  int i, j, k;
  node_coords(L, n, i, j, k);
  T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
    const int ii = i + dx, jj = j + dy, kk = k + dz;
    if (ii < 0 || ii >= L.nxn || jj < 0 || jj >= L.nyn || kk < 0 || kk >= L.nzn) continue;
    const T* un = u + 3ll * (n + dx + L.nxn * (dy + L.nyn * dz));
    const T v0 = un[0], v1 = un[1], v2 = un[2];
    const long long s0 = (long long)(9 * o) * L.nn + n;
    const long long st = L.nn;
    a0 += stencil_coef(S, s0) * v0 + stencil_coef(S, s0 + st) * v1 + stencil_coef(S, s0 + 2 * st) * v2;
    a1 += stencil_coef(S, s0 + 3 * st) * v0 + stencil_coef(S, s0 + 4 * st) * v1 + stencil_coef(S, s0 + 5 * st) * v2;
    a2 += stencil_coef(S, s0 + 6 * st) * v0 + stencil_coef(S, s0 + 7 * st) * v1 + stencil_coef(S, s0 + 8 * st) * v2;
  }
  if (sexp) {  // binary16 rows were stored scaled by 2^s
    const int e = -sexp[n];
    a0 = ldexp(a0, e);
    a1 = ldexp(a1, e);
    a2 = ldexp(a2, e);
  }
  const long long b = 3ll * n;
  if (MODE == kApply) {
    y[b] = a0;
    y[b + 1] = a1;
    y[b + 2] = a2;
  } else if (MODE == kSmooth) {
    y[b] = u[b] + wdinv[b] * (f[b] - a0);
    y[b + 1] = u[b + 1] + wdinv[b + 1] * (f[b + 1] - a1);
    y[b + 2] = u[b + 2] + wdinv[b + 2] * (f[b + 2] - a2);
  } else {
    y[b] = f[b] - a0;
    y[b + 1] = f[b + 1] - a1;
    y[b + 2] = f[b + 2] - a2;
  }
}

__global__ void k_stencil_diag(Level L, const double* __restrict__ S, double omega, double* __restrict__ wd64,
                               float* __restrict__ wd32) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= L.nn) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double w = omega / S[(long long)(9 * 13 + 4 * c) * L.nn + n];
    if (wd64) wd64[3ll * n + c] = w;  // either output may be absent
    if (wd32) wd32[3ll * n + c] = (float)w;
  }
}

// grid (ceil(N / kBlock), N): dense operator entry (r, c) from the stencil
__global__ void k_dense_from_stencil(Level C, const double* __restrict__ S, double* __restrict__ A) {
  const int N = 3 * C.nn;
  const int c = blockIdx.x * kBlock + threadIdx.x, r = blockIdx.y;
  if (c >= N) return;
  const int m = r / 3, ci = r % 3, m2 = c / 3, cj = c % 3;
  int I, J, K, I2, J2, K2;
  node_coords(C, m, I, J, K);
  node_coords(C, m2, I2, J2, K2);
  const int dx = I2 - I, dy = J2 - J, dz = K2 - K;
  double v = 0.0;
  if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) {
    const int o = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
    v = S[(long long)(9 * o + 3 * ci + cj) * C.nn + m];
  }
  A[(long long)r * N + c] = v;
}

inline int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

void launch_galerkin_first(const Level& F, const Level& C, const double* E, const double* G, const double* Ke,
                           double* S64, float* S32, hipStream_t s) {
  k_galerkin_first<<<dim3(blocks_for(C.nn), 27), kBlock, 0, s>>>(F, C, E, G, Ke, S64, S32);
}

void launch_galerkin_coarsen(const Level& F, const Level& C, const double* Sf, double* S64, float* S32,
                             hipStream_t s) {
  k_galerkin_coarsen<<<dim3(blocks_for(C.nn), 27), kBlock, 0, s>>>(F, C, Sf, S64, S32);
}

namespace {
template <typename T, typename SP>
void launch_stencil_sp(int mode, const Level& L, SP S, const int8_t* sexp, const T* u, const T* f, const T* wd,
                       T* y, int nrhs, const int* act, hipStream_t s, const LaunchTimer& t) {
  const dim3 g(blocks_for(L.nn), nrhs);
  if (mode == kApply)
    launch_timed(k_stencil<T, SP, kApply>, g, dim3(kBlock), s, t, L, S, sexp, u, f, wd, y, act);
  else if (mode == kSmooth)
    launch_timed(k_stencil<T, SP, kSmooth>, g, dim3(kBlock), s, t, L, S, sexp, u, f, wd, y, act);
  else
    launch_timed(k_stencil<T, SP, kResidual>, g, dim3(kBlock), s, t, L, S, sexp, u, f, wd, y, act);
}
}  // namespace

template <typename T>
void launch_stencil(int mode, const Level& L, const T* S, const T* u, const T* f, const T* wd, T* y, int nrhs,
                    const int* act, hipStream_t s, const LaunchTimer& t) {
  launch_stencil_sp<T, const T*>(mode, L, S, nullptr, u, f, wd, y, nrhs, act, s, t);
}

void launch_stencil16(int store, int mode, const Level& L, const uint16_t* S16, const int8_t* sexp, const float* u,
                      const float* f, const float* wd, float* y, int nrhs, const int* act, hipStream_t s,
                      const LaunchTimer& t) {
  if (store == HEXMG_STENCIL_BF16)
    launch_stencil_sp<float, Stored16<Bf16Tag>>(mode, L, Stored16<Bf16Tag>{S16}, nullptr, u, f, wd, y, nrhs, act,
                                                 s, t);
  else
    launch_stencil_sp<float, Stored16<F16Tag>>(mode, L, Stored16<F16Tag>{S16}, sexp, u, f, wd, y, nrhs, act, s, t);
}

void launch_stencil_to16(int store, const Level& L, const double* S64, uint16_t* S16, int8_t* sexp,
                         hipStream_t s) {
  if (store == HEXMG_STENCIL_BF16)
    k_stencil_to16<HEXMG_STENCIL_BF16><<<blocks_for(L.nn), kBlock, 0, s>>>(L, S64, S16, sexp);
  else
    k_stencil_to16<HEXMG_STENCIL_F16><<<blocks_for(L.nn), kBlock, 0, s>>>(L, S64, S16, sexp);
}
template void launch_stencil<double>(int, const Level&, const double*, const double*, const double*, const double*,
                                     double*, int, const int*, hipStream_t, const LaunchTimer&);
template void launch_stencil<float>(int, const Level&, const float*, const float*, const float*, const float*,
                                    float*, int, const int*, hipStream_t, const LaunchTimer&);

void launch_stencil_diag(const Level& L, const double* S, double omega, double* wd64, float* wd32, hipStream_t s) {
  k_stencil_diag<<<blocks_for(L.nn), kBlock, 0, s>>>(L, S, omega, wd64, wd32);
}

void launch_dense_from_stencil(const Level& C, const double* S, double* A, hipStream_t s) {
  const int N = 3 * C.nn;
  k_dense_from_stencil<<<dim3(blocks_for(N), N), kBlock, 0, s>>>(C, S, A);
}

// G_c = P_c^T K0 P_c for the eight children c of a coarse element (host):
// G[c][(3a+ci)*24 + 3b+cj], a, b the coarse corners.
void galerkin_child_matrices(const double* Ke, double* G) {
  auto w1 = [](int t, int a) { return a == 0 ? (t == 0 ? 1.0 : (t == 1 ? 0.5 : 0.0)) : (t == 2 ? 1.0 : (t == 1 ? 0.5 : 0.0)); };
  for (int c = 0; c < 8; ++c) {
    const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
    double P[8][8];  // P[p][a]: weight of coarse corner a at fine corner p of child c
    for (int p = 0; p < 8; ++p)
      for (int a = 0; a < 8; ++a)
        P[p][a] = w1(cx + (p & 1), a & 1) * w1(cy + ((p >> 1) & 1), (a >> 1) & 1) * w1(cz + (p >> 2), a >> 2);
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        for (int ci = 0; ci < 3; ++ci)
          for (int cj = 0; cj < 3; ++cj) {
            double s = 0.0;
            for (int p = 0; p < 8; ++p) {
              if (P[p][a] == 0.0) continue;
              for (int q = 0; q < 8; ++q) s += P[p][a] * P[q][b] * Ke[(3 * p + ci) * 24 + 3 * q + cj];
            }
            G[c * 576 + (3 * a + ci) * 24 + 3 * b + cj] = s;
          }
  }
}

}  // namespace hexmg
