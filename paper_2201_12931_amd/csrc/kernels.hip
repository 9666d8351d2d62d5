// HIP kernels of the hexmg hot path for gfx950 (wave64).
//
// Layout: node-major vectors (DOF 3n + c); element moduli per element; support
// bits per node.  Every reduction is a fixed-shape two-stage tree (kReduceBlocks
// partial sums, then one block in a fixed order) so results are reproducible
// run to run; no floating-point atomics are used anywhere.
#include <algorithm>

#include "hexmg_impl.h"
#include "node_ops.h"

namespace hexmg {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over a block of kBlock threads; the result is valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double part[kBlock / 64];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s += part[i];
  }
  return s;
}

// Sum over a block of kBlock threads, returned to every thread (fixed order).
__device__ inline double block_sum_all(double v) {
  __shared__ double part[kBlock / 64];
  __shared__ double total;
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) part[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s += part[i];
    total = s;
  }
  __syncthreads();
  return total;
}

// sum of the kReduceBlocks partials of one right-hand side, in every thread
__device__ inline double sum_partials(const double* __restrict__ partials) {
  double s = 0.0;
  for (int i = threadIdx.x; i < kReduceBlocks; i += kBlock) s += partials[i];
  return block_sum_all(s);
}

inline int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

// rho^p of the SIMP law (Eq. 2): the paper's p = 3 (and p = 1) by products,
// other exponents by pow
__device__ inline double simp_pow(double r, double p) {
  if (p == 3.0) return r * r * r;
  if (p == 1.0) return r;
  return pow(r, p);
}

// ---------------------------------------------------------------------------
// Matrix-free K u (Sec. 4.2.1), node-gather form: one thread per node (see
// gather_node).
template <typename T, int MODE, typename TU = T>
__global__ __launch_bounds__(kBlock) void k_gather(Level L, const T* __restrict__ Ke,
                                                   const T* __restrict__ E, const TU* __restrict__ u,
                                                   const T* __restrict__ f,
                                                   const T* __restrict__ wdinv, T* __restrict__ y,
                                                   const int* __restrict__ act) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= L.nn || (act && !act[blockIdx.y])) return;
  const long long off = 3ll * L.nn * blockIdx.y;  // right-hand side blockIdx.y: vectors are [nrhs][3 nn]
  gather_node<T, MODE, TU>(L, Ke, E, u + off, MODE != kApply ? f + off : f, wdinv, y + off, n);
}

// First sweep from a zero guess: u = omega D^{-1} f.
template <typename T>
__global__ void k_jacobi_first(long long n, const T* __restrict__ wdinv, const T* __restrict__ f,
                               T* __restrict__ u, const int* __restrict__ act) {
  if (act && !act[blockIdx.y]) return;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long off = n * blockIdx.y;  // right-hand side
  if (i < n) u[off + i] = wdinv[i] * f[off + i];
}

__global__ void k_jacobi_first_from64(long long n, const float* __restrict__ wdinv, const double* __restrict__ r,
                                      float* __restrict__ f32, float* __restrict__ u, const int* __restrict__ act) {
  if (act && !act[blockIdx.y]) return;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long off = n * blockIdx.y;
  if (i < n) {
    const float fv = (float)r[off + i];
    f32[off + i] = fv;
    u[off + i] = wdinv[i] * fv;
  }
}

// The launch's blocks (x dimension) in slabs of `slab` consecutive blocks,
// each slab in XCD bands (xcd_band_index): with a slab of about one plane of
// the grid, the blocks that read the same rows of the other level run on one
// L2, and the next slab's band (the next plane) re-reads rows the same L2 has
// just held.
__device__ inline int xcd_band_block(int slab) {
  const int n = (int)gridDim.x, b = (int)blockIdx.x;
  const int s0 = b - b % slab;
  return s0 + xcd_band_index(b - s0, min(slab, n - s0), (long long)n * blockIdx.y + s0);
}
// A slab of about one plane of `per_plane` blocks, a multiple of 8.
inline int band_slab(long long per_plane) { return (int)std::max<long long>(8, (per_plane + 7) / 8 * 8); }

// Coarse right-hand side f_c = M_c P^T r (see restrict_node); with wdc set,
// also the coarse level's first Jacobi sweep from zero, tc = wdc * f_c.
// (bx, rhs): the workgroup's place in a launch of (ceil(C.nn / kBlock), nrhs).
template <typename T>
__device__ __forceinline__ void restrict_block(const Level& F, const Level& C, const T* __restrict__ r,
                                               T* __restrict__ fc, const int* __restrict__ act,
                                               const T* __restrict__ wdc, T* __restrict__ tc, int bx, int rhs) {
  const int m = bx * kBlock + threadIdx.x;
  if (m >= C.nn || (act && !act[rhs])) return;
  restrict_node<T>(F, C, r + 3ll * F.nn * rhs, fc + 3ll * C.nn * rhs, wdc, wdc ? tc + 3ll * C.nn * rhs : tc, m);
}
template <typename T>
__global__ void k_restrict(Level F, Level C, const T* __restrict__ r, T* __restrict__ fc,
                           const int* __restrict__ act, const T* __restrict__ wdc, T* __restrict__ tc, int slab) {
  restrict_block<T>(F, C, r, fc, act, wdc, tc, xcd_band_block(slab), blockIdx.y);
}
template <typename T>
__global__ void k_restrict_batch(Batch<RestrictTask<T>> tb) {
  const int t = batch_task(tb.begin, tb.n, (int)blockIdx.x);
  const RestrictTask<T>& a = tb.a[t];
  const int local = (int)blockIdx.x - tb.begin[t];
  restrict_block<T>(a.F, a.C, a.r, a.fc, a.act, a.wdc, a.tc, local % a.gx, local / a.gx);
}

// Fine correction u += M P e_c by rows: each wave takes 64 consecutive nodes of
// the four fine node rows (2J + dj, 2K + dk), dj, dk in {0, 1}, so which
// coarse rows contribute to which row, with which weights, is uniform over the
// wave, and along x a node takes the mean of its two coarse neighbours (the
// same node twice where i is even).  The four x-interpolated coarse rows
// (J + dj, K + dk) serve all four fine rows: the even rows take them as they
// are, the odd ones the means (in the order of the per-node form, so both
// forms agree bit for bit).  A block covers 64 columns of 4 row quads: bx =
// column block + cols * quad block, cols = ceil(nxn / 64).  u and the support
// bits are requested before the coarse values, and every component is written
// back (the fixed ones unchanged), so no load waits behind a branch.
template <typename T>
__device__ __forceinline__ void prolong_block(const Level& F, const Level& C, const T* __restrict__ ec,
                                              T* __restrict__ u, const int* __restrict__ act, int bx, int rhs) {
  if (act && !act[rhs]) return;
  const int cols = (F.nxn + 63) >> 6;
  const int nyq = (F.nyn + 1) >> 1, nzq = (F.nzn + 1) >> 1;
  const int quad = __builtin_amdgcn_readfirstlane((bx / cols) * 4 + (int)(threadIdx.x >> 6));  // J + nyq K
  const int i = (bx % cols) * 64 + (int)(threadIdx.x & 63);
  if (quad >= nyq * nzq || i >= F.nxn) return;
  const int J = quad % nyq, K = quad / nyq;
  const bool jo = 2 * J + 1 < F.nyn, ko = 2 * K + 1 < F.nzn;  // uniform: the odd rows exist
  const T* e = ec + 3ll * C.nn * rhs;
  u += 3ll * F.nn * rhs;
  const long long row = F.nxn, pl = (long long)F.nxn * F.nyn;
  const long long n00 = i + row * (2 * J) + pl * (2 * K);
  long long nn[4] = {n00, n00 + row, n00 + pl, n00 + row + pl};  // (dj, dk) = (0,0) (1,0) (0,1) (1,1)
  const bool has[4] = {true, jo, ko, jo && ko};
  int m[4];
  T uv[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    m[q] = has[q] ? (int)F.mask[nn[q]] : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) uv[q][c] = has[q] ? u[3 * nn[q] + c] : T(0);
  }
  const int I0 = i >> 1, I1 = (i + 1) >> 1;
  // x-interpolated coarse row (Jc, Kc) at this node
  auto xrow = [&](int Jc, int Kc, T (&v)[3]) {
    const T* a = e + 3ll * (I0 + C.nxn * (Jc + C.nyn * Kc));
    const T* b = e + 3ll * (I1 + C.nxn * (Jc + C.nyn * Kc));
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = T(0.5) * (a[c] + b[c]);
  };
  auto put = [&](int q, const T (&s)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) u[3 * nn[q] + c] = ((m[q] >> c) & 1) ? uv[q][c] : uv[q][c] + s[c];
  };
  T a[3], b[3], cz[3], d[3], s[3];
  xrow(J, K, a);
  put(0, a);
  if (jo) {
    xrow(J + 1, K, b);
#pragma unroll
    for (int c = 0; c < 3; ++c) b[c] = T(0.5) * (a[c] + b[c]);  // the mean over coarse rows J, J + 1
    put(1, b);
  }
  if (ko) {
    xrow(J, K + 1, cz);
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = T(0.5) * (a[c] + cz[c]);
    put(2, s);
    if (jo) {
      xrow(J + 1, K + 1, d);
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c] = T(0.5) * (b[c] + T(0.5) * (cz[c] + d[c]));
      put(3, s);
    }
  }
}
template <typename T>
__global__ void k_prolong_add(Level F, Level C, const T* __restrict__ ec, T* __restrict__ u,
                              const int* __restrict__ act, int slab) {
  prolong_block<T>(F, C, ec, u, act, xcd_band_block(slab), blockIdx.y);
}
template <typename T>
__global__ void k_prolong_add_batch(Batch<ProlongTask<T>> tb) {
  const int t = batch_task(tb.begin, tb.n, (int)blockIdx.x);
  const ProlongTask<T>& a = tb.a[t];
  const int local = (int)blockIdx.x - tb.begin[t];
  prolong_block<T>(a.F, a.C, a.ec, a.u, a.act, local % a.gx, local / a.gx);
}

// ---------------------------------------------------------------------------
// Set-up: SIMP moduli (Eq. 2), homogenized coarse densities (Sec. 4.2.2),
// Jacobi diagonal, supports.
__global__ void k_simp(int ne, const double* __restrict__ rho, double E0, double Emin, double p,
                       double scale, double* __restrict__ E64, float* __restrict__ E32,
                       double* __restrict__ rho_copy, int* __restrict__ flags) {
  int bad = 0;
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < ne; e += gridDim.x * kBlock) {
    const double r = rho[e];
    if (!(r >= 0.0 && r <= 1.0)) bad = 1;  // also catches NaN
    rho_copy[e] = r;
    const double E = scale * (Emin + simp_pow(r, p) * (E0 - Emin));
    E64[e] = E;
    E32[e] = (float)E;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flags[blockIdx.x] = bad;
}

__global__ void k_or_flags(int n, const int* __restrict__ flags, int* __restrict__ out) {
  int v = 0;
  for (int i = threadIdx.x; i < n; i += kBlock) v |= flags[i];
  v = __syncthreads_or(v);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ void k_homogenize(Level F, Level C, const double* __restrict__ vf, double* __restrict__ vc) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= C.ne) return;
  const int I = e % C.nx, t = e / C.nx, J = t % C.ny, K = t / C.ny;
  double s = 0.0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) s += vf[(2 * I + dx) + F.nx * ((2 * J + dy) + F.ny * (2 * K + dz))];
  vc[e] = 0.125 * s;
}

__global__ void k_modulus_from_density(int ne, const double* __restrict__ rho, double E0, double Emin,
                                       double p, double scale, double* __restrict__ E64,
                                       float* __restrict__ E32) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= ne) return;
  const double E = scale * (Emin + simp_pow(rho[e], p) * (E0 - Emin));
  E64[e] = E;
  E32[e] = (float)E;
}

// Moduli of the coarsest level straight from level 0, one block per coarsest
// element: the mean of the blk^3 fine densities (density averaging) or fine
// moduli (modulus averaging) of its block -- the nested means of the level
// hierarchy, summed in one pass -- then the SIMP modulus of the mean density
// times scale, or scale times the mean modulus.  Feeds only the coarsest
// operator, so that its assembly does not wait for the other levels.
__global__ void k_coarsest_moduli(Level F, Level C, int blk, const double* __restrict__ v0, int density,
                                  double E0, double Emin, double p, double scale, double* __restrict__ Ec) {
  const int e = blockIdx.x;
  const int I = e % C.nx, t = e / C.nx, J = t % C.ny, K = t / C.ny;
  const int nb = blk * blk * blk;
  double s = 0.0;
#pragma unroll 8
  for (int q = threadIdx.x; q < nb; q += kBlock) {
    const int dx = q % blk, r = q / blk, dy = r % blk, dz = r / blk;
    s += v0[(I * blk + dx) + (long long)F.nx * ((J * blk + dy) + (long long)F.ny * (K * blk + dz))];
  }
  s = block_sum(s);
  if (threadIdx.x == 0) {
    const double m = s / nb;
    Ec[e] = density ? scale * (Emin + simp_pow(m, p) * (E0 - Emin)) : scale * m;
  }
}

__global__ void k_modulus_from_mean(Level F, Level C, const double* __restrict__ Ef, double scale,
                                    double* __restrict__ E64, float* __restrict__ E32) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= C.ne) return;
  const int I = e % C.nx, t = e / C.nx, J = t % C.ny, K = t / C.ny;
  double s = 0.0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) s += Ef[(2 * I + dx) + F.nx * ((2 * J + dy) + F.ny * (2 * K + dz))];
  const double E = scale * 0.125 * s;
  E64[e] = E;
  E32[e] = (float)E;
}

__global__ void k_diag(Level L, const double* __restrict__ Ke, const double* __restrict__ E,
                       double omega, double* __restrict__ wd64, float* __restrict__ wd32) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= L.nn) return;
  int i, j, k;
  node_coords(L, n, i, j, k);
  double d0 = 0, d1 = 0, d2 = 0;
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const int ei = i - ax, ej = j - ay, ek = k - az;
    if (ei < 0 || ei >= L.nx || ej < 0 || ej >= L.ny || ek < 0 || ek >= L.nz) continue;
    const double Ee = E[ei + L.nx * (ej + L.ny * ek)];
    d0 += Ee * Ke[(3 * a + 0) * 25];
    d1 += Ee * Ke[(3 * a + 1) * 25];
    d2 += Ee * Ke[(3 * a + 2) * 25];
  }
  const int mk = L.mask[n];
  const double w0 = omega / ((mk & 1) ? 1.0 : d0);
  const double w1 = omega / ((mk & 2) ? 1.0 : d1);
  const double w2 = omega / ((mk & 4) ? 1.0 : d2);
  if (wd64) {  // either output may be absent (the grid holds one precision)
    wd64[3ll * n] = w0;
    wd64[3ll * n + 1] = w1;
    wd64[3ll * n + 2] = w2;
  }
  if (wd32) {
    wd32[3ll * n] = (float)w0;
    wd32[3ll * n + 1] = (float)w1;
    wd32[3ll * n + 2] = (float)w2;
  }
}

__global__ void k_mask_default(Level L, uint8_t* __restrict__ mask) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= L.nn) return;
  mask[n] = (n % L.nxn == 0) ? 7 : 0;
}

__global__ void k_mask_inject(Level F, Level C, const uint8_t* __restrict__ mf, uint8_t* __restrict__ mc) {
  const int m = blockIdx.x * kBlock + threadIdx.x;
  if (m >= C.nn) return;
  int I, J, K;
  node_coords(C, m, I, J, K);
  mc[m] = mf[2 * I + F.nxn * (2 * J + F.nyn * 2 * K)];
}

// ---------------------------------------------------------------------------
// Coarsest level: dense A_c, in-place Gauss-Jordan inverse (SPD, so no pivoting),
// and the direct solve e = A_c^{-1} f as a GEMV (Alg. 3, coarsest grid).
__global__ void k_coarse_assemble(Level C, const double* __restrict__ Ke, const double* __restrict__ E,
                                  double* __restrict__ A) {
  const int N = 3 * C.nn;
  const int c = blockIdx.x * kBlock + threadIdx.x, r = blockIdx.y;
  if (c >= N) return;
  const long long idx = (long long)r * N + c;
  const int m1 = r / 3, c1 = r % 3, m2 = c / 3, c2 = c % 3;
  const bool fixed = ((C.mask[m1] >> c1) & 1) || ((C.mask[m2] >> c2) & 1);
  if (fixed) {
    A[idx] = (r == c) ? 1.0 : 0.0;
    return;
  }
  int i1, j1, k1, i2, j2, k2;
  node_coords(C, m1, i1, j1, k1);
  node_coords(C, m2, i2, j2, k2);
  double s = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const int ei = i1 - ax, ej = j1 - ay, ek = k1 - az;
    if (ei < 0 || ei >= C.nx || ej < 0 || ej >= C.ny || ek < 0 || ek >= C.nz) continue;
    const int bx = i2 - ei, by = j2 - ej, bz = k2 - ek;
    if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
    const int b = bx + 2 * by + 4 * bz;
    s += E[ei + C.nx * (ej + C.ny * ek)] * Ke[(3 * a + c1) * 24 + 3 * b + c2];
  }
  A[idx] = s;
}

// Blocked Gauss-Jordan.  For the pivot block K (rows/columns k0 .. k0+nb-1):
//   D = A_KK^{-1};  X_J = D A_KJ (row panel, with X_K = D);
//   B_K* = X,  B_IK = -A_IK D,  B_IJ = A_IJ - A_IK X_J,
// which is nb scalar Gauss-Jordan steps applied at once.  A is read, B written.
// The SPD coarse matrix (identity rows at fixed DOFs) needs no pivoting.
//
// Gauss-Jordan on a pivot block K of size b (b consecutive scalar steps at
// once): with Q = A_KK^{-1}, every element takes
//   a_ij <- z_ij - sum_h c_ih r_hj   (h = 0..b-1),
// z = a with the rows and columns of K cleared, c_i = (a_i,k+h)_h for i not
// in K and -e_i for i in K, r_j = Q (a_k+h,j)_h for j not in K and the column
// Q e_j for j in K.  That leaves Q on K x K, Q A_Kj on the pivot rows,
// -A_iK Q on the pivot columns and A_ij - A_iK Q A_Kj elsewhere.  The diagonal
// blocks of an SPD matrix and of its Schur complements are SPD, so no
// pivoting is needed.  For b = 4, Q comes from the 2x2 block form (inverse of
// the leading 2x2 block, of its Schur complement, then the off-diagonal
// blocks).
__device__ inline void inv2(double a00, double a01, double a10, double a11, double (&q)[2][2]) {
  // 1/det: hardware reciprocal and two Newton steps (each squares the
  // relative error), shorter than the IEEE division on this latency-bound chain
  const double det = a00 * a11 - a01 * a10;
  double id = __builtin_amdgcn_rcp(det);
  id = fma(id, fma(-det, id, 1.0), id);
  id = fma(id, fma(-det, id, 1.0), id);
  q[0][0] = a11 * id;
  q[0][1] = -a01 * id;
  q[1][0] = -a10 * id;
  q[1][1] = a00 * id;
}

__device__ inline void inv4(const double (&p)[4][4], double (&q)[4][4]) {
  double ai[2][2], x[2][2], y[2][2], sm[2][2], si[2][2];
  inv2(p[0][0], p[0][1], p[1][0], p[1][1], ai);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      x[r][c] = ai[r][0] * p[0][2 + c] + ai[r][1] * p[1][2 + c];  // A^-1 B
      y[r][c] = p[2 + r][0] * ai[0][c] + p[2 + r][1] * ai[1][c];  // C A^-1
    }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) sm[r][c] = p[2 + r][2 + c] - (y[r][0] * p[0][2 + c] + y[r][1] * p[1][2 + c]);
  inv2(sm[0][0], sm[0][1], sm[1][0], sm[1][1], si);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      q[2 + r][2 + c] = si[r][c];
      q[r][2 + c] = -(x[r][0] * si[0][c] + x[r][1] * si[1][c]);
      q[2 + r][c] = -(si[r][0] * y[0][c] + si[r][1] * y[1][c]);
    }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) q[r][c] = ai[r][c] - (q[r][2] * y[0][c] + q[r][3] * y[1][c]);
}

typedef double d4 __attribute__((ext_vector_type(4)));

// In-place inverse of the SPD 64x64 tile in LDS (row-major, padded rows; the
// identity beyond its nb x nb block), by the block's 256 threads; written
// transposed to DT (DT[j*64+i] = M_ij).  Block Gauss-Jordan with 16x16 pivot
// blocks K (four steps, the unified update above with h = 0..15):
//   Q = M_KK^{-1}                     16x16, one element per thread, by four
//                                     steps of 4x4 pivot blocks (inv4);
//   R = Q M_K*, with R_K = Q          on the matrix cores, one 16x16 tile per wave;
//   M <- Z - C R                      on the matrix cores, 16 rows per wave,
// with Z = M with the rows and columns of K cleared and C = M_*K, C_K = -I.
// sR16: 16 rows of exchange space for R; sQ, pr, pc: small exchange buffers.
template <int RR>
__device__ inline void block_inverse(double (&sM)[kGJBlock][kGJBlock + 1], double (&sR16)[RR][kGJBlock + 1],
                                     double (&sQ)[16][17], double (&pr)[2][4][16], double (&pc)[2][4][16],
                                     double* __restrict__ DT) {
  static_assert(RR >= 16 && kGJBlock == 64 && kBlock == 256, "four waves, 16x16 pivot blocks");
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int ti = t >> 4, tj = t & 15;  // element of the 16x16 pivot block
  const int lr = l & 15, lk = l >> 4;  // matrix-core operand row / k of this lane
#pragma unroll 1
  for (int s = 0; s < 4; ++s) {
    const int k0 = 16 * s;
    // Q = M_KK^{-1}: Gauss-Jordan on 4x4 pivot blocks, one element per thread
    double a = sM[k0 + ti][k0 + tj];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int kb = 4 * m, par = m & 1;
      const int hy = ti - kb, hx = tj - kb;
      const bool rowk = hy >= 0 && hy < 4, colk = hx >= 0 && hx < 4;
      if (rowk) pr[par][hy][tj] = a;
      if (colk) pc[par][hx][ti] = a;
      __syncthreads();
      double pk[4][4], q[4][4];
#pragma unroll
      for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int g = 0; g < 4; ++g) pk[h][g] = pr[par][h][kb + g];
      inv4(pk, q);
      double xg[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) xg[g] = pr[par][g][tj];
      double acc = (rowk || colk) ? 0.0 : a;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        // Q e_hx as exact 0/1 weights (a select chain here becomes an indexed stack array)
        const double qh = q[h][0] * (hx == 0 ? 1.0 : 0.0) + q[h][1] * (hx == 1 ? 1.0 : 0.0) +
                          q[h][2] * (hx == 2 ? 1.0 : 0.0) + q[h][3] * (hx == 3 ? 1.0 : 0.0);
        const double r = colk ? qh : q[h][0] * xg[0] + q[h][1] * xg[1] + q[h][2] * xg[2] + q[h][3] * xg[3];
        const double c = rowk ? (hy == h ? -1.0 : 0.0) : pc[par][h][ti];
        acc = fma(-c, r, acc);
      }
      a = acc;
    }
    sQ[ti][tj] = a;
    __syncthreads();
    // R = Q M_K* (tile w), R_K = Q
    if (w == s) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sR16[4 * v + lk][k0 + lr] = sQ[4 * v + lk][lr];
    } else {
      d4 r = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        r = __builtin_amdgcn_mfma_f64_16x16x4f64(sQ[lr][4 * ks + lk], sM[k0 + 4 * ks + lk][16 * w + lr], r, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) sR16[4 * v + lk][16 * w + lr] = r[v];
    }
    __syncthreads();
    // rows 16w..16w+15: M <- Z - C R
    {
      d4 y[4];
      double cneg[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          y[ct][v] = (w == s || ct == s) ? 0.0 : sM[16 * w + 4 * v + lk][16 * ct + lr];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        cneg[ks] = (w == s) ? (lr == 4 * ks + lk ? 1.0 : 0.0) : -sM[16 * w + lr][k0 + 4 * ks + lk];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          y[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(cneg[ks], sR16[4 * ks + lk][16 * ct + lr], y[ct], 0, 0, 0);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) sM[16 * w + 4 * v + lk][16 * ct + lr] = y[ct][v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < kGJBlock * kGJBlock / kBlock; ++e) {
    const int idx = t + kBlock * e, j = idx >> 6, i = idx & 63;
    DT[j * kGJBlock + i] = sM[i][j];
  }
}

// Inverse of the first diagonal block (later ones are formed by the panel
// update that produces them).
__global__ __launch_bounds__(kBlock) void k_gj_block_inv(int n, int k0, int nb, const double* __restrict__ A,
                                                         double* __restrict__ DT) {
  __shared__ double sM[kGJBlock][kGJBlock + 1], sR16[16][kGJBlock + 1], sQ[16][17];
  __shared__ double pr[2][4][16], pc[2][4][16];
#pragma unroll
  for (int e = 0; e < kGJBlock * kGJBlock / kBlock; ++e) {
    const int idx = threadIdx.x + kBlock * e, i = idx >> 6, j = idx & 63;
    sM[i][j] = (i < nb && j < nb) ? A[(long long)(k0 + i) * n + k0 + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  block_inverse(sM, sR16, sQ, pr, pc, DT);
}

// 64x64x64 product on the matrix cores: wave w accumulates rows 16w..16w+15
// of L^T-stored-left times right, acc[t] holding the 16x16 output tile t
// (columns 16t..16t+15).  v_mfma_f64_16x16x4f64 lane layout: the left operand
// of lane l is element (row l%16, k l/16), the right one (k l/16, column l%16),
// and output value v of lane l is element (row 4v + l/16, column l%16).
template <int P>
__device__ inline void mfma_64(const double (&sLT)[kGJBlock][P], const double (&sR)[kGJBlock][P], double sign,
                               d4 (&acc)[4]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll 4
  for (int ks = 0; ks < kGJBlock / 4; ++ks) {
    const int q = 4 * ks + (l >> 4);
    const double a = sign * sLT[q][16 * w + (l & 15)];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sR[q][16 * t + (l & 15)], acc[t], 0, 0, 0);
  }
}

// Row panel and update in one launch, grid (ceil(n / 64), ceil(n / 64)) of
// 64x64 tiles (J, I).  The block of tile (I, J) first forms its own 64 columns
// of the row panel, X_J = D A_KJ (X_K = D, from A_KK taken as the identity) --
// the ceil(n/64)-fold recomputation costs 64^3 multiply-adds per tile, less
// than a launch -- then
//   B_ij = X[i-k0][j]                                          (I = K)
//   B_ij = (J = K ? 0 : A_ij) - sum_q A[i][k0+q] X[q][j]        (otherwise).
// Both products run on the binary64 matrix cores from LDS operands, D^T /
// A_IK^T on the left (rows q, padded against bank conflicts) and A_KJ / X_J on
// the right.  The block of the next diagonal tile (kb+1, kb+1) then inverts
// its result in place and writes it transposed to DTnext, so the next step
// needs no separate launch.
__global__ __launch_bounds__(kBlock) void k_gj_panel_update(int n, int kb, int nb, const double* __restrict__ A,
                                                            const double* __restrict__ DT,
                                                            double* __restrict__ B, double* __restrict__ DTnext) {
  static_assert(kGJBlock == 64 && kBlock == 256, "four waves of 16 output rows");
  constexpr int P = kGJBlock + 1;
  __shared__ double sL[kGJBlock][P];  // D^T, then A_IK^T
  __shared__ double sR[kGJBlock][P];  // A_KJ (identity for J = K), then X_J
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int k0 = kb * kGJBlock, I = blockIdx.y, J = blockIdx.x;
  const int i0 = I * kGJBlock, j0 = J * kGJBlock;
  // row / column of output value v of tile t for this lane
  auto orow = [&](int v) { return 16 * w + 4 * v + (l >> 4); };
  auto ocol = [&](int t) { return 16 * t + (l & 15); };
  // every global load of a stage is issued before the first LDS store
  constexpr int kPer = kGJBlock * kGJBlock / kBlock;  // 16 elements per thread
  {
    double vl[kPer], vr[kPer];
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = threadIdx.x + kBlock * m, r = e >> 6, c = e & 63;
      vl[m] = (r < nb && c < nb) ? DT[r * kGJBlock + c] : 0.0;
      vr[m] = (r < nb && j0 + c < n) ? ((J == kb) ? (r == c ? 1.0 : 0.0) : A[(long long)(k0 + r) * n + j0 + c])
                                     : 0.0;
    }
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = threadIdx.x + kBlock * m, r = e >> 6, c = e & 63;
      sL[r][c] = vl[m];
      sR[r][c] = vr[m];
    }
  }
  __syncthreads();
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  mfma_64<P>(sL, sR, 1.0, acc);  // acc = X_J
  if (I == kb) {  // rows of the pivot block: B_K* = X
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + orow(v), j = j0 + ocol(t);
        if (i < n && j < n) B[(long long)i * n + j] = acc[t][v];
      }
    return;  // uniform per block
  }
  d4 y[4];
  {
    double va[kPer];
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = threadIdx.x + kBlock * m, r = e >> 6, c = e & 63;  // A[i0 + r][k0 + c] -> sL[c][r]
      va[m] = (i0 + r < n && c < nb) ? A[(long long)(i0 + r) * n + k0 + c] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + orow(v), j = j0 + ocol(t);
        y[t][v] = (J != kb && i < n && j < n) ? A[(long long)i * n + j] : 0.0;
      }
    __syncthreads();  // every read of sL and sR is done
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) sR[orow(v)][ocol(t)] = acc[t][v];
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = threadIdx.x + kBlock * m, r = e >> 6, c = e & 63;
      sL[c][r] = va[m];
    }
  }
  __syncthreads();
  mfma_64<P>(sL, sR, -1.0, y);  // y = A_IJ - A_IK X_J
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + orow(v), j = j0 + ocol(t);
      if (i < n && j < n) B[(long long)i * n + j] = y[t][v];
    }
  if (I == kb + 1 && J == kb + 1) {  // uniform per block
    // the new diagonal tile to LDS (identity beyond its nbn x nbn block), then its inverse
    __syncthreads();  // the product's reads of sR and sL are done
    const int nbn = min(n - i0, kGJBlock);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = orow(v), j = ocol(t);
        sR[i][j] = (i < nbn && j < nbn) ? y[t][v] : (i == j ? 1.0 : 0.0);
      }
    __shared__ double sQ[16][17], pr[2][4][16], pc[2][4][16];
    __syncthreads();
    block_inverse(sR, sL, sQ, pr, pc, DTnext);
  }
}

// B = (A + A^T) / 2 by 32x32 tiles: tile (I, J) reads the mirror tile (J, I)
// with rows along the lanes and transposes it through LDS, so both reads and
// the write are row-contiguous.
__global__ void k_symmetrize(int n, const double* __restrict__ A, double* __restrict__ B) {
  __shared__ double mt[32][33];
  const int i0 = 32 * blockIdx.y, j0 = 32 * blockIdx.x;
  const int c = threadIdx.x & 31, r0 = threadIdx.x >> 5;  // 8 rows of 32 per pass
#pragma unroll
  for (int p = 0; p < 4; ++p) {  // mirror tile: A[j0 + r][i0 + c] -> mt[r][c]
    const int r = r0 + 8 * p;
    mt[r][c] = (j0 + r < n && i0 + c < n) ? A[(long long)(j0 + r) * n + i0 + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int r = r0 + 8 * p, i = i0 + r, j = j0 + c;
    if (i < n && j < n) B[(long long)i * n + j] = 0.5 * (A[(long long)i * n + j] + mt[c][r]);
  }
}

template <typename T>
__device__ __forceinline__ void gemv_block(int n, const double* __restrict__ Ainv, const T* __restrict__ x,
                                           T* __restrict__ y, const int* __restrict__ act, int bx, int rhs) {
  const int row = bx * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= n || (act && !act[rhs])) return;  // uniform per wave
  gemv_row<T>(n, Ainv, x + (long long)n * rhs, y + (long long)n * rhs, row, threadIdx.x & 63);
}
template <typename T>
__global__ void k_coarse_gemv(int n, const double* __restrict__ Ainv, const T* __restrict__ x,
                              T* __restrict__ y, const int* __restrict__ act) {
  gemv_block<T>(n, Ainv, x, y, act, blockIdx.x, blockIdx.y);
}
template <typename T>
__global__ void k_coarse_gemv_batch(Batch<GemvTask<T>> tb) {
  const int t = batch_task(tb.begin, tb.n, (int)blockIdx.x);
  const GemvTask<T>& a = tb.a[t];
  const int local = (int)blockIdx.x - tb.begin[t];
  gemv_block<T>(a.n, a.Ainv, a.x, a.y, a.act, local % a.gx, local / a.gx);
}

// ---------------------------------------------------------------------------
// PCG vector kernels (binary64).
__global__ void k_dot_partial(long long n, const double* __restrict__ x, const double* __restrict__ y,
                              double* __restrict__ partials, const int* __restrict__ act) {
  x += n * blockIdx.y;  // right-hand side
  y += n * blockIdx.y;
  partials += (long long)kReduceBlocks * blockIdx.y;
  if (act && !act[blockIdx.y]) {
    if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  double s = 0.0;
#pragma unroll 4
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    s += x[i] * y[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// block r: out[r * stride] = sum of partials[r][0 .. kReduceBlocks)
__global__ void k_reduce_final(const double* __restrict__ partials, double* __restrict__ out, int stride) {
  partials += (long long)kReduceBlocks * blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < kReduceBlocks; i += kBlock) s += partials[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[(long long)stride * blockIdx.x] = s;
}

// block r: out[r] = sum of parts[r][0 .. n) in a fixed order (the partials of
// a streaming-kernel launch with more workgroups than a vector kernel's block
// should sum on its own); skipped for an inactive right-hand side.  One block
// of 1024 threads with eight independent chains each keeps enough loads in
// flight that the ~70 k partials of a large level take a few microseconds.
constexpr int kSumThreads = 1024;
// The per-iteration CG vector passes: each of the kReduceBlocks workgroups
// walks contiguous ranges of kVecChunk elements, kReduceBlocks ranges apart
// (measured faster than an element-wise grid stride at the same launch).
constexpr long long kVecChunk = 4096;
__global__ __launch_bounds__(kSumThreads) void k_sum_parts(const double* __restrict__ parts, int n,
                                                           double* __restrict__ out, const int* __restrict__ act) {
  if (act && !act[blockIdx.x]) return;
  parts += (long long)n * blockIdx.x;
  double a[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u] = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * kSumThreads < n; i += 8 * kSumThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += parts[i + u * kSumThreads];
  }
  for (; i < n; i += kSumThreads) a[0] += parts[i];
  double v = wave_sum(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
  __shared__ double part[kSumThreads / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kSumThreads / 64; ++w) t += part[w];
    out[blockIdx.x] = t;
  }
}

// grid (kReduceBlocks, nrhs): r = M f (fixed DOFs zeroed), x = 0 and the
// partials of ||r||^2 (the summation order of k_dot_partial)
__global__ void k_pcg_start(Level L, const double* __restrict__ f, double* __restrict__ r, double* __restrict__ x,
                            double* __restrict__ partials) {
  const long long n = 3ll * L.nn;
  const long long off = n * blockIdx.y;
  f += off;
  r += off;
  x += off;
  partials += (long long)kReduceBlocks * blockIdx.y;
  double acc = 0.0;
#pragma unroll 4
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int node = (int)(i / 3), c = (int)(i % 3);
    const double ri = ((L.mask[node] >> c) & 1) ? 0.0 : f[i];
    r[i] = ri;
    x[i] = 0.0;
    acc += ri * ri;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// One block per right-hand side: ff = ||M f||^2 from the partials, then
// active = (ff > 0), its = 0, stop = rtol^2 ff (rtol2 <= 0: never)
__global__ void k_pcg_init(double rtol2, const double* __restrict__ ff_partials, double* __restrict__ sc,
                           int* __restrict__ active) {
  const int r = blockIdx.x;
  const double ff = sum_partials(ff_partials + (long long)kReduceBlocks * r);
  if (threadIdx.x != 0) return;
  double* s = sc + kScalars * r;
  s[kFf] = ff;
  const bool finite = ff == ff && ff < 1e308;
  const int a = (ff > 0.0 && finite) ? 1 : 0;
  active[r] = a;
  s[kActive] = a;
  s[kIts] = 0.0;
  s[kStatus] = !finite ? -4.0 : (ff > 0.0 ? 1.0 : 0.0);
  s[kStop] = rtol2 > 0.0 ? rtol2 * ff : -1.0;
  s[kRr] = ff;
  s[kPq] = 0.0;
  s[kXPend] = 0.0;
  s[kAlphaP] = 0.0;
  s[kAlphaP + 1] = 0.0;
}

// grid (kReduceBlocks, nrhs), after q = A x: the partials of ||M f - q||^2
// (true residual) into pa and of f . x into pb (the order of k_dot_partial)
__global__ void k_pcg_final_dots(Level L, const double* __restrict__ f, const double* __restrict__ q,
                                 const double* __restrict__ x, double* __restrict__ pa, double* __restrict__ pb) {
  const long long n = 3ll * L.nn;
  const long long off = n * blockIdx.y;
  f += off;
  q += off;
  x += off;
  double a = 0.0, b = 0.0;
#pragma unroll 4
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int node = (int)(i / 3), c = (int)(i % 3);
    const double fi = f[i];
    const double ri = (((L.mask[node] >> c) & 1) ? 0.0 : fi) - q[i];
    a += ri * ri;
    b += fi * x[i];
  }
  a = block_sum(a);
  b = block_sum(b);
  if (threadIdx.x == 0) {
    pa[(long long)kReduceBlocks * blockIdx.y + blockIdx.x] = a;
    pb[(long long)kReduceBlocks * blockIdx.y + blockIdx.x] = b;
  }
}

// grid (nrhs, 2): sc[kTmp] = sum of pa, sc[kTmp2] = sum of pb, per right-hand side
__global__ void k_pcg_final_sums(const double* __restrict__ pa, const double* __restrict__ pb,
                                 double* __restrict__ sc) {
  const double* p = (blockIdx.y ? pb : pa) + (long long)kReduceBlocks * blockIdx.x;
  const double v = sum_partials(p);
  if (threadIdx.x == 0) sc[kScalars * blockIdx.x + (blockIdx.y ? kTmp2 : kTmp)] = v;
}

// grid (kReduceBlocks, nrhs).  alpha = rz / pq with pq the sum of npq partials
// per right-hand side; every block sums the same partials in the same order,
// so all blocks use the identical alpha.  r -= alpha q and the partials of
// ||r||^2, fused with the first Jacobi sweep from zero of the preconditioner
// that follows (t = omega D^{-1} r; in mixed precision on the binary32 copy of
// r, written to f32).  t may be null (no sweep: the coarsest level is the
// whole grid).  The matching x += alpha p is left to k_update_px, or to
// k_flush_x when the solve stops; s[kXPend] records whether it is due.
// TQ: q in binary64, or the binary32 A p of the binary32 outer product
// (widened on the fly).  repl (may be null): right-hand sides whose flag is
// set get only alpha and the pending flag (their residual is replaced right
// after, see k_replace_r).
template <typename TW, typename TQ>
__device__ __forceinline__ void update_r_first_block(long long n, const double* __restrict__ pq_partials, int npq,
                                                     double* __restrict__ sc, const int* __restrict__ active,
                                                     const TQ* __restrict__ q, double* __restrict__ r,
                                                     double* __restrict__ rr_partials, int parity,
                                                     const TW* __restrict__ wdinv, float* __restrict__ f32,
                                                     TW* __restrict__ t, const int* __restrict__ repl, int bx,
                                                     int rhs) {
  constexpr int gx = kReduceBlocks;
  rr_partials += (long long)kReduceBlocks * rhs;
  if (!active[rhs]) {
    if (threadIdx.x == 0) rr_partials[bx] = 0.0;
    return;
  }
  double pqs = 0.0;
  for (int i = threadIdx.x; i < npq; i += kBlock) pqs += pq_partials[(long long)npq * rhs + i];
  const double pq = block_sum_all(pqs);
  double* s = sc + kScalars * rhs;
  const double alpha = s[kRz0 + parity] / pq;
  const bool ok = pq > 0.0 && pq < 1e308;
  if (bx == 0 && threadIdx.x == 0) {
    s[kPq] = pq;
    s[kAlpha] = alpha;
    s[kXPend] = ok ? 1.0 : 0.0;
    s[kAlphaP + parity] = ok ? alpha : 0.0;
  }
  if (!ok || (repl && repl[rhs])) {  // breakdown: keep the previous iterate; the check flags it
    if (threadIdx.x == 0) rr_partials[bx] = 0.0;
    return;
  }
  const long long off = n * rhs;
  q += off;
  r += off;
  if (f32) f32 += off;
  if (t) t += off;
  double acc = 0.0;
  for (long long b0 = (long long)bx * kVecChunk; b0 < n; b0 += (long long)gx * kVecChunk) {
    const long long e = min(b0 + kVecChunk, n);
#pragma unroll 4
    for (long long i = b0 + threadIdx.x; i < e; i += kBlock) {
      const double ri = r[i] - alpha * (double)q[i];
      r[i] = ri;
      acc += ri * ri;
      if constexpr (sizeof(TW) == 4) {
        const float fv = (float)ri;
        f32[i] = fv;
        if (t) t[i] = wdinv[i] * fv;
      } else {
        if (t) t[i] = wdinv[i] * ri;
      }
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) rr_partials[bx] = acc;
}
template <typename TW, typename TQ>
__global__ void k_update_r_first(long long n, const double* __restrict__ pq_partials, int npq,
                                 double* __restrict__ sc, const int* __restrict__ active,
                                 const TQ* __restrict__ q, double* __restrict__ r,
                                 double* __restrict__ rr_partials, int parity, const TW* __restrict__ wdinv,
                                 float* __restrict__ f32, TW* __restrict__ t, const int* __restrict__ repl) {
  update_r_first_block<TW, TQ>(n, pq_partials, npq, sc, active, q, r, rr_partials, parity, wdinv, f32, t, repl,
                               blockIdx.x, blockIdx.y);
}
template <typename TW, typename TQ>
__global__ void k_update_r_first_batch(Batch<UpdateRTask<TW, TQ>> tb) {
  const int t = batch_task(tb.begin, tb.n, (int)blockIdx.x);
  const UpdateRTask<TW, TQ>& a = tb.a[t];
  const int local = (int)blockIdx.x - tb.begin[t];
  update_r_first_block<TW, TQ>(a.n, a.pq_partials, a.npq, a.sc, a.active, a.q, a.r, a.rr_partials, a.parity,
                               a.wdinv, a.f32, a.t, a.repl, local % kReduceBlocks, local / kReduceBlocks);
}


// One block per right-hand side: ||r||^2, iteration count, convergence and
// breakdown test; then the scalars are written to host_slot (pinned host
// memory, kScalars per right-hand side), where the host reads them without a
// copy.  A right-hand side that has stopped only republishes its scalars.
__device__ __forceinline__ void rr_check_block(const double* __restrict__ rr_partials, double* __restrict__ sc,
                                               int* __restrict__ active, double* __restrict__ host_slot, int rhs) {
  const double rr = sum_partials(rr_partials + (long long)kReduceBlocks * rhs);
  if (threadIdx.x != 0) return;
  double* s = sc + kScalars * rhs;
  double v[kScalars];
#pragma unroll
  for (int j = 0; j < kScalars; ++j) v[j] = s[j];
  if (active[rhs]) {
    v[kRr] = rr;
    v[kIts] += 1.0;
    const bool finite = rr == rr && rr < 1e308;
    int act = 1;
    if (!(v[kPq] > 0.0 && v[kPq] < 1e308) || !finite) {
      act = 0;
      v[kStatus] = -5.0;
    } else if (rr <= v[kStop]) {
      act = 0;
      v[kStatus] = 0.0;
    }
    v[kActive] = act;
    active[rhs] = act;
#pragma unroll
    for (int j = 0; j < kScalars; ++j) s[j] = v[j];
  }
#pragma unroll
  for (int j = 0; j < kScalars; ++j) host_slot[kScalars * rhs + j] = v[j];
  __threadfence_system();
}
__global__ void k_rr_check(const double* __restrict__ rr_partials, double* __restrict__ sc,
                           int* __restrict__ active, double* __restrict__ host_slot) {
  rr_check_block(rr_partials, sc, active, host_slot, blockIdx.x);
}
__global__ void k_rr_check_batch(Batch<RrCheckTask> tb) {
  const int t = batch_task(tb.begin, tb.n, (int)blockIdx.x);
  const RrCheckTask& a = tb.a[t];
  rr_check_block(a.rr_partials, a.sc, a.active, a.host_slot, (int)blockIdx.x - tb.begin[t]);
}

// grid (kReduceBlocks, nrhs): beta from the nrz rz partials (every block sums
// them in the same order); the previous
// iteration's x += alpha p (always due while the right-hand side is active:
// a breakdown clears the flag), then p = z + beta p.  z in binary64, or the
// binary32 V-cycle output widened on the fly.
// The x update is skipped when s[kXPend] is 0 (a residual replacement has
// already applied it); p32 (may be null) receives a binary32 copy of the new p.
template <typename TZ>
__device__ __forceinline__ void update_px_block(long long n, const double* __restrict__ rz_partials, int nrz,
                                                double* __restrict__ sc, const int* __restrict__ active,
                                                const TZ* __restrict__ z, double* __restrict__ p,
                                                double* __restrict__ x, int parity, float* __restrict__ p32,
                                                float* __restrict__ p32b, int bx, int rhs) {
  constexpr int gx = kReduceBlocks;
  if (!active[rhs]) return;
  double rzs = 0.0;
  for (int i = threadIdx.x; i < nrz; i += kBlock) rzs += rz_partials[(long long)nrz * rhs + i];
  const double rz = block_sum_all(rzs);
  double* s = sc + kScalars * rhs;
  const double beta = rz / s[kRz0 + parity];
  const double alpha = s[kXPend] != 0.0 ? s[kAlpha] : 0.0;
  if (bx == 0 && threadIdx.x == 0) {
    s[kRz0 + 1 - parity] = rz;
    s[kBeta] = beta;
  }
  const long long off = n * rhs;
  z += off;
  x += off;
  if (p32) p32 += off;
  if (!p) {
    // The direction is held in binary32 only, p_k of iteration k in p32 (k odd)
    // or p32b (k even); parity = (k - 1) & 1.  After an odd k: p_(k+1) = z +
    // beta p_k into p32b.  After an even k: x += alpha_(k-1) p_(k-1) (p32), x +=
    // alpha_k p_k (p32b), and p_(k+1) = z + beta p_k into p32, over p_(k-1).
    p32b += off;
    if (parity) {
      const double a_odd = s[kAlphaP], a_even = s[kAlphaP + 1];
      for (long long b0 = (long long)bx * kVecChunk; b0 < n; b0 += (long long)gx * kVecChunk) {
        const long long e = min(b0 + kVecChunk, n);
#pragma unroll 4
        for (long long i = b0 + threadIdx.x; i < e; i += kBlock) {
          const double po = (double)p32[i], pe = (double)p32b[i];
          double xi = x[i];
          xi += a_odd * po;
          xi += a_even * pe;
          x[i] = xi;
          p32[i] = (float)((double)z[i] + beta * pe);
        }
      }
    } else {
      for (long long b0 = (long long)bx * kVecChunk; b0 < n; b0 += (long long)gx * kVecChunk) {
        const long long e = min(b0 + kVecChunk, n);
#pragma unroll 4
        for (long long i = b0 + threadIdx.x; i < e; i += kBlock)
          p32b[i] = (float)((double)z[i] + beta * (double)p32[i]);
      }
    }
    return;
  }
  p += off;
  for (long long b0 = (long long)bx * kVecChunk; b0 < n; b0 += (long long)gx * kVecChunk) {
    const long long e = min(b0 + kVecChunk, n);
    if (p32) {
#pragma unroll 4
      for (long long i = b0 + threadIdx.x; i < e; i += kBlock) {
        const double pi = p[i];
        x[i] += alpha * pi;
        const double pn = (double)z[i] + beta * pi;
        p[i] = pn;
        p32[i] = (float)pn;
      }
    } else {
#pragma unroll 4
      for (long long i = b0 + threadIdx.x; i < e; i += kBlock) {
        const double pi = p[i];
        x[i] += alpha * pi;
        p[i] = (double)z[i] + beta * pi;
      }
    }
  }
}
template <typename TZ>
__global__ void k_update_px(long long n, const double* __restrict__ rz_partials, int nrz, double* __restrict__ sc,
                            const int* __restrict__ active, const TZ* __restrict__ z, double* __restrict__ p,
                            double* __restrict__ x, int parity, float* __restrict__ p32, float* __restrict__ p32b) {
  update_px_block<TZ>(n, rz_partials, nrz, sc, active, z, p, x, parity, p32, p32b, blockIdx.x, blockIdx.y);
}
template <typename TZ>
__global__ void k_update_px_batch(Batch<UpdatePxTask<TZ>> tb) {
  const int t = batch_task(tb.begin, tb.n, (int)blockIdx.x);
  const UpdatePxTask<TZ>& a = tb.a[t];
  const int local = (int)blockIdx.x - tb.begin[t];
  update_px_block<TZ>(a.n, a.rz_partials, a.nrz, a.sc, a.active, a.z, a.p, a.x, a.parity, a.p32, a.p32b,
                      local % kReduceBlocks, local / kReduceBlocks);
}

// grid (kReduceBlocks, nrhs), residual replacement after q = A x in binary64
// (x complete, its pending update already applied): r = M f - q, the partials
// of ||r||^2 (the order of k_dot_partial), the binary32 copy of r and the
// preconditioner's first sweep t = omega D^-1 r (t may be null); clears
// s[kXPend].  Right-hand sides whose flag is 0 are skipped.
__global__ void k_replace_r(Level L, const double* __restrict__ f, const double* __restrict__ q,
                            double* __restrict__ r, double* __restrict__ rr_partials, const float* __restrict__ wdinv,
                            float* __restrict__ f32, float* __restrict__ t, double* __restrict__ sc,
                            const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  rr_partials += (long long)kReduceBlocks * rhs;
  if (!active[rhs]) {
    if (threadIdx.x == 0) rr_partials[blockIdx.x] = 0.0;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[kScalars * rhs + kXPend] = 0.0;
  const long long n = 3ll * L.nn;
  const long long off = n * rhs;
  f += off;
  q += off;
  r += off;
  f32 += off;
  if (t) t += off;
  double acc = 0.0;
#pragma unroll 4
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int node = (int)(i / 3), c = (int)(i % 3);
    const double ri = (((L.mask[node] >> c) & 1) ? 0.0 : f[i]) - q[i];
    r[i] = ri;
    acc += ri * ri;
    const float fv = (float)ri;
    f32[i] = fv;
    if (t) t[i] = wdinv[i] * fv;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) rr_partials[blockIdx.x] = acc;
}

// One thread per right-hand side: repl = the right-hand side is active and
// the iteration about to run is a multiple of every (its iterations so far + 1).
__global__ void k_replace_flags(const double* __restrict__ sc, const int* __restrict__ active,
                                int* __restrict__ repl, int nrhs, int every) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  const long long next = (long long)sc[kScalars * rhs + kIts] + 1;
  repl[rhs] = (active[rhs] && next % every == 0) ? 1 : 0;
}

// One thread per right-hand side, after the binary64 residual of a finished
// solve is in s[kTmp]: a right-hand side whose recursive residual met the
// test while the binary64 one does not (and that has iterations left) is
// restarted: active again, status 1, ||r||^2 = that residual.
__global__ void k_pcg_restart(double* __restrict__ sc, int* __restrict__ active, int nrhs, int maxit) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  double* s = sc + kScalars * rhs;
  const bool again = s[kStatus] == 0.0 && s[kTmp] > s[kStop] && s[kIts] < maxit;
  active[rhs] = again ? 1 : 0;
  s[kActive] = again ? 1.0 : 0.0;
  if (again) {
    s[kStatus] = 1.0;
    s[kRr] = s[kTmp];
  }
}

// grid (kReduceBlocks, nrhs): the x += alpha p still due when the solve stops
// (act, may be null: only the right-hand sides whose flag is set)
template <typename TP>
__global__ void k_flush_x(long long n, const double* __restrict__ sc, const TP* __restrict__ p,
                          double* __restrict__ x, const int* __restrict__ act) {
  const int rhs = blockIdx.y;
  const double* s = sc + kScalars * rhs;
  if (s[kXPend] == 0.0 || (act && !act[rhs])) return;
  const double alpha = s[kAlpha];
  const long long off = n * rhs;
  p += off;
  x += off;
#pragma unroll 4
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    x[i] += alpha * (double)p[i];
}
// The same for the binary32 directions of the mixed form (launch_update_px):
// after the last iteration k, p_k (p32 for odd k) is pending, and for even k
// p_(k-1) (p32) before it; a breakdown left its alpha 0.
__global__ void k_flush_x_pair(long long n, const double* __restrict__ sc, const float* __restrict__ p32,
                               const float* __restrict__ p32b, double* __restrict__ x, const int* __restrict__ act) {
  const int rhs = blockIdx.y;
  const double* s = sc + kScalars * rhs;
  const long long k = (long long)s[kIts];
  if (k == 0 || (act && !act[rhs])) return;
  const bool even = (k & 1) == 0;
  const double a_odd = s[kAlphaP], a_even = s[kAlphaP + 1];
  const long long off = n * rhs;
  p32 += off;
  p32b += off;
  x += off;
  if (even && a_even == 0.0) {  // breakdown in the last iteration: only p_(k-1) is due
    if (a_odd == 0.0) return;
#pragma unroll 4
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
      x[i] += a_odd * (double)p32[i];
  } else if (even) {
#pragma unroll 4
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
      double xi = x[i];
      xi += a_odd * (double)p32[i];
      xi += a_even * (double)p32b[i];
      x[i] = xi;
    }
  } else if (a_odd != 0.0) {
#pragma unroll 4
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
      x[i] += a_odd * (double)p32[i];
  }
}

// partials of r . (double) u32 (grid (kReduceBlocks, nrhs)); the widened z is not stored
__global__ void k_dot_mixed(long long n, const float* __restrict__ u32, const double* __restrict__ r,
                            double* __restrict__ partials, const int* __restrict__ act) {
  const int rhs = blockIdx.y;
  partials += (long long)kReduceBlocks * rhs;
  if (act && !act[rhs]) {
    if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  const long long off = n * rhs;
  double acc = 0.0;
#pragma unroll 4
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    acc += r[off + i] * (double)u32[off + i];
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// z = (double) u32 and the partials of r . z (grid (kReduceBlocks, nrhs))
__global__ void k_to64_dot(long long n, const float* __restrict__ u32, const double* __restrict__ r,
                           double* __restrict__ z, double* __restrict__ partials, const int* __restrict__ act) {
  const int rhs = blockIdx.y;
  partials += (long long)kReduceBlocks * rhs;
  if (act && !act[rhs]) {
    if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  const long long off = n * rhs;
  double acc = 0.0;
#pragma unroll 4
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const double zi = (double)u32[off + i];
    z[off + i] = zi;
    acc += r[off + i] * zi;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ void k_f64_to_f32(long long n, const double* __restrict__ a, float* __restrict__ b,
                             const int* __restrict__ act) {
  if (act && !act[blockIdx.y]) return;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long off = n * blockIdx.y;
  if (i < n) b[off + i] = (float)a[off + i];
}

}  // namespace

// ---- launchers ------------------------------------------------------------
template <typename T>
void launch_gather(int mode, const Level& L, const T* Ke, const T* E, const T* u, const T* f,
                   const T* wdinv, T* y, int nrhs, const int* act, hipStream_t s, const LaunchTimer& t) {
  const dim3 g(blocks_for(L.nn), nrhs);
  if (mode == kApply)
    launch_timed(k_gather<T, kApply>, g, dim3(kBlock), s, t, L, Ke, E, u, f, wdinv, y, act);
  else if (mode == kSmooth)
    launch_timed(k_gather<T, kSmooth>, g, dim3(kBlock), s, t, L, Ke, E, u, f, wdinv, y, act);
  else
    launch_timed(k_gather<T, kResidual>, g, dim3(kBlock), s, t, L, Ke, E, u, f, wdinv, y, act);
}
template void launch_gather<double>(int, const Level&, const double*, const double*, const double*,
                                    const double*, const double*, double*, int, const int*, hipStream_t,
                                    const LaunchTimer&);
template void launch_gather<float>(int, const Level&, const float*, const float*, const float*,
                                   const float*, const float*, float*, int, const int*, hipStream_t,
                                   const LaunchTimer&);
void launch_gather_apply_u32(const Level& L, const double* Ke, const double* E, const float* u, double* y, int nrhs,
                             const int* act, hipStream_t s, const LaunchTimer& t) {
  const dim3 g(blocks_for(L.nn), nrhs);
  launch_timed(k_gather<double, kApply, float>, g, dim3(kBlock), s, t, L, Ke, E, u, (const double*)nullptr,
               (const double*)nullptr, y, act);
}

template <typename T>
void launch_jacobi_first(long long n, const T* wdinv, const T* f, T* u, int nrhs, const int* act, hipStream_t s) {
  k_jacobi_first<T><<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(n, wdinv, f, u, act);
}
template void launch_jacobi_first<double>(long long, const double*, const double*, double*, int, const int*,
                                          hipStream_t);
template void launch_jacobi_first<float>(long long, const float*, const float*, float*, int, const int*,
                                         hipStream_t);
void launch_jacobi_first_from64(long long n, const float* wdinv, const double* r, float* f32, float* u, int nrhs,
                                const int* act, hipStream_t s) {
  k_jacobi_first_from64<<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(n, wdinv, r, f32, u, act);
}

template <typename T>
void launch_restrict(const Level& F, const Level& C, const T* r, T* fc, int nrhs, const int* act, hipStream_t s,
                     const T* wdc, T* tc) {
  // a slab: the blocks of one coarse plane
  const int slab = band_slab(((long long)C.nxn * C.nyn + kBlock - 1) / kBlock);
  k_restrict<T><<<dim3(blocks_for(C.nn), nrhs), kBlock, 0, s>>>(F, C, r, fc, act, wdc, tc, slab);
}
template void launch_restrict<double>(const Level&, const Level&, const double*, double*, int, const int*,
                                      hipStream_t, const double*, double*);
template void launch_restrict<float>(const Level&, const Level&, const float*, float*, int, const int*,
                                     hipStream_t, const float*, float*);

template <typename T>
void launch_prolong_add(const Level& F, const Level& C, const T* ec, T* u, int nrhs, const int* act,
                        hipStream_t s) {
  // a slab: the blocks of the row quads of one pair of fine planes
  const int slab = band_slab((long long)((F.nxn + 63) / 64) * ((((F.nyn + 1) / 2) + 3) / 4));
  k_prolong_add<T><<<dim3(prolong_blocks(F), nrhs), kBlock, 0, s>>>(F, C, ec, u, act, slab);
}
template void launch_prolong_add<double>(const Level&, const Level&, const double*, double*, int, const int*,
                                         hipStream_t);
template void launch_prolong_add<float>(const Level&, const Level&, const float*, float*, int, const int*,
                                        hipStream_t);

void launch_simp(int ne, const double* rho, double E0, double Emin, double p, double scale,
                 double* E64, float* E32, double* rho_copy, int* bad_flags, hipStream_t s) {
  k_simp<<<kReduceBlocks, kBlock, 0, s>>>(ne, rho, E0, Emin, p, scale, E64, E32, rho_copy, bad_flags);
}
void launch_or_flags(int n, const int* flags, int* out, hipStream_t s) {
  k_or_flags<<<1, kBlock, 0, s>>>(n, flags, out);
}
void launch_homogenize(const Level& F, const Level& C, const double* vf, double* vc, hipStream_t s) {
  k_homogenize<<<blocks_for(C.ne), kBlock, 0, s>>>(F, C, vf, vc);
}
void launch_modulus_from_density(int ne, const double* rho, double E0, double Emin, double p,
                                 double scale, double* E64, float* E32, hipStream_t s) {
  k_modulus_from_density<<<blocks_for(ne), kBlock, 0, s>>>(ne, rho, E0, Emin, p, scale, E64, E32);
}
void launch_modulus_from_mean(const Level& F, const Level& C, const double* Ef, double scale,
                              double* E64, float* E32, hipStream_t s) {
  k_modulus_from_mean<<<blocks_for(C.ne), kBlock, 0, s>>>(F, C, Ef, scale, E64, E32);
}
void launch_coarsest_moduli(const Level& F, const Level& C, int blk, const double* v0, bool density, double E0,
                            double Emin, double p, double scale, double* Ec, hipStream_t s) {
  k_coarsest_moduli<<<C.ne, kBlock, 0, s>>>(F, C, blk, v0, density ? 1 : 0, E0, Emin, p, scale, Ec);
}
void launch_diag(const Level& L, const double* Ke, const double* E, double omega, double* wdinv64,
                 float* wdinv32, hipStream_t s) {
  k_diag<<<blocks_for(L.nn), kBlock, 0, s>>>(L, Ke, E, omega, wdinv64, wdinv32);
}
void launch_mask_default(const Level& L, uint8_t* mask, hipStream_t s) {
  k_mask_default<<<blocks_for(L.nn), kBlock, 0, s>>>(L, mask);
}
void launch_mask_inject(const Level& F, const Level& C, const uint8_t* mf, uint8_t* mc, hipStream_t s) {
  k_mask_inject<<<blocks_for(C.nn), kBlock, 0, s>>>(F, C, mf, mc);
}

void launch_coarse_assemble(const Level& C, const double* Ke, const double* E, double* A, hipStream_t s) {
  const int N = 3 * C.nn;
  k_coarse_assemble<<<dim3(blocks_for(N), N), kBlock, 0, s>>>(C, Ke, E, A);
}
void launch_gj_blocked(int n, double* A, double* B, double* D, double** result, hipStream_t s) {
  double* buf[2] = {A, B};
  double* dt[2] = {D, D + kGJBlock * kGJBlock};  // pivot inverses, alternating by step
  int cur = 0;
  const int t = (n + 63) / 64;
  k_gj_block_inv<<<1, kBlock, 0, s>>>(n, 0, n < kGJBlock ? n : kGJBlock, A, dt[0]);
  for (int kb = 0; kb < t; ++kb) {
    const int k0 = kb * kGJBlock;
    const int nb = (n - k0) < kGJBlock ? (n - k0) : kGJBlock;
    k_gj_panel_update<<<dim3(t, t), kBlock, 0, s>>>(n, kb, nb, buf[cur], dt[kb & 1], buf[1 - cur], dt[(kb + 1) & 1]);
    cur = 1 - cur;
  }
  *result = buf[cur];
}
void launch_symmetrize(int n, const double* A, double* B, hipStream_t s) {
  k_symmetrize<<<dim3((n + 31) / 32, (n + 31) / 32), kBlock, 0, s>>>(n, A, B);
}
template <typename T>
void launch_coarse_gemv(int n, const double* Ainv, const T* x, T* y, int nrhs, const int* act, hipStream_t s) {
  const int rows_per_block = kBlock / 64;
  k_coarse_gemv<T><<<dim3((n + rows_per_block - 1) / rows_per_block, nrhs), kBlock, 0, s>>>(n, Ainv, x, y, act);
}
template void launch_coarse_gemv<double>(int, const double*, const double*, double*, int, const int*, hipStream_t);
template void launch_coarse_gemv<float>(int, const double*, const float*, float*, int, const int*, hipStream_t);

void launch_dot_partial(long long n, const double* x, const double* y, double* partials, int nrhs, const int* act,
                        hipStream_t s) {
  k_dot_partial<<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, x, y, partials, act);
}
void launch_sum_parts(const double* parts, int n, double* out, int nrhs, const int* act, hipStream_t s) {
  k_sum_parts<<<nrhs, kSumThreads, 0, s>>>(parts, n, out, act);
}
void launch_reduce_final(const double* partials, double* out, int stride, int nrhs, hipStream_t s) {
  k_reduce_final<<<nrhs, kBlock, 0, s>>>(partials, out, stride);
}
void launch_pcg_start(const Level& L, const double* f, double* r, double* x, double* partials, int nrhs,
                      hipStream_t s) {
  k_pcg_start<<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(L, f, r, x, partials);
}
void launch_pcg_init(double rtol2, const double* ff_partials, double* sc, int* active, int nrhs, hipStream_t s) {
  k_pcg_init<<<nrhs, kBlock, 0, s>>>(rtol2, ff_partials, sc, active);
}
void launch_pcg_final(const Level& L, const double* f, const double* q, const double* x, double* pa, double* pb,
                      double* sc, int nrhs, hipStream_t s) {
  k_pcg_final_dots<<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(L, f, q, x, pa, pb);
  k_pcg_final_sums<<<dim3(nrhs, 2), kBlock, 0, s>>>(pa, pb, sc);
}
template <typename TW, typename TQ>
void launch_update_r_first(long long n, const double* pq_partials, int npq, double* sc, const int* active,
                           const TQ* q, double* r, double* rr_partials, int parity, const TW* wdinv, float* f32,
                           TW* t, int nrhs, hipStream_t s, const int* repl) {
  k_update_r_first<TW, TQ><<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, pq_partials, npq, sc, active, q, r,
                                                                         rr_partials, parity, wdinv, f32, t, repl);
}
template void launch_update_r_first<double, double>(long long, const double*, int, double*, const int*,
                                                    const double*, double*, double*, int, const double*, float*,
                                                    double*, int, hipStream_t, const int*);
template void launch_update_r_first<float, double>(long long, const double*, int, double*, const int*,
                                                   const double*, double*, double*, int, const float*, float*,
                                                   float*, int, hipStream_t, const int*);
template void launch_update_r_first<float, float>(long long, const double*, int, double*, const int*,
                                                  const float*, double*, double*, int, const float*, float*, float*,
                                                  int, hipStream_t, const int*);
void launch_replace_flags(const double* sc, const int* active, int* repl, int nrhs, int every, hipStream_t s) {
  k_replace_flags<<<(nrhs + 63) / 64, 64, 0, s>>>(sc, active, repl, nrhs, every);
}
void launch_replace_r(const Level& L, const double* f, const double* q, double* r, double* rr_partials,
                      const float* wdinv, float* f32, float* t, double* sc, const int* active, int nrhs,
                      hipStream_t s) {
  k_replace_r<<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(L, f, q, r, rr_partials, wdinv, f32, t, sc, active);
}
void launch_pcg_restart(double* sc, int* active, int nrhs, int maxit, hipStream_t s) {
  k_pcg_restart<<<(nrhs + 63) / 64, 64, 0, s>>>(sc, active, nrhs, maxit);
}

void launch_rr_check(const double* rr_partials, double* sc, int* active, double* host_slot, int nrhs,
                     hipStream_t s) {
  k_rr_check<<<nrhs, kBlock, 0, s>>>(rr_partials, sc, active, host_slot);
}
template <typename TZ>
void launch_update_px(long long n, const double* rz_partials, int nrz, double* sc, const int* active, const TZ* z,
                      double* p, double* x, int parity, int nrhs, hipStream_t s, float* p32, float* p32b) {
  k_update_px<TZ><<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, rz_partials, nrz, sc, active, z, p, x, parity,
                                                                p32, p32b);
}
template void launch_update_px<double>(long long, const double*, int, double*, const int*, const double*, double*,
                                       double*, int, int, hipStream_t, float*, float*);
template void launch_update_px<float>(long long, const double*, int, double*, const int*, const float*, double*,
                                      double*, int, int, hipStream_t, float*, float*);
void launch_flush_x(long long n, const double* sc, const double* p, double* x, int nrhs, hipStream_t s,
                    const int* act, const float* p32, const float* p32b) {
  if (p)
    k_flush_x<double><<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, sc, p, x, act);
  else if (p32b)
    k_flush_x_pair<<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, sc, p32, p32b, x, act);
  else
    k_flush_x<float><<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, sc, p32, x, act);
}
void launch_dot_mixed(long long n, const float* u32, const double* r, double* partials, int nrhs, const int* act,
                      hipStream_t s) {
  k_dot_mixed<<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, u32, r, partials, act);
}
void launch_to64_dot(long long n, const float* u32, const double* r, double* z, double* partials, int nrhs,
                     const int* act, hipStream_t s) {
  k_to64_dot<<<dim3(kReduceBlocks, nrhs), kBlock, 0, s>>>(n, u32, r, z, partials, act);
}
void launch_f64_to_f32(long long n, const double* a, float* b, int nrhs, const int* act, hipStream_t s) {
  k_f64_to_f32<<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(n, a, b, act);
}

// ---------------------------------------------------------------------------
// Batched launches (several grids; see Batch in hexmg_impl.h).
int restrict_blocks(const Level& C) { return blocks_for(C.nn); }
int prolong_blocks(const Level& F) {
  return ((F.nxn + 63) / 64) * ((((F.nyn + 1) / 2) * ((F.nzn + 1) / 2) + 3) / 4);
}
int gemv_blocks(int n) { return (n + kBlock / 64 - 1) / (kBlock / 64); }

template <typename T>
void launch_restrict_batch(const Batch<RestrictTask<T>>& b, hipStream_t s) {
  k_restrict_batch<T><<<b.begin[b.n], kBlock, 0, s>>>(b);
}
template void launch_restrict_batch<float>(const Batch<RestrictTask<float>>&, hipStream_t);
template void launch_restrict_batch<double>(const Batch<RestrictTask<double>>&, hipStream_t);

template <typename T>
void launch_prolong_add_batch(const Batch<ProlongTask<T>>& b, hipStream_t s) {
  k_prolong_add_batch<T><<<b.begin[b.n], kBlock, 0, s>>>(b);
}
template void launch_prolong_add_batch<float>(const Batch<ProlongTask<float>>&, hipStream_t);
template void launch_prolong_add_batch<double>(const Batch<ProlongTask<double>>&, hipStream_t);

template <typename T>
void launch_coarse_gemv_batch(const Batch<GemvTask<T>>& b, hipStream_t s) {
  k_coarse_gemv_batch<T><<<b.begin[b.n], kBlock, 0, s>>>(b);
}
template void launch_coarse_gemv_batch<float>(const Batch<GemvTask<float>>&, hipStream_t);
template void launch_coarse_gemv_batch<double>(const Batch<GemvTask<double>>&, hipStream_t);

template <typename TW, typename TQ>
void launch_update_r_first_batch(const Batch<UpdateRTask<TW, TQ>>& b, hipStream_t s) {
  k_update_r_first_batch<TW, TQ><<<b.begin[b.n], kBlock, 0, s>>>(b);
}
template void launch_update_r_first_batch<double, double>(const Batch<UpdateRTask<double, double>>&, hipStream_t);
template void launch_update_r_first_batch<float, double>(const Batch<UpdateRTask<float, double>>&, hipStream_t);
template void launch_update_r_first_batch<float, float>(const Batch<UpdateRTask<float, float>>&, hipStream_t);

void launch_rr_check_batch(const Batch<RrCheckTask>& b, hipStream_t s) {
  k_rr_check_batch<<<b.begin[b.n], kBlock, 0, s>>>(b);
}

template <typename TZ>
void launch_update_px_batch(const Batch<UpdatePxTask<TZ>>& b, hipStream_t s) {
  k_update_px_batch<TZ><<<b.begin[b.n], kBlock, 0, s>>>(b);
}
template void launch_update_px_batch<double>(const Batch<UpdatePxTask<double>>&, hipStream_t);
template void launch_update_px_batch<float>(const Batch<UpdatePxTask<float>>&, hipStream_t);

}  // namespace hexmg
