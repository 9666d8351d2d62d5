// Internal declarations of the hexmg library (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <array>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hexmg.h"

namespace hexmg {

// Host-side element stiffness (element.hip).
void modal_quadratic_form(double nu, double Q[24][24]);
void element_matrix(double nu, double Ke[576]);

// Geometry of one multigrid level as seen by the kernels.
struct Level {
  int nx, ny, nz;     // elements
  int nxn, nyn, nzn;  // nodes
  int nn;             // node count
  int ne;             // element count
  const uint8_t* mask;  // per-node support bits (device)
};

// Haar-basis block coefficients of the unit element (already divided by 64):
// normal block diag-off d1 and off b1, rank-one shear g, bilinear 2x2 (a2, b2),
// bilinear 3x3 diag-off d3 and off b3, trilinear a4.
template <typename T>
struct HaarCoef {
  T d1, b1, g, a2, b2, d3, b3, a4;
};
// Extracts the block coefficients from the modal quadratic form and checks
// that Q has exactly the 14-block pattern; returns false if it does not.
bool haar_coefficients(double nu, HaarCoef<double>* q);

// Streaming-kernel shapes (see stream.hip): number of shapes per precision and
// output rows per workgroup tile of each.
int stream_shapes(bool f32);
int stream_out_rows(bool f32, int shape);

// maskin: u may be non-zero at fixed DOFs (masked on load); otherwise the
// caller guarantees u = 0 there (every vector inside the solver).
// Optional timing of one launch: with both events set, the kernel is launched
// with hipExtLaunchKernelGGL, which stamps the events at the start and the end
// of the dispatch itself (the interval a kernel trace reports).
struct LaunchTimer {
  hipEvent_t start = nullptr, stop = nullptr;
};

template <typename... KArgs, typename... Args>
void launch_timed(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, const LaunchTimer& t,
                  Args... args) {
  if (t.start && t.stop)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t.start, t.stop, 0, static_cast<KArgs>(args)...);
  else
    kernel<<<grid, block, 0, s>>>(static_cast<KArgs>(args)...);
}

// dotp (K u and the sweep, without input masking only; may be null): one
// partial per workgroup of u . (A u) (K u) or of f . y (sweep), per
// right-hand side stream_blocks(...) of them, right-hand side r at
// dotp + r * stream_blocks(...).
template <typename T>
void launch_stream(int mode, bool maskin, int shape, const Level& L, const HaarCoef<T>& q, const T* E, const T* u,
                   const T* f, const T* wd, T* y, int zchunk, int nrhs, const int* act, hipStream_t s,
                   const LaunchTimer& t = {}, double* dotp = nullptr);
// binary64 K u (mode apply, input not masked) of the binary32 u: the
// product on the mixed solver's binary32 search direction; shape is a
// binary64 shape, dotp as for launch_stream
void launch_apply_u32(int shape, const Level& L, const HaarCoef<double>& q, const double* E, const float* u,
                      double* y, int zchunk, int nrhs, const int* act, hipStream_t s, const LaunchTimer& t = {},
                      double* dotp = nullptr);
// adjoint sensitivity dc_e = coef rho_e^pm1 u_e^T K0 u_e (accumulate: added
// to dc) with the element energy in the Haar basis of q
void launch_sensitivity_haar(const Level& L, const HaarCoef<double>& q, const double* rho, const double* u,
                             double coef, double pm1, int accumulate, double* dc, hipStream_t s);
// whether streaming shape `shape` has a kSmoothFirst form (launch_stream and
// launch_stream_batch take that mode only for such shapes, input unmasked, no dotp)
bool first_shape_ok(bool f32, int shape);
// workgroups of one right-hand side's launch of the streaming kernel
int stream_blocks(const Level& L, bool f32, int shape, int zchunk);

// ---------------------------------------------------------------------------
// Launches that cover several grids (hexmg_batch_solve).  A batched launch
// carries a table of tasks (one per grid, each the arguments of that grid's own
// launch) by value in its kernel arguments; workgroup b belongs to the task t
// with begin[t] <= b < begin[t + 1] and does what workgroup b - begin[t] of the
// grid's own launch would do, so every grid's arithmetic is that of its single
// launch.
constexpr int kMaxBatch = 24;
template <typename A>
struct Batch {
  int n = 0;
  int begin[kMaxBatch + 1] = {};
  A a[kMaxBatch];
};
__device__ inline int batch_task(const int* begin, int n, int b) {
  int lo = 0, hi = n - 1;  // largest t with begin[t] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Work order for the eight XCDs, each with its own L2, which take a launch's
// workgroups round-robin by linear id.  For the workgroup with index l in a
// range of T consecutive workgroups whose first has linear id `first`, the
// item of the range it takes: the range is cut into eight contiguous bands and
// XCD c takes band c, so items that read overlapping data run on one L2.  A
// bijection on [0, T): only the order of the items changes.
__device__ inline int xcd_band_index(int l, int T, long long first) {
  const int r0 = (int)(first & 7);  // XCD of the range's first workgroup
  const int c = (r0 + l) & 7;       // XCD of this workgroup
  const int q = T >> 3, rem = T & 7;
  // XCD k takes the range's workgroups l = ((k - r0) & 7) + 8 j: q + 1 of them
  // where (k - r0) & 7 < rem, else q; band c starts after the bands of XCDs
  // 0..c-1
  int start = c * q;
  for (int k = 0; k < c; ++k) start += ((k - r0) & 7) < rem;
  return start + (l >> 3);
}
template <typename T>
struct StreamTask {
  Level L;
  const T* E;
  const T* u;
  const float* u32;  // binary64 K u of a binary32 input (u unused; batches launched with u32in)
  const T* f;
  const T* wd;
  T* y;
  const int* act;
  double* dotp;
  int zchunk, nchunks, gx, gy;
};
// mode, shape and pre (z-chunk of one preloaded plane) and dot (partials of the
// mode's dot product) are common to the batch.
template <typename T>
void launch_stream_batch(int mode, int shape, bool pre, bool dot, const Batch<StreamTask<T>>& b,
                         const HaarCoef<T>& q, hipStream_t s, bool u32in = false);
// the launch grid of one grid's streaming-kernel launch: (gx, gy, nchunks)
void stream_grid(const Level& L, bool f32, int shape, int zchunk, int* gx, int* gy, int* nchunks);

// Tasks of the other batched kernels: the arguments of the single launch and
// gx, the workgroups per right-hand side of that launch (the vector kernels
// always use kReduceBlocks).  Launchers in kernels.hip.
template <typename T>
struct RestrictTask {
  Level F, C;
  const T* r;
  T* fc;
  const int* act;
  const T* wdc;
  T* tc;
  int gx;
};
template <typename T>
struct ProlongTask {
  Level F, C;
  const T* ec;
  T* u;
  const int* act;
  int gx;
};
template <typename T>
struct GemvTask {
  int n;
  const double* Ainv;
  const T* x;
  T* y;
  const int* act;
  int gx;
};
template <typename TW, typename TQ>
struct UpdateRTask {
  long long n;
  const double* pq_partials;
  int npq, parity;
  double* sc;
  const int* active;
  const TQ* q;
  double* r;
  double* rr_partials;
  const TW* wdinv;
  float* f32;
  TW* t;
  const int* repl;
};
struct RrCheckTask {
  const double* rr_partials;
  double* sc;
  int* active;
  double* host_slot;
};
template <typename TZ>
struct UpdatePxTask {
  long long n;
  const double* rz_partials;
  int nrz, parity;
  double* sc;
  const int* active;
  const TZ* z;
  double* p;
  double* x;
  float* p32;
  float* p32b;
};
template <typename T>
void launch_restrict_batch(const Batch<RestrictTask<T>>& b, hipStream_t s);
template <typename T>
void launch_prolong_add_batch(const Batch<ProlongTask<T>>& b, hipStream_t s);
template <typename T>
void launch_coarse_gemv_batch(const Batch<GemvTask<T>>& b, hipStream_t s);
template <typename TW, typename TQ>
void launch_update_r_first_batch(const Batch<UpdateRTask<TW, TQ>>& b, hipStream_t s);
void launch_rr_check_batch(const Batch<RrCheckTask>& b, hipStream_t s);
template <typename TZ>
void launch_update_px_batch(const Batch<UpdatePxTask<TZ>>& b, hipStream_t s);
// the task tables travel in the kernel arguments
static_assert(sizeof(Batch<StreamTask<double>>) <= 4096, "stream task table too large for kernel arguments");
static_assert(sizeof(Batch<RestrictTask<double>>) <= 4096, "restriction task table too large for kernel arguments");
static_assert(sizeof(Batch<UpdateRTask<double, double>>) <= 4096, "update task table too large for kernel arguments");
// workgroups per right-hand side of the single launches
int restrict_blocks(const Level& C);
int prolong_blocks(const Level& F);
int gemv_blocks(int n);
// most partials a fused dot product may leave per right-hand side
constexpr int kMaxDotParts = 8192;  // partials a vector kernel's block sums itself
// out[r] = sum of parts[r * n .. r * n + n) (fixed order; inactive r skipped)
void launch_sum_parts(const double* parts, int n, double* out, int nrhs, const int* act, hipStream_t s);

constexpr int kReduceBlocks = 1024;  // partial sums per reduction (fixed: deterministic)
constexpr int kOcProbes = 32;       // Lagrange multipliers evaluated per OC pass
constexpr int kBlock = 256;
constexpr int kGJBlock = 64;  // pivot block of the blocked Gauss-Jordan inverse

// ---- kernel launchers (kernels.hip) --------------------------------------
// `act` (device, one int per right-hand side, may be null): right-hand sides
// whose flag is 0 are skipped by every kernel that takes it.
template <typename T>
void launch_gather(int mode, const Level& L, const T* Ke, const T* E, const T* u, const T* f,
                   const T* wdinv, T* y, int nrhs, const int* act, hipStream_t s,
                   const LaunchTimer& t = {});
// binary64 y = A u of the binary32 u (node-gather form of launch_apply_u32)
void launch_gather_apply_u32(const Level& L, const double* Ke, const double* E, const float* u, double* y, int nrhs,
                             const int* act, hipStream_t s, const LaunchTimer& t = {});
// mode: 0 y = A u; 1 y = u + wdinv (f - A u); 2 y = f - A u
// element-product modes; kSmoothFirst (streaming kernel only): a Jacobi sweep
// whose input is the first sweep from zero, (omega/D) f, formed on load
enum { kApply = 0, kSmooth = 1, kResidual = 2, kSmoothFirst = 3 };

template <typename T>
void launch_jacobi_first(long long n, const T* wdinv, const T* f, T* u, int nrhs, const int* act, hipStream_t s);
// binary32 first sweep from a binary64 right-hand side: f32 = (float) r, u = wdinv f32
void launch_jacobi_first_from64(long long n, const float* wdinv, const double* r, float* f32, float* u, int nrhs,
                                const int* act, hipStream_t s);
template <typename T>
void launch_restrict(const Level& F, const Level& C, const T* r, T* fc, int nrhs, const int* act, hipStream_t s,
                     const T* wdc = nullptr, T* tc = nullptr);
template <typename T>
void launch_prolong_add(const Level& F, const Level& C, const T* ec, T* u, int nrhs, const int* act, hipStream_t s);

void launch_simp(int ne, const double* rho, double E0, double Emin, double p, double scale,
                 double* E64, float* E32, double* rho_copy, int* bad_flags, hipStream_t s);
void launch_homogenize(const Level& F, const Level& C, const double* vf, double* vc, hipStream_t s);
void launch_modulus_from_density(int ne, const double* rho, double E0, double Emin, double p,
                                 double scale, double* E64, float* E32, hipStream_t s);
void launch_modulus_from_mean(const Level& F, const Level& C, const double* Ef, double scale,
                              double* E64, float* E32, hipStream_t s);
// Coarsest-level moduli from level 0 in one launch (one block per coarsest
// element, blocks of blk^3 fine elements; v0 = densities or fine moduli).
void launch_coarsest_moduli(const Level& F, const Level& C, int blk, const double* v0, bool density, double E0,
                            double Emin, double p, double scale, double* Ec, hipStream_t s);
void launch_diag(const Level& L, const double* Ke, const double* E, double omega, double* wdinv64,
                 float* wdinv32, hipStream_t s);
void launch_mask_default(const Level& L, uint8_t* mask, hipStream_t s);
void launch_mask_inject(const Level& F, const Level& C, const uint8_t* mf, uint8_t* mc, hipStream_t s);
void launch_or_flags(int n, const int* flags, int* out, hipStream_t s);

void launch_coarse_assemble(const Level& C, const double* Ke, const double* E, double* A, hipStream_t s);
template <typename T>
void launch_coarse_gemv(int n, const double* Ainv, const T* x, T* y, int nrhs, const int* act, hipStream_t s);

// BLAS-1 in binary64 with deterministic two-stage reductions.
// All take nrhs vectors stored [nrhs][n]; partials are [nrhs][kReduceBlocks],
// scalars [nrhs][kScalars].
void launch_dot_partial(long long n, const double* x, const double* y, double* partials, int nrhs, const int* act,
                        hipStream_t s);
// out[r * stride] = sum of partials[r][0..kReduceBlocks)
void launch_reduce_final(const double* partials, double* out, int stride, int nrhs, hipStream_t s);
// CG steps with the scalars computed on the device (see ScalarSlot):
// start: r = M f, x = 0, partials of ||r||^2 ([nrhs][kReduceBlocks])
void launch_pcg_start(const Level& L, const double* f, double* r, double* x, double* partials, int nrhs,
                      hipStream_t s);
// init: ff from the start's partials; active = (ff > 0), its = 0, stop = rtol^2 ff (rtol2 <= 0: never)
void launch_pcg_init(double rtol2, const double* ff_partials, double* sc, int* active, int nrhs, hipStream_t s);
// after q = A x: sc[kTmp] = ||M f - q||^2 and sc[kTmp2] = f . x per right-hand
// side (pa, pb: [nrhs][kReduceBlocks] partials)
void launch_pcg_final(const Level& L, const double* f, const double* q, const double* x, double* pa, double* pb,
                      double* sc, int nrhs, hipStream_t s);
// alpha = rz[parity] / (sum of the npq pq partials of a right-hand side, which
// are also npq apart); r -= alpha q; rr partials; the first Jacobi sweep from
// zero t = wdinv * r (mixed: on the binary32 copy f32 of r; t may be null);
// x += alpha p is left to launch_update_px / launch_flush_x (s[kXPend])
// (q in binary64, or the binary32 A p of HEXMG_MIXED32; repl, may be null:
// right-hand sides that get only alpha and s[kXPend], their residual being
// replaced right after)
template <typename TW, typename TQ>
void launch_update_r_first(long long n, const double* pq_partials, int npq, double* sc, const int* active,
                           const TQ* q, double* r, double* rr_partials, int parity, const TW* wdinv, float* f32,
                           TW* t, int nrhs, hipStream_t s, const int* repl = nullptr);
// repl[r] = active[r] and (iterations of r so far + 1) divisible by every
void launch_replace_flags(const double* sc, const int* active, int* repl, int nrhs, int every, hipStream_t s);
// residual replacement after q = A x (binary64, x complete): r = M f - q, rr
// partials, binary32 copy of r and first sweep t (may be null); clears s[kXPend]
void launch_replace_r(const Level& L, const double* f, const double* q, double* r, double* rr_partials,
                      const float* wdinv, float* f32, float* t, double* sc, const int* active, int nrhs,
                      hipStream_t s);
// after the finish of a HEXMG_MIXED32 solve (binary64 residual in s[kTmp]):
// reactivate the right-hand sides whose binary64 residual misses the test
void launch_pcg_restart(double* sc, int* active, int nrhs, int maxit, hipStream_t s);
// rr = sum of partials; its += 1; convergence / breakdown clears active; the
// scalars of every right-hand side are written to host_slot (pinned host memory)
void launch_rr_check(const double* rr_partials, double* sc, int* active, double* host_slot, int nrhs,
                     hipStream_t s);
// rz_new = sum of the nrz rz partials of a right-hand side (nrz apart);
// beta = rz_new / rz[parity]; x += alpha p (the previous iteration's);
// p = z + beta p; rz[1-parity] = rz_new
// (x += alpha p only while s[kXPend]; p32, may be null: binary32 copy of the
// new p).  With p null the direction is binary32 alone, read widened and
// written rounded: the direction of iteration k lives in p32 when k is odd
// and in p32b when k is even, and x is brought up to date only after the even
// iterations, by the two directions then pending (x += alpha_(k-1) p_(k-1),
// then x += alpha_k p_k, the order and rounding of one update per iteration).
template <typename TZ>
void launch_update_px(long long n, const double* rz_partials, int nrz, double* sc, const int* active, const TZ* z,
                      double* p, double* x, int parity, int nrhs, hipStream_t s, float* p32 = nullptr,
                      float* p32b = nullptr);
// x += alpha p for the right-hand sides where it is still due (s[kXPend]);
// with p null, the binary32 directions still pending after the right-hand
// side's last iteration k = s[kIts]: p_k (in p32 for odd k), and for even k
// also p_(k-1), in the order of launch_update_px
void launch_flush_x(long long n, const double* sc, const double* p, double* x, int nrhs, hipStream_t s,
                    const int* act = nullptr, const float* p32 = nullptr, const float* p32b = nullptr);
// partials of r . (double) u32 (the binary32 V-cycle output, not widened in memory)
void launch_dot_mixed(long long n, const float* u32, const double* r, double* partials, int nrhs, const int* act,
                      hipStream_t s);
// z64 = (double) u32 and partials of r . z64
void launch_to64_dot(long long n, const float* u32, const double* r, double* z, double* partials, int nrhs,
                     const int* act, hipStream_t s);
void launch_f64_to_f32(long long n, const double* a, float* b, int nrhs, const int* act, hipStream_t s);

void launch_symmetrize(int n, const double* A, double* B, hipStream_t s);
// Blocked Gauss-Jordan inverse of the n x n SPD matrix in A (B is the
// ping-pong buffer, D 2 kGJBlock^2 scratch for the pivot-block inverses);
// *result receives the buffer holding the inverse.  1 + ceil(n/64) launches.
void launch_gj_blocked(int n, double* A, double* B, double* D, double** result, hipStream_t s);

// Density filter and optimality criteria (topopt.hip)
void launch_filter(int nx, int ny, int nz, double rmin, int adjoint, const double* in, double* out, double* tmp,
                   hipStream_t s);
// Element capacity of the adjoint filter's static scratch (topopt.hip), and
// its address on the current device (0, or a hipError_t value on failure).
constexpr long long kFilterScratchElems = 1ll << 22;
int filter_scratch_ptr(double** ptr);
void launch_sens_filter(int nx, int ny, int nz, double rmin, double gamma, const double* x, const double* dc,
                        double* out, hipStream_t s);
void launch_gravity_load(const Level& L, const double* rho, double g, const double* f_ext, double* f,
                         hipStream_t s);
void launch_gravity_sensitivity(const Level& L, const double* u, double coef, double* dc, hipStream_t s);
void launch_apply_passive(long long n, const uint8_t* passive, double* x, hipStream_t s);
struct OcProbes {
  double v[kOcProbes];  // lambda_p^(-eta)
};
void launch_oc_probe(long long n, const double* x, const double* dc, const double* dv, double eta, double move,
                     const OcProbes& lam_pow, double* partials, double* vol, hipStream_t s);
// x_new at the final multiplier; out[0] = max |x_new - x|, out[1] = dv . x_new
// (partials: 2 kReduceBlocks doubles of scratch)
void launch_oc_apply(long long n, const double* x, const double* dc, const double* dv, double eta, double move,
                     double lam_pow, double* xn, double* partials, double* out, hipStream_t s);
// dv_e = [passive_e == 0] / (number of such elements); count: one int of scratch
void launch_volume_weights(long long n, const uint8_t* passive, int* count, double* dv, hipStream_t s);

// Galerkin coarse operators (galerkin.hip): 27-point block stencils,
// coefficient (9 o + 3 ci + cj) of node n at S[(9 o + 3 ci + cj) * nn + n].
void launch_galerkin_first(const Level& F, const Level& C, const double* E, const double* G, const double* Ke,
                           double* S64, float* S32, hipStream_t s);
void launch_galerkin_coarsen(const Level& F, const Level& C, const double* Sf, double* S64, float* S32,
                             hipStream_t s);
template <typename T>
void launch_stencil(int mode, const Level& L, const T* S, const T* u, const T* f, const T* wd, T* y, int nrhs,
                    const int* act, hipStream_t s, const LaunchTimer& t = {});
// The binary32 stencil sweep with 16-bit coefficients (store = HEXMG_STENCIL_BF16
// or HEXMG_STENCIL_F16; sexp: binary16 rows' scale exponents), and the
// conversion of a binary64 stencil into that storage.
void launch_stencil16(int store, int mode, const Level& L, const uint16_t* S16, const int8_t* sexp, const float* u,
                      const float* f, const float* wd, float* y, int nrhs, const int* act, hipStream_t s,
                      const LaunchTimer& t = {});
void launch_stencil_to16(int store, const Level& L, const double* S64, uint16_t* S16, int8_t* sexp,
                         hipStream_t s);
void launch_stencil_diag(const Level& L, const double* S, double omega, double* wd64, float* wd32, hipStream_t s);
void launch_dense_from_stencil(const Level& C, const double* S, double* A, hipStream_t s);
void galerkin_child_matrices(const double* Ke, double* G);  // host: 8 x 576

// The coarse part of the V-cycle in one cooperative launch (coarse.hip):
// levels, operators and vectors of one precision.  f[ls] holds the restricted
// right-hand side of the first level ls of the launch and t[ls] its first
// Jacobi sweep; the cycle's result lands in u[ls].
constexpr int kMaxLevels = 12;
template <typename T>
struct CoarseCycle {
  Level lv[kMaxLevels];
  const T* E[kMaxLevels];
  const T* wd[kMaxLevels];
  T* u[kMaxLevels];
  T* t[kMaxLevels];
  T* r[kMaxLevels];
  T* f[kMaxLevels];
  const T* Ke;
  const double* Ainv;
  int nc, L, nu;
};
// Most workgroups of k_coarse_cycle<T> that can be resident at once (0 on error).
template <typename T>
int coarse_cycle_max_blocks();
template <typename T>
hipError_t launch_coarse_cycle(const CoarseCycle<T>& a, int ls, int nrhs, const int* act, int blocks,
                               hipStream_t s);

// Device scalar slots used by the PCG (one block of kScalars doubles).
// Per right-hand side, in this order, kScalars doubles each.  The CG state
// lives on the device: the convergence test runs in a kernel, and the host
// only reads copies of these slots.
enum ScalarSlot {
  kRz0 = 0,      // r^T z, double-buffered by iteration parity (kRz0 + parity)
  kRz1 = 1,
  kPq = 2,       // p^T A p of the last iteration
  kRr = 3,       // r^T r of the last iteration
  kAlpha = 4,
  kBeta = 5,
  kFf = 6,       // ||M f||^2
  kStop = 7,     // rtol^2 ||M f||^2 (-1: never)
  kIts = 8,      // iterations taken
  kStatus = 9,   // 1 running / not converged, 0 converged, -5 breakdown, -4 non-finite load
  kActive = 10,  // copy of the device active flag
  kTmp = 11,
  kTmp2 = 12,
  kXPend = 13,   // 1 while the last iteration's x += alpha p has not been applied
  kAlphaP = 14,  // alpha of the last odd iteration (14) and even one (15); 0 after a breakdown
  kScalars = 16
};

}  // namespace hexmg

namespace hexmg {
struct BatchRecorder;  // api.hip
}

// The opaque grid object behind hexmg_grid_t.
struct hexmg_grid {
  hexmg_grid_desc desc;
  int L;
  std::vector<hexmg::Level> lv;
  // per-level device arrays (carved from the caller's workspace)
  std::vector<double*> rho;      // homogenized densities (level 0: copy of the input)
  std::vector<double*> E64;      // element moduli incl. the 2^l size factor
  std::vector<float*> E32;
  std::vector<double*> wd64;     // omega / diag(A_l)
  std::vector<float*> wd32;
  std::vector<uint8_t*> mask;
  // V-cycle vectors per level: f (rhs), u (solution), t (ping-pong), r (residual)
  std::vector<double*> vf64, vu64, vt64, vr64;
  std::vector<float*> vf32, vu32, vt32, vr32;
  double* Abuf[2];  // coarsest operator / Gauss-Jordan ping-pong
  double* gjD;      // 2 kGJBlock^2
  double* Ecoarse;  // coarsest moduli for the coarsest operator (auxiliary stream)
  double* Ainv;     // points at the buffer holding the symmetrized inverse
  int nc;         // coarsest DOFs
  double* Ke64;   // 576
  float* Ke32;
  // Galerkin coarse operators (desc.coarse_op == HEXMG_COARSE_GALERKIN):
  // stencils of levels >= 1 in both precisions, and the 8 child matrices G_c
  bool galerkin = false;
  std::vector<double*> S64;
  std::vector<float*> S32;
  std::vector<uint16_t*> S16;  // 16-bit coefficients (stencil_storage != HEXMG_STENCIL_F32)
  std::vector<int8_t*> Sexp;   // binary16 rows' scale exponents
  double* Gc = nullptr;
  std::vector<double> Gc_host;
  hexmg::HaarCoef<double> hq64;
  hexmg::HaarCoef<float> hq32;
  // element-product kernel per level and precision ([level][0] binary64, [1] binary32)
  struct Choice { int kernel; int zchunk; int shape; };
  // [level][mode]: the element-product kernel per mode (K u, sweep, residual)
  std::vector<std::array<Choice, 3>> choice64, choice32;
  // first level of the cooperative coarse-cycle launch per precision (0: every
  // level launched step by step) and its workgroup count
  int tail64 = 0, tail32 = 0, tail_blocks64 = 0, tail_blocks32 = 0;
  bool tail_tuned = false;
  bool tuned;
  // PCG
  double *r, *z, *p, *q;
  // p: binary64 direction (null with HEXMG_MIXED, whose direction is p32 alone);
  // p32: binary32 direction (HEXMG_MIXED: that of the odd iterations) or
  // binary32 copy of p (HEXMG_MIXED32); p32b: the even iterations' direction
  // (HEXMG_MIXED); q32: binary32 A p of HEXMG_MIXED32
  float *p32, *p32b, *q32;
  double* partials;
  double* partials2;
  double* big_parts = nullptr;  // per-workgroup partials of level-0 launches beyond kMaxDotParts workgroups
  int big_parts_n = 0;          // its capacity per right-hand side
  double* scalars;
  int* flags;     // per-block status flags (kReduceBlocks) + 1 result
  int* active;    // per right-hand side: 1 while its CG iteration runs
  int* repl;      // per right-hand side: 1 where this iteration replaces the residual (HEXMG_MIXED32)
  double* host_ring;  // pinned: 3 slots of kScalars * max_nrhs doubles (results in flight)
  double* oc_partials;  // kReduceBlocks x kOcProbes
  double* oc_vol;       // kOcProbes
  double* host_scalars;  // pinned host mirror
  bool density_set;
  hipStream_t last_stream;
  hipStream_t own_stream = nullptr;  // created on first use by a batched solve
  // The coarsest inverse is formed on aux_stream, concurrently with the rest of
  // hexmg_set_density and the first steps of the next solve; the first use of
  // it on a stream waits for ev_coarse (coarse_waited: the stream that has).
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_coarse = nullptr, ev_flag = nullptr, ev_read = nullptr;
  hipStream_t coarse_waited = nullptr;
  bool coarse_waited_valid = false;  // coarse_waited names a stream (the null stream is one)
  bool coarse_pending = false;
  // profiling
  bool profile;
  // tag: the CG iteration a launch belongs to (0: not part of one); launches of
  // an iteration issued ahead of the convergence test that found nothing left
  // to do are dropped from the counts when the solve ends
  struct Rec { int family; hipEvent_t a, b; int tag; };
  std::vector<Rec> recs;
  int prof_tag = 0;
  // hexmg_batch_solve: while rec is set, this grid's PCG and V-cycle launches
  // are recorded, each with its place in the iteration (stage), and launched
  // later together with the other grids' launches of the same place
  hexmg::BatchRecorder* rec = nullptr;
  int rec_grid = 0;  // this grid's index in the batch
  int stage = 0;     // place of the next recorded element-product launch
  int rec_class = 0; // batched streaming-kernel launches only combine grids of one class (equal K0)
  size_t batch_launches = 0, batch_records = 0;  // of the last batched solve this grid took part in
  std::vector<hipEvent_t> event_pool;
  double prof_ms[8];
  int prof_count[8];
};
