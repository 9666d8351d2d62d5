// Internal declarations of the hexmg library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

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

template <typename T>
void launch_stream(int mode, int shape, const Level& L, const HaarCoef<T>& q, const T* E, const T* u, const T* f,
                   const T* wd, T* y, int zchunk, int nrhs, hipStream_t s);

constexpr int kReduceBlocks = 512;  // partial sums per reduction (fixed: deterministic)
constexpr int kOcProbes = 32;       // Lagrange multipliers evaluated per OC pass
constexpr int kBlock = 256;
constexpr int kGJBlock = 64;  // pivot block of the blocked Gauss-Jordan inverse

// ---- kernel launchers (kernels.hip) --------------------------------------
template <typename T>
void launch_gather(int mode, const Level& L, const T* Ke, const T* E, const T* u, const T* f,
                   const T* wdinv, T* y, int nrhs, hipStream_t s);
// mode: 0 y = A u; 1 y = u + wdinv (f - A u); 2 y = f - A u
enum { kApply = 0, kSmooth = 1, kResidual = 2 };

template <typename T>
void launch_jacobi_first(long long n, const T* wdinv, const T* f, T* u, int nrhs, hipStream_t s);
template <typename T>
void launch_restrict(const Level& F, const Level& C, const T* r, T* fc, int nrhs, hipStream_t s);
template <typename T>
void launch_prolong_add(const Level& F, const Level& C, const T* ec, T* u, int nrhs, hipStream_t s);

void launch_simp(int ne, const double* rho, double E0, double Emin, double p, double scale,
                 double* E64, float* E32, double* rho_copy, int* bad_flags, hipStream_t s);
void launch_homogenize(const Level& F, const Level& C, const double* vf, double* vc, hipStream_t s);
void launch_modulus_from_density(int ne, const double* rho, double E0, double Emin, double p,
                                 double scale, double* E64, float* E32, hipStream_t s);
void launch_modulus_from_mean(const Level& F, const Level& C, const double* Ef, double scale,
                              double* E64, float* E32, hipStream_t s);
void launch_diag(const Level& L, const double* Ke, const double* E, double omega, double* wdinv64,
                 float* wdinv32, hipStream_t s);
void launch_mask_default(const Level& L, uint8_t* mask, hipStream_t s);
void launch_mask_inject(const Level& F, const Level& C, const uint8_t* mf, uint8_t* mc, hipStream_t s);
void launch_or_flags(int n, const int* flags, int* out, hipStream_t s);

void launch_coarse_assemble(const Level& C, const double* Ke, const double* E, double* A, hipStream_t s);
template <typename T>
void launch_coarse_gemv(int n, const double* Ainv, const T* x, T* y, int nrhs, hipStream_t s);

// BLAS-1 in binary64 with deterministic two-stage reductions.
// All take nrhs vectors stored [nrhs][n]; partials are [nrhs][kReduceBlocks],
// scalars [nrhs][kScalars].
void launch_dot_partial(long long n, const double* x, const double* y, double* partials, int nrhs, hipStream_t s);
// out[r * stride] = sum of partials[r][0..kReduceBlocks)
void launch_reduce_final(const double* partials, double* out, int stride, int nrhs, hipStream_t s);
void launch_scalar_op(int op, double* sc, int nrhs, hipStream_t s);
void launch_update_xr(long long n, const double* sc, const int* active, const double* p, const double* q, double* x,
                      double* r, double* partials, int nrhs, hipStream_t s);
void launch_update_p(long long n, const double* sc, const int* active, const double* z, double* p, int nrhs,
                     hipStream_t s);
void launch_mask_copy(const Level& L, const double* f, double* r, int nrhs, hipStream_t s);
void launch_f64_to_f32(long long n, const double* a, float* b, hipStream_t s);
void launch_f32_to_f64(long long n, const float* a, double* b, hipStream_t s);
void launch_sub(long long n, const double* a, const double* b, double* c, hipStream_t s);
void launch_fill(long long n, double v, double* x, hipStream_t s);

void launch_sensitivity(const Level& L, const double* Ke, const double* rho, const double* u,
                        double coef, double pm1, int accumulate, double* dc, hipStream_t s);
void launch_symmetrize(int n, const double* A, double* B, hipStream_t s);
// In-place-style blocked Gauss-Jordan inverse of the n x n SPD matrix in A
// (B is the ping-pong buffer, D kGJBlock^2 and X kGJBlock*n scratch); *result
// receives the buffer holding the inverse.
void launch_gj_blocked(int n, double* A, double* B, double* D, double* X, double** result, hipStream_t s);

// Density filter and optimality criteria (topopt.hip)
void launch_filter(int nx, int ny, int nz, double rmin, int adjoint, const double* in, double* out, double* tmp,
                   hipStream_t s);
struct OcProbes {
  double v[kOcProbes];  // lambda_p^(-eta)
};
void launch_oc_probe(long long n, const double* x, const double* dc, const double* dv, double eta, double move,
                     const OcProbes& lam_pow, double* partials, double* vol, hipStream_t s);
void launch_oc_apply(long long n, const double* x, const double* dc, const double* dv, double eta, double move,
                     double lam_pow, double* xn, hipStream_t s);

// Device scalar slots used by the PCG (one block of kScalars doubles).
enum ScalarSlot {
  kRz = 0,      // r^T z (current)
  kPq = 1,      // p^T A p
  kRr = 2,      // r^T r
  kAlpha = 3,
  kBeta = 4,
  kRzNew = 5,
  kFf = 6,      // ||M f||^2
  kTmp = 7,
  kScalars = 8
};
enum ScalarOp { kOpAlpha = 0, kOpBeta = 1 };

}  // namespace hexmg

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
  double* gjD;      // kGJBlock^2
  double* gjX;      // kGJBlock * n_c
  double* Ainv;     // points at the buffer holding the symmetrized inverse
  int nc;         // coarsest DOFs
  double* Ke64;   // 576
  float* Ke32;
  hexmg::HaarCoef<double> hq64;
  hexmg::HaarCoef<float> hq32;
  // element-product kernel per level and precision ([level][0] binary64, [1] binary32)
  struct Choice { int kernel; int zchunk; int shape; };
  std::vector<Choice> choice64, choice32;
  bool tuned;
  // PCG
  double *r, *z, *p, *q;
  double* partials;
  double* scalars;
  int* flags;     // per-block status flags (kReduceBlocks) + 1 result
  int* active;    // per right-hand side: 1 while its CG iteration runs
  int* host_active;  // pinned mirror
  double* oc_partials;  // kReduceBlocks x kOcProbes
  double* oc_vol;       // kOcProbes
  double* host_scalars;  // pinned host mirror
  bool density_set;
  hipStream_t last_stream;
  hipStream_t own_stream = nullptr;  // created on first use by a batched solve
  // profiling
  bool profile;
  struct Rec { int family; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  double prof_ms[8];
  int prof_count[8];
};
