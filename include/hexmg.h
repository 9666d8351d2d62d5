/*
 * hexmg -- matrix-free multigrid-preconditioned CG for the SIMP linear-elastic
 * state equation K(rho) u = f on structured hex8 grids, for AMD gfx950.
 *
 * The library is the black-box state solver of the paper's framework (Sec. 4.2:
 * a solver for K u = f on a Cartesian grid of 8-node bricks, given the grid, the
 * load and the supports), plus the compliance and adjoint sensitivity that feed
 * each optimality-criteria update (Sec. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: nx*ny*nz unit cubes.  Element e = i + nx*(j + ny*k); node
 * n = i + (nx+1)*(j + (ny+1)*k); DOF 3*n + c (c = 0,1,2 for x,y,z).
 * A vector of N = 3*(nx+1)*(ny+1)*(nz+1) entries is contiguous; nrhs vectors are
 * stored back to back ([nrhs][N]).  Local element node a = ax + 2*ay + 4*az.
 *
 * Material: E(rho) = Emin + rho^p (E0 - Emin) (Eq. 2, reading K_min = Emin*K0);
 * the element stiffness is E(rho_e) K0 with K0 the isotropic hex8 stiffness of
 * unit modulus and Poisson ratio nu.
 *
 * Supports: per-node uint8 mask, bit c set = DOF 3n+c fixed (u = 0).  The
 * operator applied everywhere is A = M K M + (I - M), M = diag(free).
 *
 * Memory: all array arguments are DEVICE pointers unless marked "host".  The
 * caller owns every pointer, including the workspace given to
 * hexmg_grid_create; the library never frees caller memory and allocates no
 * device memory of its own (its only device storage is the static scratch
 * array of hexmg_filter_noalloc, 32 MiB per GPU, part of the loaded code).  Calls are asynchronous on the given stream (a
 * hipStream_t passed as void*; NULL = the null stream) except where a host
 * output is written, in which case the call synchronises that stream.
 *
 * Status codes: 0 = OK, 1 = not converged (outputs valid), negative = error;
 * hexmg_last_error() returns a message for the last non-zero status of the
 * calling thread.
 */
#ifndef HEXMG_H
#define HEXMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HEXMG_OK 0
#define HEXMG_NOT_CONVERGED 1
#define HEXMG_ERR_INVALID (-1)
#define HEXMG_ERR_WORKSPACE (-2)
#define HEXMG_ERR_DEVICE (-3)
#define HEXMG_ERR_NONFINITE (-4)
#define HEXMG_ERR_BREAKDOWN (-5)

/* precision of the solver (hexmg_grid_desc.precision) */
#define HEXMG_FP64 0  /* every step in binary64 */
#define HEXMG_MIXED 1 /* V-cycle in binary32; the search direction p stored in binary32; x, r,
                         dots, the outer K p's arithmetic (on p widened) and coarsest solve in
                         binary64 */
#define HEXMG_MIXED32 2 /* V-cycle and the outer K p in binary32 (a binary32 copy of p, binary32 q);
                           CG vectors, dots, coarsest solve and compliance in binary64; the
                           recursive residual is replaced by the binary64 M f - A x every
                           rr_every iterations, and a solve whose recursive residual meets rtol
                           while the binary64 one does not restarts CG from its iterate */

/* element type of vectors passed to hexmg_apply_K / hexmg_vcycle */
#define HEXMG_F64 0
#define HEXMG_F32 1

/* element-product kernel (hexmg_grid_desc.kernel) */
#define HEXMG_KERNEL_STREAM 0 /* z-streaming Haar-basis kernel */
#define HEXMG_KERNEL_GATHER 1 /* node-gather of dense 24x24 element rows */
#define HEXMG_KERNEL_AUTO 2   /* per level and precision, the faster of the two (timed once, default) */

/* coarse-level modulus (hexmg_grid_desc.coarse_avg) */
#define HEXMG_AVG_DENSITY 0 /* coarse rho = mean of the 8 children, then E(rho) (Sec. 4.2.2) */
#define HEXMG_AVG_MODULUS 1 /* coarse E = mean of the 8 children's E */

/* Storage of the Galerkin coarse stencils read by binary32 V-cycles (hexmg_grid_desc.stencil_storage) */
#define HEXMG_STENCIL_F32 0  /* binary32 (default) */
#define HEXMG_STENCIL_BF16 1 /* bfloat16: half the bytes, 8 significand bits, binary32's exponent range */
#define HEXMG_STENCIL_F16 2  /* binary16: half the bytes, 11 significand bits, each node's row scaled by a
                                power of two (kept per node) so that its largest coefficient is in [2^14, 2^15) */

/* Coarse operators */
#define HEXMG_COARSE_REDISCRETIZE 0 /* coarse element stiffness from the homogenized density (Sec. 4.2.2, default) */
#define HEXMG_COARSE_GALERKIN 1     /* A_{l+1} = P^T A_l P with the supports (Eq. 23), stored as 27-point stencils */

typedef struct hexmg_grid *hexmg_grid_t;

typedef struct {
  int nx, ny, nz;       /* elements per axis; each divisible by 2^(levels-1);
                           3 (nx+1)(ny+1)(nz+1) < 2^31, 24 (nx+1)(ny+1) < 2^31,
                           ny + 1 <= 65535 and nz + 1 <= 65535 */
  int levels;           /* multigrid levels, >= 1; level 0 is the given grid */
  double E0, Emin, nu, penal; /* 1, 1e-9, 0.3, 3 in the paper's examples */
  int precision;        /* HEXMG_FP64 | HEXMG_MIXED | HEXMG_MIXED32 */
  int smooth_sweeps;    /* damped-Jacobi sweeps before and after the coarse correction */
  double omega;         /* Jacobi damping, 0 < omega <= 1, or 0 = automatic: 0.6 with
                           re-discretized coarse operators, 0.5 with Galerkin ones */
  int coarse_avg;       /* HEXMG_AVG_DENSITY | HEXMG_AVG_MODULUS */
  int max_nrhs;         /* most right-hand sides per call (sizes the workspace) */
  int kernel;           /* HEXMG_KERNEL_AUTO | HEXMG_KERNEL_STREAM | HEXMG_KERNEL_GATHER */
  const uint8_t *fixed_mask; /* device, (nx+1)(ny+1)(nz+1) bytes; NULL = face x = 0 fixed.
                                Copied at hexmg_grid_create; coarse masks are injected
                                (coarse node fixed iff the coincident fine node is). */
  int coarse_op;        /* HEXMG_COARSE_REDISCRETIZE | HEXMG_COARSE_GALERKIN.  Galerkin levels
                           store 243 coefficients per node in both precisions (about
                           2.9 kB per coarse node) and are applied as stencils; the
                           cooperative coarse-cycle launch is not used with them. */
  int vcycle_both;      /* 0 (default): V-cycle vectors and Jacobi diagonals only in the solver's
                           precision (binary64 for HEXMG_FP64, binary32 otherwise), so
                           hexmg_vcycle accepts only that dtype; 1: both precisions (about
                           twice the V-cycle memory) and hexmg_vcycle accepts either */
  int rr_every;         /* HEXMG_MIXED32 only: replace the recursive residual by the binary64
                           one every rr_every iterations (0 = only when rtol is met) */
  int stencil_storage;  /* HEXMG_COARSE_GALERKIN with a binary32 V-cycle: HEXMG_STENCIL_F32 |
                           HEXMG_STENCIL_BF16 | HEXMG_STENCIL_F16.  The 16-bit forms are rounded
                           from the binary64 stencils (which set-up and binary64 V-cycles use),
                           so the binary32 V-cycle runs with a perturbed but fixed coarse operator */
  int fuse_first;       /* 1 (default): with two or more sweeps and a level-0 streaming sweep kernel
                           of a shape that has the form (hexmg_kernel_choice), the second
                           pre-smoothing sweep of each CG iteration's V-cycle forms the first
                           sweep from zero, (omega/D) r, as it loads its input, so the residual
                           update writes no first-sweep vector; 0: the residual update writes it.
                           The two give bit-identical results. */
} hexmg_grid_desc;

/* Fill *desc with the defaults (E0 1, Emin 1e-9, nu 0.3, penal 3, FP64, 2 sweeps,
 * omega automatic (0), density averaging, max_nrhs 1, automatic kernel choice, fixed face x = 0,
 * re-discretized coarse operators, V-cycle vectors in the solver's precision only,
 * residual replacement every 8 iterations, first sweep formed on load)
 * for the given grid.  Host only. */
int hexmg_default_desc(int nx, int ny, int nz, int levels, hexmg_grid_desc *desc);

/* Bytes of device workspace hexmg_grid_create needs for *desc (host only). */
int hexmg_workspace_size(const hexmg_grid_desc *desc, size_t *bytes);

/* Build a grid object on caller workspace (device, >= hexmg_workspace_size
 * bytes, 256-byte aligned).  The workspace must stay valid until
 * hexmg_grid_destroy.  Errors: -1 bad descriptor, -2 workspace too small. */
int hexmg_grid_create(const hexmg_grid_desc *desc, void *workspace, size_t bytes,
                      void *stream, hexmg_grid_t *out);

/* Release host-side state (the workspace stays the caller's). */
int hexmg_grid_destroy(hexmg_grid_t grid);

/* S1-S3 of the hot path for one density field rho (device, nx*ny*nz doubles,
 * element order): SIMP moduli on every level (Eq. 2; coarse densities by
 * homogenization, Sec. 4.2.2, coarse element of side 2^l has stiffness
 * 2^l E K0), the Jacobi diagonal of every level (Eq. 20), and the exact
 * inverse of the coarsest operator (Alg. 3 solves the coarsest grid directly).
 * rho is copied.  Returns -4 if rho holds a non-finite value or lies outside
 * [0,1] (checked on the device; this call then synchronises the stream). */
int hexmg_set_density(hexmg_grid_t grid, const double *rho, void *stream);

/* y = A_l u on level `level` (0 = finest) with the level's moduli: the
 * matrix-free element-by-element product of Sec. 4.2.1.  dtype HEXMG_F64 or
 * HEXMG_F32 selects the element type of u and y; nrhs vectors.  u and y must
 * not overlap. */
int hexmg_apply_K(hexmg_grid_t grid, int level, int dtype, const void *u, void *y,
                  int nrhs, void *stream);

/* z = V(r): one multigrid V-cycle (Alg. 3) on the finest level from a zero
 * initial guess, damped-Jacobi smoothing (Eq. 21), trilinear prolongation P,
 * restriction P^T, direct coarsest solve.  dtype HEXMG_F64 runs every level in
 * binary64, HEXMG_F32 in binary32 (coarsest solve in binary64 either way).
 * Returns -1 for a dtype whose V-cycle vectors the grid does not hold (see
 * hexmg_grid_desc.vcycle_both). */
int hexmg_vcycle(hexmg_grid_t grid, int dtype, const void *r, void *z, int nrhs,
                 void *stream);

typedef struct {
  int iterations;           /* PCG iterations taken */
  int status;               /* 0 converged, 1 not converged, -5 breakdown */
  double rel_res_recursive; /* ||r_k|| / ||M f|| of the CG recurrence */
  double rel_res_true;      /* ||M f - A u|| / ||M f|| recomputed in binary64 */
  double compliance;        /* f^T u */
  float ms_solve;           /* device time of the solve (stream events) */
} hexmg_solve_info;

/* S10: MGPCG (Alg. 1, preconditioned by hexmg_vcycle in the grid's precision)
 * for A u = M f from u0 = 0, stopping when ||r_k||_2 <= rtol ||M f||_2 or after
 * maxit iterations; rtol <= 0 runs exactly maxit iterations.  f, u: device,
 * [nrhs][N] doubles.  Up to max_nrhs right-hand sides are solved in lockstep
 * (one kernel launch covers all of them; each stops on its own criterion);
 * more are taken in blocks of max_nrhs.  info: host array of nrhs entries (may
 * be NULL).  Synchronises the stream.  Returns 1 if some right-hand side did
 * not converge, -5 on breakdown (p^T A p <= 0).  With HEXMG_MIXED32 the outer
 * product A p runs in binary32 and the recursive residual is replaced by the
 * binary64 one every rr_every iterations; when the recursive residual meets
 * rtol but the binary64 one does not, CG restarts from the current iterate
 * (at most 8 times; iterations keep counting towards maxit). */
int hexmg_solve(hexmg_grid_t grid, const double *f, double *u, int nrhs, double rtol,
                int maxit, hexmg_solve_info *info, void *stream);

/* S15: solve several grids (distinct objects, each after a successful
 * hexmg_set_density) together: grid i solves nrhs[i] <= its max_nrhs
 * right-hand sides f[i] -> u[i] (device, [nrhs[i]][N_i] doubles) exactly as
 * hexmg_solve would (same kernels, same arithmetic, bit for bit).  All grids
 * run on `stream` in lockstep: each PCG step and each V-cycle step (sweep,
 * residual, restriction, coarsest solve, prolongation) of all grids is one
 * kernel launch whose workgroups look up their grid in a task table passed
 * with the launch (grids of different depth share the launches of the levels
 * they have; grids that chose different tile shapes for a level, or whose
 * Poisson ratios differ, take separate launches of that step).  Every kernel
 * covers all right-hand sides of its grid; a converged grid or right-hand side
 * drops out.  The host waits once per iteration for all grids.  infos: host,
 * sum(nrhs) entries in grid order (may be NULL).  Synchronises `stream`.
 * Status as hexmg_solve (worst over the batch). */
int hexmg_batch_solve(hexmg_grid_t *grids, int ngrids, const double *const *f, double *const *u,
                      const int *nrhs, double rtol, int maxit, hexmg_solve_info *infos, void *stream);

/* Diagnostics of the last hexmg_batch_solve the grid took part in: the kernel
 * launches (and runtime calls) it issued for the whole batch, and how many the
 * grids would have issued one by one.  Either pointer may be NULL.  Host only. */
int hexmg_batch_stats(hexmg_grid_t grid, size_t *launches, size_t *recorded);

/* S11-S12: compliance c_r = f_r^T u_r (Eq. 6) per right-hand side into
 * c_host (host, nrhs doubles, may be NULL) and the adjoint sensitivity (Eq. 7,
 * u* = u)  dc_e = -p rho_e^(p-1) (E0 - Emin) sum_r w_r u_{r,e}^T K0 u_{r,e}
 * into dc (device, nx*ny*nz doubles, may be NULL), with weights w (host, nrhs
 * doubles; NULL = all 1).  Uses the density of the last hexmg_set_density. */
int hexmg_compliance_sensitivity(hexmg_grid_t grid, const double *f, const double *u,
                                 int nrhs, const double *weights_host, double *c_host,
                                 double *dc, void *stream);

/* S13: density filter with the weights of Eqs. 4-5, w_ei = max(0, rmin -
 * |c_e - c_i|) over the in-domain elements of an nx*ny*nz grid (element
 * order), 1 < rmin <= 8.  adjoint = 0: out = (H in) / Hs, Hs = H 1;
 * adjoint != 0: out = H (in / Hs), the transpose (tmp: device, nx*ny*nz
 * doubles of scratch, distinct from in and out; unused and may be NULL for
 * the forward filter).  in and out must not overlap.  Asynchronous. */
int hexmg_filter(int nx, int ny, int nz, double rmin, int adjoint, const double *in, double *out,
                 double *tmp, void *stream);

/* The density filter of hexmg_filter for callers that cannot allocate device
 * memory (code under graph capture, serving loops, harnesses that forbid
 * allocation): the adjoint's intermediate in / Hs lives in a static device
 * array of the library (one per GPU, 2^22 doubles = 32 MiB, held until the
 * process ends) instead of a caller buffer, and the call allocates nothing.
 * Same arguments and results as hexmg_filter without tmp; the adjoint returns
 * -1 for more than 2^22 elements (the forward filter needs no scratch and has
 * hexmg_filter's limits).  Every adjoint call on a GPU shares that GPU's
 * array, so adjoint calls that overlap on one GPU (different streams or host
 * threads without ordering) race.  Asynchronous. */
int hexmg_filter_noalloc(int nx, int ny, int nz, double rmin, int adjoint, const double *in, double *out,
                         void *stream);

/* Sensitivity filter (Eq. 3) with the same weights:
 *   out_e = (sum_i w_ei x_i dc_i) / (max(gamma, x_e) sum_i w_ei),
 * 0 < rmin <= 8, gamma > 0 (the paper's small constant against division by
 * zero; 1e-3 is usual).  x, dc, out: device, nx*ny*nz doubles in element
 * order; out must not overlap x or dc.  Asynchronous. */
int hexmg_sensitivity_filter(int nx, int ny, int nz, double rmin, double gamma, const double *x,
                             const double *dc, double *out, void *stream);

/* Self-weight of the design, the design-dependent gravity loading of the
 * paper's foot-bridge example (Sec. 5): f = f_ext + f_g(rho) with, for every
 * element of unit volume and unit mass density, the body force -gz rho_e
 * along z shared equally by its eight nodes (the consistent load of the
 * trilinear element).  rho is the density of the last hexmg_set_density.
 * f_ext: device, N doubles, or NULL (zero); f: device, N doubles, not
 * overlapping f_ext.  Asynchronous. */
int hexmg_gravity_load(hexmg_grid_t grid, double gz, const double *f_ext, double *f, void *stream);

/* Load part of the compliance derivative when f depends on the design:
 * dc/drho_e = 2 u^T df/drho_e - u^T dK/drho_e u.  Adds
 * weight * 2 * (-gz / 8) * (sum of u_z over the element's nodes) to dc
 * (device, nx*ny*nz doubles; accumulates, so call it after
 * hexmg_compliance_sensitivity).  u: device, N doubles.  Asynchronous. */
int hexmg_gravity_sensitivity(hexmg_grid_t grid, const double *u, double gz, double weight, double *dc,
                              void *stream);

/* Passive regions (the paper's bridge examples): passive[e] = 1 sets x_e = 1
 * (solid), 2 sets x_e = 0 (void), 0 leaves it (design).  n elements; passive,
 * x: device.  Elements whose dv is 0 in hexmg_oc_update stay outside the
 * volume constraint and keep their value, so passive elements are given
 * dv = 0 there and this is applied to the result.  Asynchronous. */
int hexmg_apply_passive(long long n, const uint8_t *passive, double *x, void *stream);

/* S14: one optimality-criteria update (Eqs. 8-9) on the grid's elements:
 * x_new = clamp(x B^eta, max(0, x - move), min(1, x + move)),
 * B = -dc / (lambda dv), with lambda found by bisection in log space on
 * [1e-12, 1e12] (to a relative width of 1e-12) so that dv^T x_new = volfrac,
 * where dv = dV/dx (for the filtered volume V = mean(rho~) that is
 * H (1/(Ne Hs)), so dv^T x is exactly the filtered volume).  x, dc, dv:
 * device, Ne doubles (dc <= 0, dv >= 0; an element with dv = 0 is outside the
 * volume constraint and keeps its x, e.g. a passive one); x_new: device, Ne
 * doubles, distinct from the inputs.  lambda_host (host, may be NULL)
 * receives lambda, change_host (host, may be NULL) the largest |x_new - x|
 * (the change that Alg. 4's stop test reads) and volume_host (host, may be
 * NULL) dv^T x_new, the constrained volume of the new design.
 * Synchronises the stream once per bisection pass (32 multipliers per pass),
 * and once more when change_host or volume_host is given. */
int hexmg_oc_update(hexmg_grid_t grid, const double *x, const double *dc, const double *dv, double volfrac,
                    double move, double eta, double *x_new, double *lambda_host, double *change_host,
                    double *volume_host, void *stream);

/* Derivative of the volume of the design elements for the OC update when the
 * sensitivity filter is used (the volume is the mean of x over the elements
 * that are not passive): dv_e = 1 / (number of elements with passive_e == 0)
 * for those, 0 for passive ones (which hexmg_oc_update then leaves alone).
 * passive: device, nx*ny*nz bytes (0 design, 1 solid, 2 void); dv: device,
 * nx*ny*nz doubles.  Asynchronous. */
int hexmg_volume_weights(hexmg_grid_t grid, const uint8_t *passive, double *dv, void *stream);

/* The library's unit element stiffness K0 (24x24, row-major, local DOF 3a+c)
 * for Poisson ratio nu, written to Ke_host.  Host only; needs no GPU. */
int hexmg_element_matrix(double nu, double *Ke_host);

/* The element-product kernel of `level` for dtype (HEXMG_F64/F32) in mode
 * (0 K u, 1 damped-Jacobi sweep, 2 residual): *kernel = HEXMG_KERNEL_STREAM
 * or HEXMG_KERNEL_GATHER and,
 * for the streaming kernel, the planes per z-chunk and the tile shape index
 * (rows per thread / waves per workgroup; any output pointer may be NULL).
 * With HEXMG_KERNEL_AUTO the choice is made by timing the candidates
 * (node-gather; every streaming shape with 1..64 planes per chunk -- a chunk
 * of one plane requests all its inputs before any arithmetic) on the
 * grid's stream during the first successful hexmg_set_density, separately
 * for K u, the sweep and the residual. */
int hexmg_kernel_choice(hexmg_grid_t grid, int level, int dtype, int mode, int *kernel, int *zchunk, int *shape);

/* Overrides the element-product kernel of `level` for dtype (all three
 * modes): kernel
 * HEXMG_KERNEL_STREAM (zchunk >= 1 planes per chunk, shape 0 .. number of
 * shapes - 1) or HEXMG_KERNEL_GATHER.  Later automatic tuning does not undo it.
 * Returns -1 for an unknown kernel, shape or level, and for a z-chunk so small
 * that ceil((nz_level + 1) / zchunk) * max_nrhs exceeds 65535 (the launch
 * grid's z limit). */
int hexmg_set_kernel_choice(hexmg_grid_t grid, int level, int dtype, int kernel, int zchunk, int shape);

/* The coarse part of the V-cycle (Alg. 3) may run as one cooperative launch
 * (a grid-stride kernel whose phases -- sweeps, residual, restriction,
 * coarsest solve, prolongation -- are separated by grid-wide barriers) instead
 * of one launch per step; the arithmetic is that of the node-gather kernels.
 * *level = first level of that launch (1 .. levels-2) or 0 when every level is
 * launched step by step; *blocks = its workgroup count.  By default the choice
 * is made by timing both forms on the grid's stream during the first
 * successful hexmg_set_density.  Either output pointer may be NULL.
 * The cooperative launch needs its workgroups resident together; a grid used
 * concurrently with another grid's solve on a different stream should be set
 * to 0 (hexmg_batch_solve does this itself for the duration of the call). */
int hexmg_coarse_cycle_choice(hexmg_grid_t grid, int dtype, int *level, int *blocks);

/* Overrides that choice for dtype: level 0 (off) or 1 .. levels-2; blocks 0 =
 * as many workgroups as can be resident at once (larger values are clamped to
 * that).  Later automatic tuning does not undo it.  Returns -1 for a bad level,
 * -3 if the device cannot launch the kernel cooperatively. */
int hexmg_set_coarse_cycle(hexmg_grid_t grid, int dtype, int level, int blocks);

/* Per-kernel device timing with stream events (off by default).  While
 * enabled, every finest-level launch of the named kernel family is bracketed
 * by events on its stream; hexmg_profile_query returns the number of launches and their
 * total milliseconds since the last reset (synchronises the grid's last
 * stream).  Families: "apply_f64", "apply_f32", "smooth_f64", "smooth_f32",
 * "residual_f64", "residual_f32". */
int hexmg_profile_enable(hexmg_grid_t grid, int enable);
int hexmg_profile_query(hexmg_grid_t grid, const char *family, int *launches, double *ms);

/* Message for the calling thread's last non-zero status ("" if none). */
const char *hexmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HEXMG_H */
