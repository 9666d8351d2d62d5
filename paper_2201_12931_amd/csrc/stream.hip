// z-streaming matrix-free K u in the Haar basis of the hex8 element (Sec. 4.2.1
// "local stiffness" products, re-organised for gfx950).
//
// Change of basis.  On every axis the two nodal values (v0, v1) of a trilinear
// field become the sum s = v1 + v0 and the difference d = v1 - v0.  In this
// basis the unit element stiffness is block diagonal,
//     K0 = H^T Q H / 64,   Q: 45 non-zeros in 14 blocks (8 distinct values),
// where H is the 8x8 tensor product of the per-axis [[1,1],[-1,1]] maps.
// The sums and differences are shared between neighbouring elements: the
// x-stage (per node) is shared by the 4 elements around an x-edge, the y-stage
// (per xy-face) by the 2 elements above and below it, and so are their
// adjoints (the two elements' contributions to a face are summed in the face's
// modes before the y and x adjoints); only the z-stage, the block product and
// the z adjoint are per element.  This takes K u from 576 FMA per node (dense
// 24x24 rows) to about 150 VALU operations per node.
//
// Mapping.  A wave owns 64 consecutive node columns in x (lane = column) and R
// consecutive node rows in y (held in registers); a workgroup stacks W waves in
// y; all threads march along z through a chunk of planes.  x-neighbours are
// exchanged with DPP wavefront shifts, y-neighbours inside a wave live in the
// same thread, and the only cross-wave dependency (the adjoint contribution of
// a wave's last face row to the next wave's first node row) goes through LDS,
// double-buffered by plane parity, with one barrier per plane.  Each tile reads
// a one-node halo on every side and writes the nodes whose elements it holds
// on both sides: 62 columns x (W*R-1) rows x its z-chunk.  Every output is
// written exactly once: no atomics.
//
// Out-of-domain nodes read as 0 and out-of-domain elements have modulus 0, so
// the boundary needs no special case.  Fixed DOFs read as 0 and return u.
#include "hexmg_impl.h"

namespace hexmg {

namespace {

// Value held by lane+1 (lane 63 receives 0) / lane-1 (lane 0 receives 0).
__device__ inline float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ inline float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ inline double lane_next(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), 0x130, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x130, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline double lane_prev(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), 0x138, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x138, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// t = E Q v for one element.  Modal index m: bit 0 = x difference, bit 1 = y,
// bit 2 = z; m = 0 (rigid translation) has no stiffness.  Coefficients carry
// the 1/64 of K0 = H^T Q H / 64.
template <typename T>
__device__ inline void block_product(const HaarCoef<T>& q, T E, const T (&v)[8][3], T (&t)[8][3]) {
  const T d1 = q.d1 * E, b1 = q.b1 * E, g = q.g * E, a2 = q.a2 * E, b2 = q.b2 * E;
  const T d3 = q.d3 * E, b3 = q.b3 * E, a4 = q.a4 * E;
  {  // normal strains: (1,x) (2,y) (4,z)
    const T s = b1 * (v[1][0] + v[2][1] + v[4][2]);
    t[1][0] = d1 * v[1][0] + s;
    t[2][1] = d1 * v[2][1] + s;
    t[4][2] = d1 * v[4][2] + s;
  }
  {  // shears, rank one
    const T s = g * (v[1][1] + v[2][0]);
    t[1][1] = s;
    t[2][0] = s;
  }
  {
    const T s = g * (v[1][2] + v[4][0]);
    t[1][2] = s;
    t[4][0] = s;
  }
  {
    const T s = g * (v[2][2] + v[4][1]);
    t[2][2] = s;
    t[4][1] = s;
  }
  // bilinear 2x2 blocks
  t[3][0] = a2 * v[3][0] + b2 * v[6][2];
  t[6][2] = b2 * v[3][0] + a2 * v[6][2];
  t[3][1] = a2 * v[3][1] + b2 * v[5][2];
  t[5][2] = b2 * v[3][1] + a2 * v[5][2];
  t[5][0] = a2 * v[5][0] + b2 * v[6][1];
  t[6][1] = b2 * v[5][0] + a2 * v[6][1];
  {  // bilinear 3x3 block
    const T s = b3 * (v[3][2] + v[5][1] + v[6][0]);
    t[3][2] = d3 * v[3][2] + s;
    t[5][1] = d3 * v[5][1] + s;
    t[6][0] = d3 * v[6][0] + s;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) t[7][c] = a4 * v[7][c];
#pragma unroll
  for (int c = 0; c < 3; ++c) t[0][c] = T(0);
}

// Adjoint sensitivity (Eq. 7 with the self-adjoint u* = u), one thread per
// element: dc_e = coef rho_e^(p-1) u_e^T K0 u_e, with the element energy
// formed in the Haar basis, u_e^T K0 u_e = v^T (Q / 64) v, v = H u_e (about 150
// operations instead of 576 multiply-adds on a dense K0).  coef = -p (E0 -
// Emin) times the load-case weight; with accumulate the result is added to dc.
__global__ __launch_bounds__(256) void k_sensitivity_haar(Level L, HaarCoef<double> q,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ u, double coef, double pm1,
                                                           int accumulate, double* __restrict__ dc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= L.ne) return;
  const int i = e % L.nx, t = e / L.nx, j = t % L.ny, k = t / L.ny;
  double v[8][3];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const long long m = (i + (b & 1)) + (long long)L.nxn * ((j + ((b >> 1) & 1)) + (long long)L.nyn * (k + (b >> 2)));
#pragma unroll
    for (int c = 0; c < 3; ++c) v[b][c] = u[3 * m + c];
  }
  // per axis a: the pair (lo, hi) across bit a becomes (hi + lo, hi - lo)
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
      if (!(b & (1 << a))) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double lo = v[b][c], hi = v[b | (1 << a)][c];
          v[b][c] = hi + lo;
          v[b | (1 << a)][c] = hi - lo;
        }
      }
  double tq[8][3];
  block_product<double>(q, 1.0, v, tq);
  double en = 0.0;
#pragma unroll
  for (int m = 1; m < 8; ++m)
#pragma unroll
    for (int c = 0; c < 3; ++c) en += v[m][c] * tq[m][c];
  const double r = rho[e];
  const double w = pm1 == 2.0 ? r * r : pow(r, pm1);
  const double val = coef * w * en;
  dc[e] = accumulate ? dc[e] + val : val;
}

// Buffer-resource access.  Every load and store of the kernel goes through a
// raw buffer resource that spans one z-plane of one array; the per-lane byte
// offset inside the plane is fixed for the whole z-march and only the plane
// base (a uniform value) moves.  An offset at or past the resource's size reads
// as 0 and drops the store, which is how nodes and elements outside the domain
// (or outside the tile's output window) are handled: kOutside is such an
// offset for every resource, and a resource of size 0 disables a whole plane.
constexpr int kRsrcWord3 = 0x00020000;      // raw buffer, 32-bit dwords
constexpr int kOutside = (int)0x80000000;   // planes are < 2 GiB
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
typedef unsigned u32x3 __attribute__((__vector_size__(3 * sizeof(unsigned))));

__device__ inline Rsrc plane_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, kRsrcWord3);
}
__device__ inline void load3(Rsrc r, int off, float (&v)[3]) {
  const u32x3 x = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
  v[0] = __uint_as_float(x[0]);
  v[1] = __uint_as_float(x[1]);
  v[2] = __uint_as_float(x[2]);
}
__device__ inline void load3(Rsrc r, int off, double (&v)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off + 8 * c, 0, 0);
    v[c] = __longlong_as_double((long long)(((unsigned long long)x[1] << 32) | x[0]));
  }
}
__device__ inline float load1(Rsrc r, int off, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline double load1(Rsrc r, int off, double) {
  const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return __longlong_as_double((long long)(((unsigned long long)x[1] << 32) | x[0]));
}
__device__ inline void store3(Rsrc r, int off, const float (&v)[3]) {
  const u32x3 x = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2])};
  __builtin_amdgcn_raw_buffer_store_b96(x, r, off, 0, 0);
}
__device__ inline void store3(Rsrc r, int off, const double (&v)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v[c]);
    const u32x2 x = {(unsigned)(b & 0xffffffffull), (unsigned)(b >> 32)};
    __builtin_amdgcn_raw_buffer_store_b64(x, r, off + 8 * c, 0, 0);
  }
}

// bit c of m set ? a : b, as a bit-field select.
__device__ inline float select_bit(int m, int c, float a, float b) {
  const int sel = (m << (31 - c)) >> 31;
  return __int_as_float((sel & __float_as_int(a)) | (~sel & __float_as_int(b)));
}
__device__ inline double select_bit(int m, int c, double a, double b) { return ((m >> c) & 1) ? a : b; }

// MASKIN: the input u may be non-zero at fixed DOFs (public K u and V-cycle
// entry) and is masked on load; without it (every vector inside the solver is
// zero there) only the outputs use the support bits.
// PRE > 0: zchunk is PRE and all inputs of the workgroup are requested up front.
// DOT (K u and the sweep, without MASKIN): also one partial per workgroup
// into dotp, of u . (A u) for K u and of f . y (the right-hand side times the
// new iterate) for the sweep.
// TU: the type u is stored in (T, or binary32 widened on load for the
// binary64 product on a binary32 search direction).
// One workgroup's tile: (bx, by, bz) is its place in the grid's launch of
// gx * gy * (nchunks * nrhs) workgroups (the launch grid itself, or its slot
// in a batched launch over several grids).
template <typename T, int MODE, int R, int W, bool MASKIN, int PRE, bool DOT, typename TU = T>
__device__ __forceinline__ void stream_tile(const Level& L, const HaarCoef<T>& q, const T* __restrict__ Eg,
                                            const TU* __restrict__ ug, const T* __restrict__ fg,
                                            const T* __restrict__ wg, T* __restrict__ yg, int zchunk, int nchunks,
                                            const int* __restrict__ act, double* __restrict__ dotp, int bx, int by,
                                            int bz, int gx, int gy) {
  if (act && !act[bz / nchunks]) return;  // right-hand side already converged (uniform per block)
  // kSmoothFirst: a sweep whose input is the first sweep from zero, u = (omega/D) f,
  // formed on load from f and omega/D instead of read (ug unused)
  constexpr bool FIRST = MODE == kSmoothFirst;
  {  // bz = z-chunk + nchunks * right-hand side; vectors are [nrhs][3 nn]
    const long long off = 3ll * L.nn * (bz / nchunks);
    ug += off;
    yg += off;
    if (MODE != kApply) fg += off;
  }
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  constexpr int kOutRows = W * R - 1;
  const int i = bx * 62 - 1 + lane;           // node column of this lane
  const int jt0 = by * kOutRows - 1;          // first (halo) row of the tile
  const int j0 = jt0 + w * R;                         // first row of this wave
  const int kc0 = (bz % nchunks) * zchunk;
  const int kc1 = min(kc0 + zchunk, L.nzn);           // output planes [kc0, kc1)
  const bool lane_out = lane >= 1 && lane <= 62 && i < L.nxn;
  const bool col_in = i >= 0 && i < L.nxn;
  const bool col_elem = i >= 0 && i < L.nx;
  const long long plane = (long long)L.nxn * L.nyn;
  const long long eplane = (long long)L.nx * L.ny;
  const int vbytes = (int)(3 * plane * (long long)sizeof(T));   // one plane of a nodal vector
  const int ubytes = (int)(3 * plane * (long long)sizeof(TU));  // one plane of u
  const int ebytes = (int)(eplane * (long long)sizeof(T));      // one layer of moduli
  const int mbytes = (int)plane;                                 // one plane of support bits

  // Row r of this wave is node row j0 + r; rows 0..R are read, rows 0..R-1 own
  // element rows and (when inside the tile's output window) output rows.
  // Byte offsets inside a plane; kOutside where the row is not read / written.
  int offu[R + 1], offm[R + 1], offe[R], offo[R], offmo[R];
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    const int jr = j0 + r;
    const int n = i + L.nxn * jr;
    const bool in = col_in && jr >= 0 && jr < L.nyn;
    offu[r] = in ? n * (3 * (int)sizeof(TU)) : kOutside;
    offm[r] = in ? n : kOutside;
    if (r < R) {
      offe[r] = (col_elem && jr >= 0 && jr < L.ny) ? (i + L.nx * jr) * (int)sizeof(T) : kOutside;
      const int rt = w * R + r;
      const bool out = lane_out && rt >= 1 && rt <= kOutRows && jr < L.nyn;
      offo[r] = out ? n * (3 * (int)sizeof(T)) : kOutside;
      offmo[r] = out ? n : kOutside;
    }
  }

  // Software pipeline: the raw u (and, with MASKIN, the support bits) of plane
  // kk+1 and the moduli of element layer kk are requested while plane kk is
  // being processed.
  // Plane buffers alternate by parity (A holds the planes kc0-1, kc0+1, ...,
  // B the others), so the pipeline never copies a plane between registers.
  TU uA[R + 1][3], uB[R + 1][3];
  T wA[FIRST ? R + 1 : 1][3], wB[FIRST ? R + 1 : 1][3];  // omega/D of the input planes (FIRST)
  T uo[R][3];
  int mA[R + 1], mB[R + 1];
  T EA[R], EB[R];
  __shared__ T xch[2][W][3][64];  // [parity][wave][xyz][lane]: node values for the next wave
  // Only planes kc0-1..kc1 and element layers kc0-1..kc1-1 are needed; the
  // pipeline's requests outside them are given empty resources (no traffic).
  auto load_plane = [&](int kk, TU (&u)[R + 1][3], T (&wv)[FIRST ? R + 1 : 1][3], int (&m)[R + 1]) {
    const bool pin = kk >= 0 && kk < L.nzn && kk <= kc1;
    if constexpr (FIRST) {
      const Rsrc ru = plane_rsrc(fg + 3 * plane * (pin ? kk : 0), pin ? vbytes : 0);
      const Rsrc rw = plane_rsrc(wg + 3 * plane * (pin ? kk : 0), pin ? vbytes : 0);
#pragma unroll
      for (int r = 0; r <= R; ++r) {
        load3(ru, offu[r], u[r]);
        load3(rw, offu[r], wv[r]);
      }
    } else {
      const Rsrc ru = plane_rsrc(ug + 3 * plane * (pin ? kk : 0), pin ? ubytes : 0);
#pragma unroll
      for (int r = 0; r <= R; ++r) load3(ru, offu[r], u[r]);
    }
    if (MASKIN) {
      const Rsrc rm = plane_rsrc(L.mask + plane * (pin ? kk : 0), pin ? mbytes : 0);
#pragma unroll
      for (int r = 0; r <= R; ++r) m[r] = __builtin_amdgcn_raw_buffer_load_b8(rm, offm[r], 0, 0);
    }
  };
  auto load_layer = [&](int ke, T (&E)[R]) {
    const bool lin = ke >= 0 && ke < L.nz && ke >= kc0 - 1 && ke < kc1;
    const Rsrc re = plane_rsrc(Eg + eplane * (lin ? ke : 0), lin ? ebytes : 0);
#pragma unroll
    for (int r = 0; r < R; ++r) E[r] = load1(re, offe[r], T(0));
  };

  // Face modes of the previous plane (forward transform) and top-face modes of
  // the previous element layer (adjoint), also alternating by parity: an
  // iteration reads one set and writes the other, which the next iteration
  // reads (an in-place update would cost a register move per mode).
  T FpA[R][4][3], FpB[R][4][3];
  T TpA[R][4][3], TpB[R][4][3];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uo[r][c] = T(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        FpA[r][m][c] = T(0);
        FpB[r][m][c] = T(0);
        TpA[r][m][c] = T(0);
        TpB[r][m][c] = T(0);
      }
    }
  }
  // With DOT: this thread's share of the dot product over its outputs.
  double dot = 0.0;

  // Inputs of the epilogue of iteration kk (output plane kk-1): support bits,
  // f and omega/D.
  auto load_out = [&](int kk, int (&mo)[R], T (&fo)[R][3], T (&wo)[R][3]) {
    const bool out_plane = kk - 1 >= kc0 && kk - 1 < kc1;
    const long long po = plane * (out_plane ? kk - 1 : 0);
    {
      const Rsrc rm = plane_rsrc(L.mask + po, out_plane ? mbytes : 0);
#pragma unroll
      for (int r = 0; r < R; ++r) mo[r] = __builtin_amdgcn_raw_buffer_load_b8(rm, offmo[r], 0, 0);
    }
    if (MODE != kApply) {
      const Rsrc rf = plane_rsrc(fg + 3 * po, out_plane ? vbytes : 0);
#pragma unroll
      for (int r = 0; r < R; ++r) load3(rf, offo[r], fo[r]);
    }
    if (MODE == kSmooth || FIRST) {
      const Rsrc rw = plane_rsrc(wg + 3 * po, out_plane ? vbytes : 0);
#pragma unroll
      for (int r = 0; r < R; ++r) load3(rw, offo[r], wo[r]);
    }
  };

  // Iteration kk: x and y stages of plane kk; for kk >= kc0 also element layer
  // kk-1 and the output of plane kk-1.
  // Fin/Tin: the previous plane's face modes and the previous layer's top-face
  // modes; Fout/Tout receive this plane's and this layer's.
  auto body = [&](int kk, const TU (&uc)[R + 1][3], const T (&wc)[FIRST ? R + 1 : 1][3], const int (&mc)[R + 1],
                  const T (&Ec)[R], const int (&mo)[R],
                  const T (&fo)[R][3], const T (&wo)[R][3], const T (&Fin)[R][4][3], T (&Fout)[R][4][3],
                  const T (&Tin)[R][4][3], T (&Tout)[R][4][3]) {
    const bool out_plane = kk - 1 >= kc0 && kk - 1 < kc1;
    const Rsrc ry = plane_rsrc(yg + 3 * plane * (out_plane ? kk - 1 : 0), out_plane ? vbytes : 0);
    // u of plane kk (fixed DOFs masked when the input may be non-zero there)
    // (a wave-uniform test skips the selects for rows without fixed DOFs)
    T ue[R + 1][3];
#pragma unroll
    for (int r = 0; r <= R; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) ue[r][c] = T(uc[r][c]);
      if constexpr (FIRST) {
        // rounded on its own, as where the first sweep is stored: the product
        // is not contracted into the additions that consume it
#pragma clang fp contract(off)
#pragma unroll
        for (int c = 0; c < 3; ++c) ue[r][c] = wc[r][c] * ue[r][c];
      }
      if (MASKIN && __any(mc[r] != 0)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ue[r][c] = select_bit(mc[r], c, T(0), ue[r][c]);
      }
    }
    // x-edge modes of row r: s = u(i+1) + u(i), d = u(i+1) - u(i).  The
    // difference is formed as -(u(i) - u(i+1)) so that both shifts fold into
    // their additions (lane 63 reads 0 from its missing neighbour).
    auto xedge = [&](int r, T (&xe)[2][3]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xe[0][c] = lane_next(ue[r][c]) + ue[r][c];
        xe[1][c] = -(ue[r][c] - lane_next(ue[r][c]));
      }
    };
    // x adjoint of an edge row: node i takes the "0" end of edge i and the
    // "1" end of edge i-1.
    auto xadjoint = [&](const T (&e)[2][3], T (&nv)[3]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) nv[c] = (e[0][c] - e[1][c]) + lane_prev(e[0][c] + e[1][c]);
    };
    // node update of plane kk-1 for row r
    auto finish = [&](int r, const T (&Ku)[3]) {
      T v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T Au = select_bit(mo[r], c, uo[r][c], Ku[c]);
        if (MODE == kApply) {
          v[c] = Au;
          if (DOT && out_plane && offo[r] != kOutside) dot += (double)uo[r][c] * (double)Au;
        } else if (MODE == kSmooth || FIRST) {
          v[c] = uo[r][c] + wo[r][c] * (fo[r][c] - Au);
          if (DOT && out_plane && offo[r] != kOutside) dot += (double)fo[r][c] * (double)v[c];
        } else
          v[c] = fo[r][c] - Au;
      }
      store3(ry, offo[r], v);
    };
    T xa[2][3], xb[2][3];
    xedge(0, xa);

    if (kk >= kc0) {
      // ---- element layer kk-1 (between planes kk-1 and kk) -----------------
      T carry[2][3];   // "1"-end contributions of the face row above to edge row r+1
      T e0row[2][3];   // edge row 0 ("0" ends only) awaiting the previous wave
#pragma unroll
      for (int r = 0; r < R; ++r) {
        T (&xlo)[2][3] = (r & 1) ? xb : xa;
        T (&xhi)[2][3] = (r & 1) ? xa : xb;
        xedge(r + 1, xhi);
        // y-stage of plane kk, then z-stage against plane kk-1
        T v[8][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
          for (int xm = 0; xm < 2; ++xm) {
            const T fs = xhi[xm][c] + xlo[xm][c];  // y sum
            const T fd = xhi[xm][c] - xlo[xm][c];  // y difference
            v[xm][c] = fs + Fin[r][xm][c];
            v[xm + 4][c] = fs - Fin[r][xm][c];
            v[xm + 2][c] = fd + Fin[r][xm + 2][c];
            v[xm + 6][c] = fd - Fin[r][xm + 2][c];
            Fout[r][xm][c] = fs;
            Fout[r][xm + 2][c] = fd;
          }
        }
        T t[8][3];
        block_product<T>(q, Ec[r], v, t);
        // z adjoint: bottom face (plane kk-1) = t_lo - t_hi, top face (plane kk)
        // = t_lo + t_hi.  The bottom face joins the top face of the layer below
        // (same xy face), and the y adjoint is applied once to their sum:
        // edge row r ("0" end) = F_s - F_d, edge row r+1 ("1" end) = F_s + F_d.
        T e[2][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
          for (int xm = 0; xm < 2; ++xm) {
            const T Fs = Tin[r][xm][c] + (t[xm][c] - t[xm + 4][c]);
            const T Fd = Tin[r][xm + 2][c] + (t[xm + 2][c] - t[xm + 6][c]);
            Tout[r][xm][c] = t[xm][c] + t[xm + 4][c];
            Tout[r][xm + 2][c] = t[xm + 2][c] + t[xm + 6][c];
            e[xm][c] = (r > 0) ? carry[xm][c] + (Fs - Fd) : Fs - Fd;
            carry[xm][c] = Fs + Fd;
          }
        }
        if (r == 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int xm = 0; xm < 2; ++xm) e0row[xm][c] = e[xm][c];
        } else {
          T Ku[3];
          xadjoint(e, Ku);
          finish(r, Ku);
        }
      }
      // The last face row's "1"-end contributions belong to the next wave's
      // first node row: apply the x adjoint here and hand the node values over
      // through LDS.
      T(*slot)[64] = xch[kk & 1][w];
      {
        T nv[3];
        xadjoint(carry, nv);
#pragma unroll
        for (int c = 0; c < 3; ++c) slot[c][lane] = nv[c];
      }
      __syncthreads();
      T Ku[3];
      xadjoint(e0row, Ku);
      if (w > 0) {
        T(*prev)[64] = xch[kk & 1][w - 1];
#pragma unroll
        for (int c = 0; c < 3; ++c) Ku[c] += prev[c][lane];
      }
      finish(0, Ku);
    } else {
      // first plane of the chunk: only its face modes are needed (the layer
      // below it contributes nothing: Tout stays zero)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        T (&xlo)[2][3] = (r & 1) ? xb : xa;
        T (&xhi)[2][3] = (r & 1) ? xa : xb;
        xedge(r + 1, xhi);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int xm = 0; xm < 2; ++xm) {
            Fout[r][xm][c] = xhi[xm][c] + xlo[xm][c];
            Fout[r][xm + 2][c] = xhi[xm][c] - xlo[xm][c];
            Tout[r][xm][c] = T(0);
            Tout[r][xm + 2][c] = T(0);
          }
      }
    }
    // plane kk becomes the previous plane
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) uo[r][c] = FIRST ? ue[r][c] : T(uc[r][c]);
  };

  if constexpr (PRE > 0) {
    // zchunk == PRE output planes per workgroup (the library launches PRE = 1
    // for a z-chunk of one plane): every input is requested before any
    // arithmetic, so the workgroup waits on memory once.
    constexpr int Z = PRE;
    TU up[Z + 2][R + 1][3];
    T wp[Z + 2][FIRST ? R + 1 : 1][3];
    T Ep[Z + 2][R];
    int mp[Z + 2][R + 1], mo[Z][R];
    T fo[Z][R][3], wo[Z][R][3];
#pragma unroll
    for (int t = 0; t < Z + 2; ++t) load_plane(kc0 - 1 + t, up[t], wp[t], mp[t]);
#pragma unroll
    for (int r = 0; r < R; ++r) Ep[0][r] = T(0);
#pragma unroll
    for (int t = 1; t < Z + 2; ++t) load_layer(kc0 - 2 + t, Ep[t]);
#pragma unroll
    for (int o = 0; o < Z; ++o) load_out(kc0 + 1 + o, mo[o], fo[o], wo[o]);
#pragma unroll
    for (int t = 0; t < Z + 2; ++t) {
      const int kk = kc0 - 1 + t, o = t >= 2 ? t - 2 : 0;
      if (kk <= kc1) {
        if (t & 1)
          body(kk, up[t], wp[t], mp[t], Ep[t], mo[o], fo[o], wo[o], FpB, FpA, TpB, TpA);
        else
          body(kk, up[t], wp[t], mp[t], Ep[t], mo[o], fo[o], wo[o], FpA, FpB, TpA, TpB);
      }
    }
  } else {
    // two planes per trip: A is processed while B's plane is requested, then
    // the other way round
    load_plane(kc0 - 1, uA, wA, mA);
    load_layer(kc0 - 2, EA);
    for (int kk = kc0 - 1; kk <= kc1; kk += 2) {
      {
        load_plane(kk + 1, uB, wB, mB);
        load_layer(kk, EB);
        int mo[R];
        T fo[R][3], wo[R][3];
        load_out(kk, mo, fo, wo);
        body(kk, uA, wA, mA, EA, mo, fo, wo, FpA, FpB, TpA, TpB);
      }
      if (kk + 1 > kc1) break;
      {
        load_plane(kk + 2, uA, wA, mA);
        load_layer(kk + 1, EA);
        int mo[R];
        T fo[R][3], wo[R][3];
        load_out(kk + 1, mo, fo, wo);
        body(kk + 1, uB, wB, mB, EB, mo, fo, wo, FpB, FpA, TpB, TpA);
      }
    }
  }
  if (DOT) {  // one partial per workgroup, in a fixed order
    __shared__ double wsum[W];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += __shfl_down(dot, off, 64);
    if (lane == 0) wsum[w] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < W; ++k) t += wsum[k];
      const int parts = gx * gy * nchunks;
      const int rhs = bz / nchunks;
      dotp[(long long)parts * rhs + bx + gx * (by + gy * (bz % nchunks))] = t;
    }
  }
}

// Tile (bx, by) of the workgroup with index l in its z-slab of gx * gy tiles,
// whose first workgroup has linear id `first` in the launch: XCD c takes the
// c-th contiguous band (row-major) of every slab's tiles, so the tiles whose
// halo rows and columns overlap run on one L2, while the chip as a whole still
// moves through the grid one z-slab after the other.  Every tile is computed
// once, by the same arithmetic, and keeps its partial's slot.
__device__ inline void xcd_band_tile(int gx, int gy, int l, long long first, int& bx, int& by) {
  const int t = xcd_band_index(l, gx * gy, first);
  bx = t % gx;
  by = t / gx;
}

template <typename T, int MODE, int R, int W, int MINW, bool MASKIN, int PRE, bool DOT, typename TU = T>
__global__ __launch_bounds__(64 * W, MINW) void k_stream(Level L, HaarCoef<T> q, const T* __restrict__ Eg,
                                                      const TU* __restrict__ ug, const T* __restrict__ fg,
                                                      const T* __restrict__ wg, T* __restrict__ yg, int zchunk,
                                                      int nchunks, const int* __restrict__ act,
                                                      double* __restrict__ dotp) {
  int bx, by;
  xcd_band_tile(gridDim.x, gridDim.y, (int)blockIdx.x + (int)gridDim.x * (int)blockIdx.y,
                (long long)gridDim.x * gridDim.y * blockIdx.z, bx, by);
  stream_tile<T, MODE, R, W, MASKIN, PRE, DOT, TU>(L, q, Eg, ug, fg, wg, yg, zchunk, nchunks, act, dotp, bx, by,
                                                   blockIdx.z, gridDim.x, gridDim.y);
}

// Several grids in one launch: workgroup b belongs to the task t with
// begin[t] <= b < begin[t + 1]; b - begin[t] counts the task's workgroups z-slab
// by z-slab, and inside a slab the tiles go to the XCDs in bands as in
// k_stream.
// TU = float (binary64 K p only): u is the task's binary32 u32.
template <typename T, int MODE, int R, int W, int MINW, int PRE, bool DOT, typename TU = T>
__global__ __launch_bounds__(64 * W, MINW) void k_stream_batch(Batch<StreamTask<T>> tb, HaarCoef<T> q) {
  const int t = batch_task(tb.begin, tb.n, (int)blockIdx.x);
  const StreamTask<T>& a = tb.a[t];
  const int local = (int)blockIdx.x - tb.begin[t];
  const int bz = local / (a.gx * a.gy), l = local - bz * (a.gx * a.gy);
  int bx, by;
  xcd_band_tile(a.gx, a.gy, l, (long long)blockIdx.x - l, bx, by);
  const TU* u;
  if constexpr (sizeof(TU) == sizeof(T))
    u = a.u;
  else
    u = a.u32;
  stream_tile<T, MODE, R, W, false, PRE, DOT, TU>(a.L, q, a.E, u, a.f, a.wd, a.y, a.zchunk, a.nchunks, a.act,
                                                  a.dotp, bx, by, bz, a.gx, a.gy);
}

template <typename T, int R, int W, int MINW, bool MASKIN, int PRE>
void launch_stream_mode(int mode, dim3 grid, dim3 block, const Level& L, const HaarCoef<T>& q, const T* E,
                        const T* u, const T* f, const T* wd, T* y, int zchunk, int nchunks, const int* act,
                        double* dotp, hipStream_t s, const LaunchTimer& t) {
  if (mode == kApply && dotp && !MASKIN)
    launch_timed(k_stream<T, kApply, R, W, MINW, MASKIN, PRE, !MASKIN>, grid, block, s, t, L, q, E, u, f, wd, y,
                 zchunk, nchunks, act, dotp);
  else if (mode == kApply)
    launch_timed(k_stream<T, kApply, R, W, MINW, MASKIN, PRE, false>, grid, block, s, t, L, q, E, u, f, wd, y, zchunk,
                 nchunks, act, nullptr);
  else if (mode == kSmooth && dotp && !MASKIN)
    launch_timed(k_stream<T, kSmooth, R, W, MINW, MASKIN, PRE, !MASKIN>, grid, block, s, t, L, q, E, u, f, wd, y,
                 zchunk, nchunks, act, dotp);
  else if (mode == kSmooth)
    launch_timed(k_stream<T, kSmooth, R, W, MINW, MASKIN, PRE, false>, grid, block, s, t, L, q, E, u, f, wd, y,
                 zchunk, nchunks, act, nullptr);
  else
    launch_timed(k_stream<T, kResidual, R, W, MINW, MASKIN, PRE, false>, grid, block, s, t, L, q, E, u, f, wd, y,
                 zchunk, nchunks, act, nullptr);
}

template <typename T, int R, int W, int MINW>
void launch_stream_impl(int mode, bool maskin, const Level& L, const HaarCoef<T>& q, const T* E, const T* u,
                        const T* f, const T* wd, T* y, int zchunk, int nrhs, const int* act, double* dotp,
                        hipStream_t s, const LaunchTimer& t) {
  constexpr int kOutRows = W * R - 1;
  const int nchunks = (L.nzn + zchunk - 1) / zchunk;
  dim3 grid((L.nxn + 61) / 62, (L.nyn + kOutRows - 1) / kOutRows, nchunks * nrhs);
  dim3 block(64 * W);
  // a z-chunk of one plane takes the preloaded form
  if (maskin && zchunk == 1)
    launch_stream_mode<T, R, W, MINW, true, 1>(mode, grid, block, L, q, E, u, f, wd, y, zchunk, nchunks, act, dotp,
                                               s, t);
  else if (maskin)
    launch_stream_mode<T, R, W, MINW, true, 0>(mode, grid, block, L, q, E, u, f, wd, y, zchunk, nchunks, act, dotp,
                                               s, t);
  else if (zchunk == 1)
    launch_stream_mode<T, R, W, MINW, false, 1>(mode, grid, block, L, q, E, u, f, wd, y, zchunk, nchunks, act, dotp,
                                                s, t);
  else
    launch_stream_mode<T, R, W, MINW, false, 0>(mode, grid, block, L, q, E, u, f, wd, y, zchunk, nchunks, act, dotp,
                                                s, t);
}


// binary64 K u on binary32 input (the search direction of the mixed solver)
template <int R, int W, int MINW>
void launch_apply_u32_impl(const Level& L, const HaarCoef<double>& q, const double* E, const float* u, double* y,
                           int zchunk, int nrhs, const int* act, double* dotp, hipStream_t s, const LaunchTimer& t) {
  constexpr int kOutRows = W * R - 1;
  const int nchunks = (L.nzn + zchunk - 1) / zchunk;
  dim3 grid((L.nxn + 61) / 62, (L.nyn + kOutRows - 1) / kOutRows, nchunks * nrhs);
  dim3 block(64 * W);
  const double* none = nullptr;
  if (zchunk == 1 && dotp)
    launch_timed(k_stream<double, kApply, R, W, MINW, false, 1, true, float>, grid, block, s, t, L, q, E, u, none,
                 none, y, zchunk, nchunks, act, dotp);
  else if (zchunk == 1)
    launch_timed(k_stream<double, kApply, R, W, MINW, false, 1, false, float>, grid, block, s, t, L, q, E, u, none,
                 none, y, zchunk, nchunks, act, (double*)nullptr);
  else if (dotp)
    launch_timed(k_stream<double, kApply, R, W, MINW, false, 0, true, float>, grid, block, s, t, L, q, E, u, none,
                 none, y, zchunk, nchunks, act, dotp);
  else
    launch_timed(k_stream<double, kApply, R, W, MINW, false, 0, false, float>, grid, block, s, t, L, q, E, u, none,
                 none, y, zchunk, nchunks, act, (double*)nullptr);
}

// The sweep on the first sweep from zero (kSmoothFirst), one launch or a batch.
template <typename T, int R, int W, int MINW>
void launch_first_impl(const Level& L, const HaarCoef<T>& q, const T* E, const T* f, const T* wd, T* y, int zchunk,
                       int nrhs, const int* act, hipStream_t s, const LaunchTimer& t) {
  constexpr int kOutRows = W * R - 1;
  const int nchunks = (L.nzn + zchunk - 1) / zchunk;
  dim3 grid((L.nxn + 61) / 62, (L.nyn + kOutRows - 1) / kOutRows, nchunks * nrhs);
  dim3 block(64 * W);
  const T* none = nullptr;
  if (zchunk == 1)
    launch_timed(k_stream<T, kSmoothFirst, R, W, MINW, false, 1, false>, grid, block, s, t, L, q, E, none, f, wd, y,
                 zchunk, nchunks, act, (double*)nullptr);
  else
    launch_timed(k_stream<T, kSmoothFirst, R, W, MINW, false, 0, false>, grid, block, s, t, L, q, E, none, f, wd, y,
                 zchunk, nchunks, act, (double*)nullptr);
}
template <typename T, int R, int W, int MINW>
void launch_first_batch_impl(bool pre, const Batch<StreamTask<T>>& b, const HaarCoef<T>& q, hipStream_t s) {
  const dim3 grid(b.begin[b.n]), block(64 * W);
  if (pre) k_stream_batch<T, kSmoothFirst, R, W, MINW, 1, false><<<grid, block, 0, s>>>(b, q);
  else k_stream_batch<T, kSmoothFirst, R, W, MINW, 0, false><<<grid, block, 0, s>>>(b, q);
}

}  // namespace

// Shapes (rows per thread R, waves per workgroup W, minimum waves per SIMD the
// register allocation targets).  binary32: (2,4,2) (3,4,2) (4,4,1) (3,8,1)
// (2,8,1) (1,8,2) (1,4,2); binary64: (1,8,2) (2,4,1) (1,4,2) (taller binary64
// tiles spill).  A tile computes W*R element rows for W*R-1 output node rows, so the
// taller tiles repeat less work at their edges, and the one-row shapes have
// the shortest chain per thread (small, latency-bound levels).  All fit
// without spilling to memory.
int stream_shapes(bool f32) { return f32 ? 7 : 3; }
int stream_out_rows(bool f32, int shape) {
  static const int r32[7] = {4 * 2 - 1, 4 * 3 - 1, 4 * 4 - 1, 8 * 3 - 1, 8 * 2 - 1, 8 * 1 - 1, 4 * 1 - 1};
  static const int r64[3] = {8 * 1 - 1, 4 * 2 - 1, 4 * 1 - 1};
  return f32 ? r32[shape] : r64[shape];
}

// Shapes with a kSmoothFirst form: the one-row tiles and binary32's 2x4 (which
// holds omega/D of its input planes in three waves per SIMD's registers); the
// taller tiles would spill.
bool first_shape_ok(bool f32, int shape) { return f32 ? (shape == 0 || shape == 5 || shape == 6) : shape != 1; }

template <typename T>
void launch_stream(int mode, bool maskin, int shape, const Level& L, const HaarCoef<T>& q, const T* E, const T* u,
                   const T* f, const T* wd, T* y, int zchunk, int nrhs, const int* act, hipStream_t s,
                   const LaunchTimer& t, double* dotp) {
  if (mode == kSmoothFirst) {  // the caller checked first_shape_ok; no input masking, no partials
    if constexpr (sizeof(T) == 4) {
      if (shape == 0) launch_first_impl<T, 2, 4, 3>(L, q, E, f, wd, y, zchunk, nrhs, act, s, t);
      else if (shape == 5) launch_first_impl<T, 1, 8, 2>(L, q, E, f, wd, y, zchunk, nrhs, act, s, t);
      else launch_first_impl<T, 1, 4, 2>(L, q, E, f, wd, y, zchunk, nrhs, act, s, t);
    } else {
      if (shape == 0) launch_first_impl<T, 1, 8, 2>(L, q, E, f, wd, y, zchunk, nrhs, act, s, t);
      else launch_first_impl<T, 1, 4, 2>(L, q, E, f, wd, y, zchunk, nrhs, act, s, t);
    }
    return;
  }
  if constexpr (sizeof(T) == 4) {
    if (shape == 0)
      launch_stream_impl<T, 2, 4, 2>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else if (shape == 1)
      launch_stream_impl<T, 3, 4, 2>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else if (shape == 2)
      launch_stream_impl<T, 4, 4, 1>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else if (shape == 3)
      launch_stream_impl<T, 3, 8, 1>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else if (shape == 4)
      launch_stream_impl<T, 2, 8, 1>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else if (shape == 5)
      launch_stream_impl<T, 1, 8, 2>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else
      launch_stream_impl<T, 1, 4, 2>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
  } else {
    if (shape == 0)
      launch_stream_impl<T, 1, 8, 2>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else if (shape == 1)
      launch_stream_impl<T, 2, 4, 1>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
    else
      launch_stream_impl<T, 1, 4, 2>(mode, maskin, L, q, E, u, f, wd, y, zchunk, nrhs, act, dotp, s, t);
  }
}
template void launch_stream<float>(int, bool, int, const Level&, const HaarCoef<float>&, const float*,
                                   const float*, const float*, const float*, float*, int, int, const int*,
                                   hipStream_t, const LaunchTimer&, double*);
template void launch_stream<double>(int, bool, int, const Level&, const HaarCoef<double>&, const double*,
                                    const double*, const double*, const double*, double*, int, int, const int*,
                                    hipStream_t, const LaunchTimer&, double*);

void launch_sensitivity_haar(const Level& L, const HaarCoef<double>& q, const double* rho, const double* u,
                             double coef, double pm1, int accumulate, double* dc, hipStream_t s) {
  k_sensitivity_haar<<<(L.ne + 255) / 256, 256, 0, s>>>(L, q, rho, u, coef, pm1, accumulate, dc);
}

void launch_apply_u32(int shape, const Level& L, const HaarCoef<double>& q, const double* E, const float* u,
                      double* y, int zchunk, int nrhs, const int* act, hipStream_t s, const LaunchTimer& t,
                      double* dotp) {
  // the binary32 input leaves the one-row, four-wave tile room for three
  // waves per SIMD without spilling
  if (shape == 0)
    launch_apply_u32_impl<1, 8, 2>(L, q, E, u, y, zchunk, nrhs, act, dotp, s, t);
  else if (shape == 1)
    launch_apply_u32_impl<2, 4, 1>(L, q, E, u, y, zchunk, nrhs, act, dotp, s, t);
  else
    launch_apply_u32_impl<1, 4, 3>(L, q, E, u, y, zchunk, nrhs, act, dotp, s, t);
}

namespace {
// binary64 K u of the tasks' binary32 u32
template <int R, int W, int MINW>
void launch_stream_batch_u32(bool pre, bool dot, const Batch<StreamTask<double>>& b, const HaarCoef<double>& q,
                             hipStream_t s) {
  const dim3 grid(b.begin[b.n]), block(64 * W);
  if (pre && dot) k_stream_batch<double, kApply, R, W, MINW, 1, true, float><<<grid, block, 0, s>>>(b, q);
  else if (pre) k_stream_batch<double, kApply, R, W, MINW, 1, false, float><<<grid, block, 0, s>>>(b, q);
  else if (dot) k_stream_batch<double, kApply, R, W, MINW, 0, true, float><<<grid, block, 0, s>>>(b, q);
  else k_stream_batch<double, kApply, R, W, MINW, 0, false, float><<<grid, block, 0, s>>>(b, q);
}

template <typename T, int R, int W, int MINW>
void launch_stream_batch_impl(int mode, bool pre, bool dot, const Batch<StreamTask<T>>& b, const HaarCoef<T>& q,
                              hipStream_t s) {
  const dim3 grid(b.begin[b.n]), block(64 * W);
  if (mode == kApply) {
    if (pre && dot) k_stream_batch<T, kApply, R, W, MINW, 1, true><<<grid, block, 0, s>>>(b, q);
    else if (pre) k_stream_batch<T, kApply, R, W, MINW, 1, false><<<grid, block, 0, s>>>(b, q);
    else if (dot) k_stream_batch<T, kApply, R, W, MINW, 0, true><<<grid, block, 0, s>>>(b, q);
    else k_stream_batch<T, kApply, R, W, MINW, 0, false><<<grid, block, 0, s>>>(b, q);
  } else if (mode == kSmooth) {
    if (pre && dot) k_stream_batch<T, kSmooth, R, W, MINW, 1, true><<<grid, block, 0, s>>>(b, q);
    else if (pre) k_stream_batch<T, kSmooth, R, W, MINW, 1, false><<<grid, block, 0, s>>>(b, q);
    else if (dot) k_stream_batch<T, kSmooth, R, W, MINW, 0, true><<<grid, block, 0, s>>>(b, q);
    else k_stream_batch<T, kSmooth, R, W, MINW, 0, false><<<grid, block, 0, s>>>(b, q);
  } else {
    if (pre) k_stream_batch<T, kResidual, R, W, MINW, 1, false><<<grid, block, 0, s>>>(b, q);
    else k_stream_batch<T, kResidual, R, W, MINW, 0, false><<<grid, block, 0, s>>>(b, q);
  }
}
}  // namespace

template <typename T>
void launch_stream_batch(int mode, int shape, bool pre, bool dot, const Batch<StreamTask<T>>& b,
                         const HaarCoef<T>& q, hipStream_t s, bool u32in) {
  if (mode == kSmoothFirst) {  // shapes of launch_stream's kSmoothFirst
    if constexpr (sizeof(T) == 4) {
      if (shape == 0) launch_first_batch_impl<T, 2, 4, 3>(pre, b, q, s);
      else if (shape == 5) launch_first_batch_impl<T, 1, 8, 2>(pre, b, q, s);
      else launch_first_batch_impl<T, 1, 4, 2>(pre, b, q, s);
    } else {
      if (shape == 0) launch_first_batch_impl<T, 1, 8, 2>(pre, b, q, s);
      else launch_first_batch_impl<T, 1, 4, 2>(pre, b, q, s);
    }
    return;
  }
  if constexpr (sizeof(T) == 4) {
    if (shape == 0) launch_stream_batch_impl<T, 2, 4, 2>(mode, pre, dot, b, q, s);
    else if (shape == 1) launch_stream_batch_impl<T, 3, 4, 2>(mode, pre, dot, b, q, s);
    else if (shape == 2) launch_stream_batch_impl<T, 4, 4, 1>(mode, pre, dot, b, q, s);
    else if (shape == 3) launch_stream_batch_impl<T, 3, 8, 1>(mode, pre, dot, b, q, s);
    else if (shape == 4) launch_stream_batch_impl<T, 2, 8, 1>(mode, pre, dot, b, q, s);
    else if (shape == 5) launch_stream_batch_impl<T, 1, 8, 2>(mode, pre, dot, b, q, s);
    else launch_stream_batch_impl<T, 1, 4, 2>(mode, pre, dot, b, q, s);
  } else if (u32in) {  // the shapes of launch_apply_u32
    if (shape == 0) launch_stream_batch_u32<1, 8, 2>(pre, dot, b, q, s);
    else if (shape == 1) launch_stream_batch_u32<2, 4, 1>(pre, dot, b, q, s);
    else launch_stream_batch_u32<1, 4, 3>(pre, dot, b, q, s);
  } else {
    if (shape == 0) launch_stream_batch_impl<T, 1, 8, 2>(mode, pre, dot, b, q, s);
    else if (shape == 1) launch_stream_batch_impl<T, 2, 4, 1>(mode, pre, dot, b, q, s);
    else launch_stream_batch_impl<T, 1, 4, 2>(mode, pre, dot, b, q, s);
  }
}
template void launch_stream_batch<float>(int, int, bool, bool, const Batch<StreamTask<float>>&,
                                         const HaarCoef<float>&, hipStream_t, bool);
template void launch_stream_batch<double>(int, int, bool, bool, const Batch<StreamTask<double>>&,
                                          const HaarCoef<double>&, hipStream_t, bool);

void stream_grid(const Level& L, bool f32, int shape, int zchunk, int* gx, int* gy, int* nchunks) {
  const int rows = stream_out_rows(f32, shape);
  *gx = (L.nxn + 61) / 62;
  *gy = (L.nyn + rows - 1) / rows;
  *nchunks = (L.nzn + zchunk - 1) / zchunk;
}

int stream_blocks(const Level& L, bool f32, int shape, int zchunk) {
  const int rows = stream_out_rows(f32, shape);
  return ((L.nxn + 61) / 62) * ((L.nyn + rows - 1) / rows) * ((L.nzn + zchunk - 1) / zchunk);
}

}  // namespace hexmg
