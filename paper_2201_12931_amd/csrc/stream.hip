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
// (per xy-face) by the 2 elements above and below it; only the z-stage, the
// block product and their adjoints are per element.  This takes K u from
// 576 FMA per node (dense 24x24 rows) to ~150 VALU operations per node.
//
// Mapping.  A wave owns 64 consecutive node columns in x (lane = column) and R
// consecutive node rows in y (held in registers); a workgroup stacks W waves in
// y; all threads march along z through a chunk of planes.  x-neighbours are
// exchanged with DPP wavefront shifts, y-neighbours inside a wave live in the
// same thread, and the only cross-wave dependency (the adjoint contribution of
// a wave's last face row to the next wave's first node row) goes through LDS,
// double-buffered by plane parity, with one barrier per plane.  Each tile reads
// a one-node halo on every side and writes the interior: 62 columns x (W*R-2)
// rows x its z-chunk.  Every output is written exactly once: no atomics.
//
// Out-of-domain nodes read as 0 and out-of-domain elements have modulus 0, so
// the boundary needs no special case.  Fixed DOFs read as 0 and return u.
#include "hexmg_impl.h"

namespace hexmg {

namespace {

template <typename T>
struct StreamArgs {
  Level L;
  HaarCoef<T> q;
  const T* __restrict__ E;
  const T* __restrict__ u;
  const T* __restrict__ f;
  const T* __restrict__ wd;
  T* __restrict__ y;
  int zchunk;
};

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

// Epilogue for one node of a completed plane: A u from the node sum (u itself
// at fixed DOFs), then y = A u, the Jacobi update or the residual.
template <typename T, int MODE>
__device__ inline void finish_node(const StreamArgs<T>& a, long long n, const T (&Ku)[3]) {
  const int mk = a.L.mask[n];
  const T* uo = a.u + 3 * n;
  T* yo = a.y + 3 * n;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T uc = uo[c];
    const T Au = ((mk >> c) & 1) ? uc : Ku[c];
    if (MODE == kApply)
      yo[c] = Au;
    else if (MODE == kSmooth)
      yo[c] = uc + a.wd[3 * n + c] * (a.f[3 * n + c] - Au);
    else
      yo[c] = a.f[3 * n + c] - Au;
  }
}

template <typename T, int MODE, int R, int W>
__global__ __launch_bounds__(64 * W, 2) void k_stream(StreamArgs<T> a) {
  const Level& L = a.L;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  constexpr int kOutRows = W * R - 2;
  const int i = blockIdx.x * 62 - 1 + lane;           // node column of this lane
  const int jt0 = blockIdx.y * kOutRows - 1;          // first (halo) row of the tile
  const int j0 = jt0 + w * R;                         // first row of this wave
  const int kc0 = blockIdx.z * a.zchunk;
  const int kc1 = min(kc0 + a.zchunk, L.nzn);         // output planes [kc0, kc1)
  const bool lane_out = lane >= 1 && lane <= 62 && i < L.nxn;
  const bool col_in = i >= 0 && i < L.nxn;
  const bool col_elem = i >= 0 && i < L.nx;
  const long long plane = (long long)L.nxn * L.nyn;
  const long long eplane = (long long)L.nx * L.ny;

  __shared__ T xch[2][W][6][64];  // [parity][wave][bottom xyz, top xyz][lane]

  T Fp[R][4][3];   // face modes of the previous plane
  T Yp[R][3];      // pending node sums of the previous plane
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Yp[r][c] = T(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) Fp[r][m][c] = T(0);
    }

  for (int kk = kc0 - 1; kk <= kc1; ++kk) {
    const bool plane_in = kk >= 0 && kk < L.nzn;
    // ---- load plane kk, rows 0..R (out of domain or fixed reads as 0) --------
    T ue[R + 1][3];
#pragma unroll
    for (int r = 0; r <= R; ++r) {
      const int jr = j0 + r;
      T u0 = T(0), u1 = T(0), u2 = T(0);
      if (plane_in && col_in && jr >= 0 && jr < L.nyn) {
        const long long n = (long long)i + (long long)L.nxn * jr + plane * kk;
        const int mk = L.mask[n];
        const T* p = a.u + 3 * n;
        u0 = (mk & 1) ? T(0) : p[0];
        u1 = (mk & 2) ? T(0) : p[1];
        u2 = (mk & 4) ? T(0) : p[2];
      }
      ue[r][0] = u0;
      ue[r][1] = u1;
      ue[r][2] = u2;
    }
    // x-edge modes of row r: s = u(i+1) + u(i), d = u(i+1) - u(i)
    auto xedge = [&](int r, T (&xe)[2][3]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T nx_ = lane_next(ue[r][c]);
        xe[0][c] = nx_ + ue[r][c];
        xe[1][c] = nx_ - ue[r][c];
      }
    };
    T xa[2][3], xb[2][3];
    xedge(0, xa);

    if (kk >= kc0) {
      // ---- element layer kk-1 (between planes kk-1 and kk) -----------------
      const int ke = kk - 1;
      const bool layer_in = ke >= 0 && ke < L.nz;
      const bool out_plane = ke >= kc0;  // plane kk-1 is an output plane
      T carry_b[2][3], carry_t[2][3];    // "1"-end edge contributions to row r+1
      T x0b[2][3], x0t[2][3];            // row 0 edge sums awaiting the previous wave
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int jr = j0 + r;
        T Ee = T(0);
        if (layer_in && col_elem && jr >= 0 && jr < L.ny) Ee = a.E[i + (long long)L.nx * jr + eplane * ke];
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
            v[xm][c] = fs + Fp[r][xm][c];
            v[xm + 4][c] = fs - Fp[r][xm][c];
            v[xm + 2][c] = fd + Fp[r][xm + 2][c];
            v[xm + 6][c] = fd - Fp[r][xm + 2][c];
            Fp[r][xm][c] = fs;
            Fp[r][xm + 2][c] = fd;
          }
        }
        T t[8][3];
        block_product<T>(a.q, Ee, v, t);
        // z adjoint: bottom face (plane kk-1) = t_s - t_d, top face (plane kk) = t_s + t_d;
        // y adjoint: edge row r ("0" end) = G_s - G_d, edge row r+1 ("1" end) = G_s + G_d.
        T eb0[2][3], et0[2][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
          for (int xm = 0; xm < 2; ++xm) {
            const T bs = t[xm][c] - t[xm + 4][c], bd = t[xm + 2][c] - t[xm + 6][c];
            const T ts = t[xm][c] + t[xm + 4][c], td = t[xm + 2][c] + t[xm + 6][c];
            eb0[xm][c] = bs - bd;
            et0[xm][c] = ts - td;
            if (r > 0) {
              eb0[xm][c] += carry_b[xm][c];
              et0[xm][c] += carry_t[xm][c];
            }
            carry_b[xm][c] = bs + bd;
            carry_t[xm][c] = ts + td;
          }
        }
        if (r == 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int xm = 0; xm < 2; ++xm) {
              x0b[xm][c] = eb0[xm][c];
              x0t[xm][c] = et0[xm][c];
            }
        } else {
          // edge row r complete: x adjoint gives the node sums of row r
          T Ku[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T bs = eb0[0][c], bd = eb0[1][c], ts = et0[0][c], td = et0[1][c];
            Ku[c] = Yp[r][c] + (bs - bd) + lane_prev(bs + bd);
            Yp[r][c] = (ts - td) + lane_prev(ts + td);
          }
          const int rt = w * R + r;
          if (out_plane && lane_out && rt <= kOutRows && jr < L.nyn)
            finish_node<T, MODE>(a, (long long)i + (long long)L.nxn * jr + plane * ke, Ku);
        }
      }
      // The last face row's "1"-end edge contributions belong to the next
      // wave's first node row: apply the x adjoint here and hand over the node
      // values through LDS.
      T(*slot)[64] = xch[kk & 1][w];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T bs = carry_b[0][c], bd = carry_b[1][c], ts = carry_t[0][c], td = carry_t[1][c];
        slot[c][lane] = (bs - bd) + lane_prev(bs + bd);
        slot[3 + c][lane] = (ts - td) + lane_prev(ts + td);
      }
      __syncthreads();
      T Ku[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T bs = x0b[0][c], bd = x0b[1][c], ts = x0t[0][c], td = x0t[1][c];
        Ku[c] = Yp[0][c] + (bs - bd) + lane_prev(bs + bd);
        Yp[0][c] = (ts - td) + lane_prev(ts + td);
      }
      if (w > 0) {
        T(*prev)[64] = xch[kk & 1][w - 1];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Ku[c] += prev[c][lane];
          Yp[0][c] += prev[3 + c][lane];
        }
      }
      const int rt0 = w * R;
      if (out_plane && lane_out && rt0 >= 1 && j0 < L.nyn)
        finish_node<T, MODE>(a, (long long)i + (long long)L.nxn * j0 + plane * ke, Ku);
    } else {
      // first plane of the chunk: only its face modes are needed
#pragma unroll
      for (int r = 0; r < R; ++r) {
        T (&xlo)[2][3] = (r & 1) ? xb : xa;
        T (&xhi)[2][3] = (r & 1) ? xa : xb;
        xedge(r + 1, xhi);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int xm = 0; xm < 2; ++xm) {
            Fp[r][xm][c] = xhi[xm][c] + xlo[xm][c];
            Fp[r][xm + 2][c] = xhi[xm][c] - xlo[xm][c];
          }
      }
    }
  }
}

template <typename T, int R, int W>
void launch_stream_impl(int mode, const StreamArgs<T>& a, hipStream_t s) {
  constexpr int kOutRows = W * R - 2;
  dim3 grid((a.L.nxn + 61) / 62, (a.L.nyn + kOutRows - 1) / kOutRows, (a.L.nzn + a.zchunk - 1) / a.zchunk);
  dim3 block(64 * W);
  if (mode == kApply)
    k_stream<T, kApply, R, W><<<grid, block, 0, s>>>(a);
  else if (mode == kSmooth)
    k_stream<T, kSmooth, R, W><<<grid, block, 0, s>>>(a);
  else
    k_stream<T, kResidual, R, W><<<grid, block, 0, s>>>(a);
}

}  // namespace

template <typename T>
void launch_stream(int mode, const Level& L, const HaarCoef<T>& q, const T* E, const T* u, const T* f,
                   const T* wd, T* y, int zchunk, hipStream_t s) {
  StreamArgs<T> a{L, q, E, u, f, wd, y, zchunk};
  if constexpr (sizeof(T) == 4)
    launch_stream_impl<T, kStreamRows32, kStreamWaves32>(mode, a, s);
  else
    launch_stream_impl<T, kStreamRows64, kStreamWaves64>(mode, a, s);
}
template void launch_stream<float>(int, const Level&, const HaarCoef<float>&, const float*, const float*,
                                   const float*, const float*, float*, int, hipStream_t);
template void launch_stream<double>(int, const Level&, const HaarCoef<double>&, const double*, const double*,
                                    const double*, const double*, double*, int, hipStream_t);

}  // namespace hexmg
