// Density filter (weights of Eqs. 4-5) and the optimality-criteria update
// (Eqs. 8-9) on the GPU.
//
// Filter: rho~_e = sum_i w_ei x_i / sum_i w_ei over in-domain elements i with
// w_ei = max(0, r - |c_e - c_i|).  The weight sum is recomputed per element
// (it only depends on how the stencil is cut by the domain), so no array of
// weight sums is stored.  The adjoint is g_x = H (g / Hs) (H is symmetric).
//
// OC: x_new(lambda) = clamp(x B^eta, max(0, x - m), min(1, x + m)) with
// B = -dc / (lambda dv).  Because x B^eta = s_e lambda^(-eta) with
// s_e = x_e (-dc_e / dv_e)^eta, one pass over the elements evaluates the volume
// dv^T x_new(lambda) (the filtered volume is linear in x) for kOcProbes values
// of lambda at once; the host narrows the bracket by that factor per pass.
#include <cmath>
#include <mutex>
#include <vector>

#include "hexmg_impl.h"

namespace hexmg {

namespace {

__device__ inline double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// MODE 0: out = (H in) / Hs;  1: out = in / Hs;  2: out = H in.
template <int MODE>
__global__ void k_filter(int nx, int ny, int nz, double rmin, int R, const double* __restrict__ in,
                         double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (i >= nx) return;
  const long long me = i + (long long)nx * (j + (long long)ny * k);
  double s = 0.0, ws = 0.0;
  for (int dk = -R; dk <= R; ++dk) {
    const int kk = k + dk;
    if (kk < 0 || kk >= nz) continue;
    for (int dj = -R; dj <= R; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= ny) continue;
      for (int di = -R; di <= R; ++di) {
        const int ii = i + di;
        if (ii < 0 || ii >= nx) continue;
        const double w = rmin - sqrt((double)(di * di + dj * dj + dk * dk));
        if (w <= 0.0) continue;
        ws += w;
        if (MODE != 1) s += w * in[ii + (long long)nx * (jj + (long long)ny * kk)];
      }
    }
  }
  if (MODE == 0)
    out[me] = s / ws;
  else if (MODE == 1)
    out[me] = in[me] / ws;
  else
    out[me] = s;
}

// Sensitivity filter (Eq. 3): out_e = (sum_i w_ei x_i dc_i) / (max(gamma, x_e) sum_i w_ei)
__global__ void k_sens_filter(int nx, int ny, int nz, double rmin, int R, double gamma, const double* __restrict__ x,
                              const double* __restrict__ dc, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (i >= nx) return;
  const long long me = i + (long long)nx * (j + (long long)ny * k);
  double s = 0.0, ws = 0.0;
  for (int dk = -R; dk <= R; ++dk) {
    const int kk = k + dk;
    if (kk < 0 || kk >= nz) continue;
    for (int dj = -R; dj <= R; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= ny) continue;
      for (int di = -R; di <= R; ++di) {
        const int ii = i + di;
        if (ii < 0 || ii >= nx) continue;
        const double w = rmin - sqrt((double)(di * di + dj * dj + dk * dk));
        if (w <= 0.0) continue;
        const long long o = ii + (long long)nx * (jj + (long long)ny * kk);
        ws += w;
        s += w * x[o] * dc[o];
      }
    }
  }
  out[me] = s / (fmax(gamma, x[me]) * ws);
}

// Self-weight: f = f_ext - (g / 8) sum_{e adjacent} rho_e along z (each of an
// element's eight nodes takes an eighth of its weight).  f_ext may be null.
__global__ void k_gravity_load(Level L, const double* __restrict__ rho, double g, const double* __restrict__ f_ext,
                               double* __restrict__ f) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= L.nn) return;
  const int i = n % L.nxn, t = n / L.nxn, j = t % L.nyn, k = t / L.nyn;
  double s = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int ei = i - (a & 1), ej = j - ((a >> 1) & 1), ek = k - (a >> 2);
    if (ei < 0 || ei >= L.nx || ej < 0 || ej >= L.ny || ek < 0 || ek >= L.nz) continue;
    s += rho[ei + L.nx * (ej + L.ny * ek)];
  }
  const long long b = 3ll * n;
  f[b] = f_ext ? f_ext[b] : 0.0;
  f[b + 1] = f_ext ? f_ext[b + 1] : 0.0;
  f[b + 2] = (f_ext ? f_ext[b + 2] : 0.0) - 0.125 * g * s;
}

// dc_e += coef * sum of u_z over the element's nodes (coef = 2 w (-g / 8))
__global__ void k_gravity_sensitivity(Level L, const double* __restrict__ u, double coef, double* __restrict__ dc) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= L.ne) return;
  const int i = e % L.nx, t = e / L.nx, j = t % L.ny, k = t / L.ny;
  double s = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int m = (i + (a & 1)) + L.nxn * ((j + ((a >> 1) & 1)) + L.nyn * (k + (a >> 2)));
    s += u[3ll * m + 2];
  }
  dc[e] += coef * s;
}

// passive elements: 1 = solid (x = 1), 2 = void (x = 0); others unchanged
__global__ void k_apply_passive(long long n, const uint8_t* __restrict__ passive, double* __restrict__ x) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int p = passive[e];
  if (p == 1) x[e] = 1.0;
  else if (p == 2) x[e] = 0.0;
}

// Volume at kOcProbes multipliers: partial[block][p] = sum_e dv_e x_new_e(lambda_p)
__global__ __launch_bounds__(kBlock) void k_oc_probe(long long n, const double* __restrict__ x,
                                                     const double* __restrict__ dc, const double* __restrict__ dv,
                                                     double eta, double move, OcProbes lam_pow,
                                                     double* __restrict__ partials) {
  __shared__ double part[kBlock / 64][kOcProbes];
  double acc[kOcProbes];
#pragma unroll
  for (int p = 0; p < kOcProbes; ++p) acc[p] = 0.0;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock) {
    const double xe = x[e], ve = dv[e];
    if (ve == 0.0) continue;  // outside the volume constraint (passive)
    const double B = -dc[e] / ve;
    const double se = xe * pow(B > 0.0 ? B : 0.0, eta);
    const double lo = fmax(0.0, xe - move), hi = fmin(1.0, xe + move);
#pragma unroll
    for (int p = 0; p < kOcProbes; ++p) acc[p] += ve * fmin(hi, fmax(lo, se * lam_pow.v[p]));
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int p = 0; p < kOcProbes; ++p) {
    const double v = wave_sum64(acc[p]);
    if (lane == 0) part[w][p] = v;
  }
  __syncthreads();
  if (threadIdx.x < kOcProbes) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) s += part[q][threadIdx.x];
    partials[(long long)blockIdx.x * kOcProbes + threadIdx.x] = s;
  }
}

__global__ void k_oc_probe_final(const double* __restrict__ partials, double* __restrict__ vol) {
  // one thread per probe, fixed order over the blocks
  const int p = threadIdx.x;
  if (p >= kOcProbes) return;
  double s = 0.0;
  for (int b = 0; b < kReduceBlocks; ++b) s += partials[(long long)b * kOcProbes + p];
  vol[p] = s;
}

// Number of design elements (passive == 0) per block: count[b].
__global__ __launch_bounds__(kBlock) void k_count_design(long long n, const uint8_t* __restrict__ passive,
                                                         int* __restrict__ count) {
  __shared__ int part[kBlock / 64];
  int c = 0;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock)
    c += passive[e] == 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) t += part[q];
    count[blockIdx.x] = t;
  }
}

// dv_e = [passive_e == 0] / (number of design elements); every block sums the
// kReduceBlocks counts itself.
__global__ __launch_bounds__(kBlock) void k_volume_weights(long long n, const uint8_t* __restrict__ passive,
                                                           const int* __restrict__ count, double* __restrict__ dv) {
  __shared__ long long tot;
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int b = 0; b < kReduceBlocks; ++b) t += count[b];
    tot = t;
  }
  __syncthreads();
  const double w = tot > 0 ? 1.0 / (double)tot : 0.0;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock)
    dv[e] = passive[e] == 0 ? w : 0.0;
}

// x_new at the final multiplier, one grid-stride pass (kReduceBlocks blocks);
// each block also writes the largest |x_new - x| and the partial sum of
// dv x_new over its elements to partials[2 b], partials[2 b + 1].
__global__ __launch_bounds__(kBlock) void k_oc_apply(long long n, const double* __restrict__ x,
                                                     const double* __restrict__ dc, const double* __restrict__ dv,
                                                     double eta, double move, double lam_pow,
                                                     double* __restrict__ xn, double* __restrict__ partials) {
  __shared__ double part[kBlock / 64][2];
  double ch = 0.0, vol = 0.0;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock) {
    const double xe = x[e], ve = dv[e];
    double y = xe;  // outside the volume constraint: left to the caller (passive)
    if (ve != 0.0) {
      const double B = -dc[e] / ve;
      const double se = xe * pow(B > 0.0 ? B : 0.0, eta);
      y = fmin(fmin(1.0, xe + move), fmax(fmax(0.0, xe - move), se * lam_pow));
    }
    xn[e] = y;
    ch = fmax(ch, fabs(y - xe));
    vol += ve * y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ch = fmax(ch, __shfl_down(ch, off, 64));
    vol += __shfl_down(vol, off, 64);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    part[w][0] = ch;
    part[w][1] = vol;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double c = 0.0, v = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
      c = fmax(c, part[q][0]);
      v += part[q][1];
    }
    partials[2ll * blockIdx.x] = c;
    partials[2ll * blockIdx.x + 1] = v;
  }
}

// out[0] = largest change, out[1] = dv . x_new (fixed order over the blocks)
__global__ void k_oc_apply_final(const double* __restrict__ partials, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double c = 0.0, v = 0.0;
  for (int b = 0; b < kReduceBlocks; ++b) {
    c = fmax(c, partials[2 * b]);
    v += partials[2 * b + 1];
  }
  out[0] = c;
  out[1] = v;
}

}  // namespace

void launch_filter(int nx, int ny, int nz, double rmin, int adjoint, const double* in, double* out, double* tmp,
                   hipStream_t s) {
  const int R = (int)std::ceil(rmin) - 1;
  const int bx = 64;
  dim3 grid((nx + bx - 1) / bx, ny, nz);
  if (adjoint) {
    k_filter<1><<<grid, bx, 0, s>>>(nx, ny, nz, rmin, R, in, tmp);
    k_filter<2><<<grid, bx, 0, s>>>(nx, ny, nz, rmin, R, tmp, out);
  } else {
    k_filter<0><<<grid, bx, 0, s>>>(nx, ny, nz, rmin, R, in, out);
  }
}

// Scratch of the adjoint filter for callers that cannot allocate: in / Hs for
// up to kFilterScratchElems elements.  Each device holds its own copy for the
// life of the process; its device address is looked up once per device (the
// array's name is a host-side stand-in and is never passed to a kernel).
__device__ __align__(256) double scratch[kFilterScratchElems];

int filter_scratch_ptr(double** ptr) {
  static std::mutex mu;
  static std::vector<double*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return 0;
}

void launch_sens_filter(int nx, int ny, int nz, double rmin, double gamma, const double* x, const double* dc,
                        double* out, hipStream_t s) {
  const int R = (int)std::ceil(rmin) - 1;
  const int bx = 64;
  k_sens_filter<<<dim3((nx + bx - 1) / bx, ny, nz), bx, 0, s>>>(nx, ny, nz, rmin, R, gamma, x, dc, out);
}

void launch_gravity_load(const Level& L, const double* rho, double g, const double* f_ext, double* f,
                         hipStream_t s) {
  k_gravity_load<<<(L.nn + kBlock - 1) / kBlock, kBlock, 0, s>>>(L, rho, g, f_ext, f);
}

void launch_gravity_sensitivity(const Level& L, const double* u, double coef, double* dc, hipStream_t s) {
  k_gravity_sensitivity<<<(L.ne + kBlock - 1) / kBlock, kBlock, 0, s>>>(L, u, coef, dc);
}

void launch_apply_passive(long long n, const uint8_t* passive, double* x, hipStream_t s) {
  k_apply_passive<<<(int)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, passive, x);
}

void launch_oc_probe(long long n, const double* x, const double* dc, const double* dv, double eta, double move,
                     const OcProbes& lam_pow, double* partials, double* vol, hipStream_t s) {
  k_oc_probe<<<kReduceBlocks, kBlock, 0, s>>>(n, x, dc, dv, eta, move, lam_pow, partials);
  k_oc_probe_final<<<1, 64, 0, s>>>(partials, vol);
}

void launch_volume_weights(long long n, const uint8_t* passive, int* count, double* dv, hipStream_t s) {
  k_count_design<<<kReduceBlocks, kBlock, 0, s>>>(n, passive, count);
  k_volume_weights<<<kReduceBlocks, kBlock, 0, s>>>(n, passive, count, dv);
}

void launch_oc_apply(long long n, const double* x, const double* dc, const double* dv, double eta, double move,
                     double lam_pow, double* xn, double* partials, double* out, hipStream_t s) {
  k_oc_apply<<<kReduceBlocks, kBlock, 0, s>>>(n, x, dc, dv, eta, move, lam_pow, xn, partials);
  k_oc_apply_final<<<1, 64, 0, s>>>(partials, out);
}

}  // namespace hexmg
