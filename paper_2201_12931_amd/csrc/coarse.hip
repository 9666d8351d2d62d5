// The coarse part of the V-cycle (Alg. 3) in one cooperative launch.
//
// Below some level the grids are so small that every step of the V-cycle is a
// launch of a few microseconds whose cost is its own start-up, not its work.
// This kernel runs levels ls .. L-1 of the cycle -- the remaining pre-sweeps,
// residual, restriction, the coarsest solve, prolongation and post-sweeps --
// as phases of one grid-stride kernel separated by grid-wide barriers.  Each
// phase does exactly what the corresponding separate kernel does (the per-node
// functions are shared), in the same order, so the cycle is unchanged.
//
// The launch is cooperative (hipLaunchCooperativeKernel): the runtime only
// starts it when every workgroup is resident at once, which is what makes the
// grid barrier safe; it fails with an error rather than waiting otherwise.
#include <hip/hip_cooperative_groups.h>

#include "hexmg_impl.h"
#include "node_ops.h"

namespace hexmg {

namespace {

namespace cg = cooperative_groups;

template <typename T, int MODE>
__device__ void phase_gather(const CoarseCycle<T>& a, int l, const T* u, const T* f, T* y, int nrhs, const int* act,
                             long long gtid, long long gsize) {
  const Level& L = a.lv[l];
  for (int r = 0; r < nrhs; ++r) {
    if (act && !act[r]) continue;
    const long long off = 3ll * L.nn * r;
    for (long long n = gtid; n < L.nn; n += gsize)
      gather_node<T, MODE>(L, a.Ke, a.E[l], u + off, MODE != kApply ? f + off : f, a.wd[l], y + off, (int)n);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_cycle(CoarseCycle<T> a, int ls, int nrhs, const int* act) {
  cg::grid_group grid = cg::this_grid();
  const long long gtid = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long gsize = (long long)gridDim.x * kBlock;
  const int Lc = a.L - 1;  // coarsest level
  // Descent.  Level l starts with its first sweep (omega D^-1 f) in t[l].
  for (int l = ls; l < Lc; ++l) {
    T* buf[2] = {a.t[l], a.u[l]};
    int cur = 0;
    for (int it = 1; it < a.nu; ++it) {
      phase_gather<T, kSmooth>(a, l, buf[cur], a.f[l], buf[1 - cur], nrhs, act, gtid, gsize);
      grid.sync();
      cur = 1 - cur;
    }
    phase_gather<T, kResidual>(a, l, buf[cur], a.f[l], a.r[l], nrhs, act, gtid, gsize);
    grid.sync();
    const Level& F = a.lv[l];
    const Level& C = a.lv[l + 1];
    const bool fuse = l + 1 < Lc;
    for (int r = 0; r < nrhs; ++r) {
      if (act && !act[r]) continue;
      const long long fo = 3ll * F.nn * r, co = 3ll * C.nn * r;
      for (long long m = gtid; m < C.nn; m += gsize)
        restrict_node<T>(F, C, a.r[l] + fo, a.f[l + 1] + co, fuse ? a.wd[l + 1] : nullptr,
                         fuse ? a.t[l + 1] + co : nullptr, (int)m);
    }
    grid.sync();
  }
  // Coarsest solve: one wave per row.
  {
    const int lane = threadIdx.x & 63;
    const long long wave = gtid >> 6, nwaves = gsize >> 6;
    for (int r = 0; r < nrhs; ++r) {
      if (act && !act[r]) continue;
      const long long off = (long long)a.nc * r;
      for (long long row = wave; row < a.nc; row += nwaves)
        gemv_row<T>(a.nc, a.Ainv, a.f[Lc] + off, a.u[Lc] + off, (int)row, lane);
    }
    grid.sync();
  }
  // Ascent: u_l (in buf[cur]) += P e_{l+1}, then nu post-sweeps ending in u[l].
  for (int l = Lc - 1; l >= ls; --l) {
    T* buf[2] = {a.t[l], a.u[l]};
    int cur = (a.nu - 1) & 1;
    const Level& F = a.lv[l];
    const Level& C = a.lv[l + 1];
    for (int r = 0; r < nrhs; ++r) {
      if (act && !act[r]) continue;
      const long long fo = 3ll * F.nn * r, co = 3ll * C.nn * r;
      for (long long n = gtid; n < F.nn; n += gsize) prolong_node<T>(F, C, a.u[l + 1] + co, buf[cur] + fo, (int)n);
    }
    grid.sync();
    for (int it = 0; it < a.nu; ++it) {
      phase_gather<T, kSmooth>(a, l, buf[cur], a.f[l], buf[1 - cur], nrhs, act, gtid, gsize);
      if (!(l == ls && it == a.nu - 1)) grid.sync();  // the kernel's end orders the last phase
      cur = 1 - cur;
    }
  }
}

}  // namespace

template <typename T>
int coarse_cycle_max_blocks() {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_coarse_cycle<T>, kBlock, 0) != hipSuccess) return 0;
  return per_cu * prop.multiProcessorCount;
}
template int coarse_cycle_max_blocks<double>();
template int coarse_cycle_max_blocks<float>();

template <typename T>
hipError_t launch_coarse_cycle(const CoarseCycle<T>& a, int ls, int nrhs, const int* act, int blocks,
                               hipStream_t s) {
  CoarseCycle<T> arg = a;
  void* args[] = {(void*)&arg, (void*)&ls, (void*)&nrhs, (void*)&act};
  return hipLaunchCooperativeKernel((const void*)k_coarse_cycle<T>, dim3(blocks), dim3(kBlock), args, 0, s);
}
template hipError_t launch_coarse_cycle<double>(const CoarseCycle<double>&, int, int, const int*, int, hipStream_t);
template hipError_t launch_coarse_cycle<float>(const CoarseCycle<float>&, int, int, const int*, int, hipStream_t);

}  // namespace hexmg
