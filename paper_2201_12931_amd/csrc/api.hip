// C ABI of the hexmg library: grid set-up, K u, V-cycle, MGPCG solve,
// compliance and sensitivity.  Host orchestration only; all arithmetic of the
// hot path runs in the kernels of kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>

#include "hexmg_impl.h"

namespace hexmg {

// Launches of several grids recorded during hexmg_batch_solve.  Each record
// holds its grid, its place in that grid's PCG iteration (stage: a stage not
// above the grid's previous one starts the grid's next chunk, i.e. its next
// iteration) and its single launch; a launch of a batchable kernel also holds
// its task and a signature (kernel and template arguments).  flush() launches
// everything in (chunk, stage) order: each grid's own launches keep their
// order, and the records of one (chunk, stage) and signature from several grids
// go out as one launch over all of them.
struct BatchRecorder {
  struct Rec {
    int grid = 0, chunk = 0, stage = 0, blocks = 0;
    unsigned long long sig = 0;  // 0: launched on its own
    std::function<hipError_t(hipStream_t)> one;
    std::function<hipError_t(const std::vector<const Rec*>&, hipStream_t)> group;
    std::vector<unsigned char> task;
  };
  std::vector<Rec> recs;
  std::vector<int> last, chunk;
  size_t launches = 0, records = 0;  // launches issued / records taken (statistics)
  explicit BatchRecorder(int ngrids) : last(ngrids, -1), chunk(ngrids, 0) {}
  void add(int grid, int stage, Rec r) {
    if (stage <= last[grid]) ++chunk[grid];
    last[grid] = stage;
    r.grid = grid;
    r.chunk = chunk[grid];
    r.stage = stage;
    recs.push_back(std::move(r));
  }
  hipError_t flush(hipStream_t s) {
    std::vector<const Rec*> order;
    order.reserve(recs.size());
    for (const Rec& r : recs) order.push_back(&r);
    std::stable_sort(order.begin(), order.end(), [](const Rec* a, const Rec* b) {
      if (a->chunk != b->chunk) return a->chunk < b->chunk;
      if (a->stage != b->stage) return a->stage < b->stage;
      if (a->sig != b->sig) return a->sig < b->sig;
      return a->grid < b->grid;
    });
    hipError_t err = hipSuccess;
    for (size_t i = 0; i < order.size();) {
      const Rec* a = order[i];
      size_t j = i + 1;
      if (a->sig != 0)
        while (j < order.size() && order[j]->chunk == a->chunk && order[j]->stage == a->stage &&
               order[j]->sig == a->sig)
          ++j;
      hipError_t e = hipSuccess;
      if (j - i == 1) {
        e = a->one(s);
      } else {
        std::vector<const Rec*> grp(order.begin() + i, order.begin() + j);
        e = a->group(grp, s);
      }
      ++launches;
      if (e != hipSuccess && err == hipSuccess) err = e;
      i = j;
    }
    records += recs.size();
    recs.clear();
    std::fill(last.begin(), last.end(), -1);
    std::fill(chunk.begin(), chunk.end(), 0);
    return err;
  }
};

}  // namespace hexmg

using namespace hexmg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(x)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return fail(HEXMG_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---- launching or recording (hexmg_batch_solve) ------------------------------
// Places of the launches in a PCG iteration; a V-cycle's descent at level l
// (0 first sweep, 1.. further sweeps, 90 residual, 95 restriction), its
// coarsest solve, its ascent at level l (0 prolongation, 1.. sweeps), and the
// CG steps after it.
constexpr int kStStart = 10, kStInit = 30, kStRestart = 40, kStReplace = 50;
constexpr int kStCoarse = 5000, kStEnd = 9000;
inline int st_down(int l, int step) { return 1000 + 100 * l + step; }
inline int st_up(int l, int step) { return 6000 + 100 * (kMaxLevels - l) + step; }

// A kernel launch (fn(stream) launches it): now, or recorded while batching.
template <typename F>
void emit_launch(hexmg_grid* g, int stage, hipStream_t s, F fn) {
  if (!g->rec) {
    fn(s);
    return;
  }
  BatchRecorder::Rec r;
  r.one = [fn](hipStream_t st) {
    fn(st);
    return hipGetLastError();
  };
  g->rec->add(g->rec_grid, stage, std::move(r));
}
// A runtime call returning its status (event records, copies): now, or recorded.
template <typename F>
hipError_t emit_api(hexmg_grid* g, int stage, hipStream_t s, F fn) {
  if (!g->rec) return fn(s);
  BatchRecorder::Rec r;
  r.one = fn;
  g->rec->add(g->rec_grid, stage, std::move(r));
  return hipSuccess;
}
// A launch of a batchable kernel: task A with `blocks` workgroups; sig
// identifies kernel and template arguments; one(stream) is its single launch,
// many(batch, stream) launches a Batch<A>.
template <typename A, typename One, typename Many>
void emit_task(hexmg_grid* g, int stage, hipStream_t s, unsigned long long sig, const A& task, int blocks, One one,
               Many many) {
  if (!g->rec) {
    one(s);
    return;
  }
  BatchRecorder::Rec r;
  r.sig = sig;
  r.blocks = blocks;
  r.task.resize(sizeof(A));
  std::memcpy(r.task.data(), &task, sizeof(A));
  r.one = [one](hipStream_t st) {
    one(st);
    return hipGetLastError();
  };
  r.group = [many](const std::vector<const BatchRecorder::Rec*>& rs, hipStream_t st) {
    for (size_t i = 0; i < rs.size(); i += kMaxBatch) {
      Batch<A> b;
      b.n = (int)std::min<size_t>(kMaxBatch, rs.size() - i);
      b.begin[0] = 0;
      for (int t = 0; t < b.n; ++t) {
        std::memcpy(&b.a[t], rs[i + t]->task.data(), sizeof(A));
        b.begin[t + 1] = b.begin[t] + rs[i + t]->blocks;
      }
      many(b, st);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  g->rec->add(g->rec_grid, stage, std::move(r));
}
// signature of a batchable launch: kernel kind, element sizes, mode/shape/flags
inline unsigned long long batch_sig(int kind, int a = 0, int b = 0, int c = 0, int d = 0, int e = 0) {
  return (unsigned long long)(kind + 1) | ((unsigned long long)(a & 0xff) << 8) |
         ((unsigned long long)(b & 0xff) << 16) | ((unsigned long long)(c & 0xff) << 24) |
         ((unsigned long long)(d & 0xff) << 32) | ((unsigned long long)(e & 0xff) << 40);
}
enum BatchKind { kBkStream, kBkRestrict, kBkProlong, kBkGemv, kBkUpdateR, kBkRrCheck, kBkUpdatePx, kBkStreamU32 };

// smooth1: the sweep on the first sweep from zero, formed on load (kSmoothFirst)
const char* kFamilies[] = {"apply_f64", "apply_f32", "smooth_f64", "smooth_f32", "residual_f64",
                           "residual_f32", "smooth1_f64", "smooth1_f32"};
constexpr int kNumFamilies = 8;

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

int validate(const hexmg_grid_desc* d) {
  if (!d) return fail(HEXMG_ERR_INVALID, "null descriptor");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(HEXMG_ERR_INVALID, "grid dimensions must be >= 1");
  if (d->levels < 1 || d->levels > 12) return fail(HEXMG_ERR_INVALID, "levels must be in [1, 12]");
  const int q = 1 << (d->levels - 1);
  if (d->nx % q || d->ny % q || d->nz % q)
    return fail(HEXMG_ERR_INVALID, "grid dimensions must be divisible by 2^(levels-1)");
  const long long nn = (long long)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
  if (3 * nn >= (1ll << 31)) return fail(HEXMG_ERR_INVALID, "grid too large (3*nodes must be < 2^31)");
  if (24ll * (d->nx + 1) * (d->ny + 1) >= (1ll << 31))
    return fail(HEXMG_ERR_INVALID, "xy plane too large (24*(nx+1)*(ny+1) must be < 2^31)");
  if (d->ny + 1 > 65535 || d->nz + 1 > 65535)
    return fail(HEXMG_ERR_INVALID, "ny + 1 and nz + 1 must be <= 65535 (launch grid limits)");
  const long long nnc = (long long)(d->nx / q + 1) * (d->ny / q + 1) * (d->nz / q + 1);
  if (3 * nnc > 6144) return fail(HEXMG_ERR_INVALID, "coarsest level too large for the dense solve (> 6144 DOFs); add levels");
  if (!(d->Emin > 0.0) || !(d->E0 > d->Emin) || !std::isfinite(d->E0))
    return fail(HEXMG_ERR_INVALID, "need 0 < Emin < E0 < inf");
  if (!(d->nu > -1.0 && d->nu < 0.5)) return fail(HEXMG_ERR_INVALID, "need -1 < nu < 0.5");
  if (!(d->penal >= 1.0 && d->penal <= 16.0)) return fail(HEXMG_ERR_INVALID, "need 1 <= penal <= 16");
  if (d->precision != HEXMG_FP64 && d->precision != HEXMG_MIXED && d->precision != HEXMG_MIXED32)
    return fail(HEXMG_ERR_INVALID, "bad precision");
  if (d->vcycle_both != 0 && d->vcycle_both != 1) return fail(HEXMG_ERR_INVALID, "vcycle_both must be 0 or 1");
  if (d->rr_every < 0) return fail(HEXMG_ERR_INVALID, "rr_every must be >= 0");
  if (d->smooth_sweeps < 1 || d->smooth_sweeps > 64) return fail(HEXMG_ERR_INVALID, "smooth_sweeps in [1,64]");
  if (!(d->omega == 0.0 || (d->omega > 0.0 && d->omega <= 1.0)))
    return fail(HEXMG_ERR_INVALID, "need omega = 0 (automatic) or 0 < omega <= 1");
  if (d->coarse_avg != HEXMG_AVG_DENSITY && d->coarse_avg != HEXMG_AVG_MODULUS)
    return fail(HEXMG_ERR_INVALID, "bad coarse_avg");
  if (d->max_nrhs < 1) return fail(HEXMG_ERR_INVALID, "max_nrhs must be >= 1");
  if (d->kernel != HEXMG_KERNEL_STREAM && d->kernel != HEXMG_KERNEL_GATHER && d->kernel != HEXMG_KERNEL_AUTO)
    return fail(HEXMG_ERR_INVALID, "bad kernel");
  if (d->coarse_op != HEXMG_COARSE_REDISCRETIZE && d->coarse_op != HEXMG_COARSE_GALERKIN)
    return fail(HEXMG_ERR_INVALID, "bad coarse_op");
  if (d->fuse_first != 0 && d->fuse_first != 1) return fail(HEXMG_ERR_INVALID, "fuse_first must be 0 or 1");
  if (d->stencil_storage != HEXMG_STENCIL_F32 && d->stencil_storage != HEXMG_STENCIL_BF16 &&
      d->stencil_storage != HEXMG_STENCIL_F16)
    return fail(HEXMG_ERR_INVALID, "bad stencil_storage");
  return 0;
}

void make_levels(const hexmg_grid_desc* d, std::vector<Level>& lv) {
  lv.clear();
  for (int l = 0; l < d->levels; ++l) {
    Level L;
    L.nx = d->nx >> l;
    L.ny = d->ny >> l;
    L.nz = d->nz >> l;
    L.nxn = L.nx + 1;
    L.nyn = L.ny + 1;
    L.nzn = L.nz + 1;
    L.nn = L.nxn * L.nyn * L.nzn;
    L.ne = L.nx * L.ny * L.nz;
    L.mask = nullptr;
    lv.push_back(L);
  }
}

// One layout function serves hexmg_workspace_size (base = nullptr) and
// hexmg_grid_create.
size_t carve(hexmg_grid* g, char* base) {
  Carver c{base};
  const int L = g->L;
  g->rho.assign(L, nullptr);
  g->E64.assign(L, nullptr);
  g->E32.assign(L, nullptr);
  g->wd64.assign(L, nullptr);
  g->wd32.assign(L, nullptr);
  g->mask.assign(L, nullptr);
  g->vf64.assign(L, nullptr);
  g->vu64.assign(L, nullptr);
  g->vt64.assign(L, nullptr);
  g->vr64.assign(L, nullptr);
  g->vf32.assign(L, nullptr);
  g->vu32.assign(L, nullptr);
  g->vt32.assign(L, nullptr);
  g->vr32.assign(L, nullptr);
  const size_t R = (size_t)g->desc.max_nrhs;
  // V-cycle vectors and Jacobi diagonals in the solver's precision, and in the
  // other one only when the descriptor asks for both.
  const bool v64 = g->desc.precision == HEXMG_FP64 || g->desc.vcycle_both;
  const bool v32 = g->desc.precision != HEXMG_FP64 || g->desc.vcycle_both;
  for (int l = 0; l < L; ++l) {
    const Level& lv = g->lv[l];
    const size_t N = 3ull * lv.nn;
    g->rho[l] = c.take<double>(lv.ne);
    g->E64[l] = c.take<double>(lv.ne);
    g->E32[l] = c.take<float>(lv.ne);
    g->mask[l] = c.take<uint8_t>(lv.nn);
    if (v64) {
      g->wd64[l] = c.take<double>(N);
      g->vf64[l] = c.take<double>(N * R);
      g->vu64[l] = c.take<double>(N * R);
      g->vt64[l] = c.take<double>(N * R);
      g->vr64[l] = c.take<double>(N * R);
    }
    if (v32) {
      g->wd32[l] = c.take<float>(N);
      g->vf32[l] = c.take<float>(N * R);
      g->vu32[l] = c.take<float>(N * R);
      g->vt32[l] = c.take<float>(N * R);
      g->vr32[l] = c.take<float>(N * R);
    }
  }
  const size_t nc = 3ull * g->lv[L - 1].nn;
  g->nc = (int)nc;
  g->Abuf[0] = c.take<double>(nc * nc);
  g->Abuf[1] = c.take<double>(nc * nc);
  g->gjD = c.take<double>(2 * kGJBlock * kGJBlock);
  g->Ecoarse = c.take<double>(g->lv[L - 1].ne);
  g->Ke64 = c.take<double>(576);
  g->Ke32 = c.take<float>(576);
  const size_t N0 = 3ull * g->lv[0].nn;
  g->r = c.take<double>(N0 * R);
  // binary64 z only for binary64 solves (mixed precision keeps z in binary32)
  g->z = g->desc.precision == HEXMG_FP64 ? c.take<double>(N0 * R) : nullptr;
  // the search direction: binary64 (binary64 solves; the binary32 outer K p
  // keeps a binary32 copy), binary32 alone in the mixed form
  g->p = g->desc.precision != HEXMG_MIXED ? c.take<double>(N0 * R) : nullptr;
  g->q = c.take<double>(N0 * R);
  g->p32 = g->desc.precision != HEXMG_FP64 ? c.take<float>(N0 * R) : nullptr;
  // the mixed form alternates its binary32 direction between two buffers
  g->p32b = g->desc.precision == HEXMG_MIXED ? c.take<float>(N0 * R) : nullptr;
  g->q32 = g->desc.precision == HEXMG_MIXED32 ? c.take<float>(N0 * R) : nullptr;
  g->partials = c.take<double>((size_t)kMaxDotParts * R);  // >= kReduceBlocks
  {  // the most workgroups a level-0 streaming launch can have (z-chunk 1)
    int np = 0;
    for (bool f32 : {false, true})
      for (int sh = 0; sh < stream_shapes(f32); ++sh) np = std::max(np, stream_blocks(g->lv[0], f32, sh, 1));
    g->big_parts_n = np > kMaxDotParts ? np : 0;
    g->big_parts = np > kMaxDotParts ? c.take<double>((size_t)np * R) : nullptr;
  }
  g->partials2 = c.take<double>(kReduceBlocks * R);
  g->scalars = c.take<double>(kScalars * R);
  g->flags = c.take<int>(kReduceBlocks + 1);
  g->active = c.take<int>(R);
  g->repl = c.take<int>(R);
  g->oc_partials = c.take<double>((size_t)kReduceBlocks * kOcProbes);
  g->oc_vol = c.take<double>(kOcProbes);
  g->galerkin = g->desc.coarse_op == HEXMG_COARSE_GALERKIN && L > 1;
  g->S64.assign(L, nullptr);
  g->S32.assign(L, nullptr);
  g->S16.assign(L, nullptr);
  g->Sexp.assign(L, nullptr);
  g->Gc = c.take<double>(8 * 576);
  if (g->galerkin) {
    // binary64 stencils for the set-up (and binary64 V-cycles); the binary32
    // V-cycle's copy in its storage precision
    const int store = g->desc.stencil_storage;
    for (int l = 1; l < L; ++l) {
      const size_t nq = 243ull * g->lv[l].nn;
      g->S64[l] = c.take<double>(nq);
      if (store == HEXMG_STENCIL_F32) g->S32[l] = c.take<float>(nq);  // binary32 K u at any precision
      if (v32 && store != HEXMG_STENCIL_F32) g->S16[l] = c.take<uint16_t>(nq);
      if (v32 && store == HEXMG_STENCIL_F16) g->Sexp[l] = c.take<int8_t>(g->lv[l].nn);
    }
  }
  return c.off + 256;
}

// ---- profiling ------------------------------------------------------------
int family_of(int mode, bool f32) {
  return 2 * mode + (f32 ? 1 : 0);  // apply 0/1, smooth 2/3, residual 4/5
}

hipEvent_t take_event(hexmg_grid* g) {
  if (!g->event_pool.empty()) {
    hipEvent_t e = g->event_pool.back();
    g->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// z-chunk of the streaming kernel: enough workgroups to fill the chip
// (about 1024), at least 4 and at most 64 planes per chunk.
int stream_zchunk(const Level& L, bool f32, int shape) {
  const int rows = stream_out_rows(f32, shape);
  const long long tiles = (long long)((L.nxn + 61) / 62) * ((L.nyn + rows - 1) / rows);
  long long zc = (L.nzn * tiles + 1023) / 1024;
  if (zc < 4) zc = 4;
  if (zc > 64) zc = 64;
  return (int)zc;
}

// maskin: u may be non-zero at fixed DOFs (the public K u); every vector
// inside the solver is zero there, so the streaming kernel can skip masking it.
template <typename T>
void launch_choice_now(hexmg_grid* g, const hexmg_grid::Choice& ch, int mode, int level, const T* u, const T* f,
                       const T* wd, T* y, int nrhs, hipStream_t s, bool maskin = false, const int* act = nullptr,
                       const LaunchTimer& t = {}, double* dotp = nullptr) {
  const bool f32 = sizeof(T) == 4;
  const T* Ke = f32 ? (const T*)g->Ke32 : (const T*)g->Ke64;
  const T* E = f32 ? (const T*)g->E32[level] : (const T*)g->E64[level];
  const Level& L = g->lv[level];
  if (g->galerkin && level > 0) {
    if constexpr (sizeof(T) == 4) {
      if (g->S16[level])
        launch_stencil16(g->desc.stencil_storage, mode, L, g->S16[level], g->Sexp[level], u, f, wd, y, nrhs, act, s,
                         t);
      else
        launch_stencil<T>(mode, L, g->S32[level], u, f, wd, y, nrhs, act, s, t);
    } else {
      launch_stencil<T>(mode, L, g->S64[level], u, f, wd, y, nrhs, act, s, t);
    }
  } else if (ch.kernel == HEXMG_KERNEL_GATHER) {
    launch_gather<T>(mode, L, Ke, E, u, f, wd, y, nrhs, act, s, t);
  } else {
    const HaarCoef<T>& q = *reinterpret_cast<const HaarCoef<T>*>(f32 ? (const void*)&g->hq32 : (const void*)&g->hq64);
    launch_stream<T>(mode, maskin, ch.shape, L, q, E, u, f, wd, y, ch.zchunk, nrhs, act, s, t, dotp);
  }
}

// The element-product launch of (mode, level) with kernel choice ch; while the
// grid is batched it is recorded (at stage g->stage), the streaming kernel as a
// batchable task.
template <typename T>
void launch_choice(hexmg_grid* g, const hexmg_grid::Choice& ch, int mode, int level, const T* u, const T* f,
                   const T* wd, T* y, int nrhs, hipStream_t s, bool maskin = false, const int* act = nullptr,
                   const LaunchTimer& t = {}, double* dotp = nullptr) {
  if (!g->rec) {
    launch_choice_now<T>(g, ch, mode, level, u, f, wd, y, nrhs, s, maskin, act, t, dotp);
    return;
  }
  const bool f32 = sizeof(T) == 4;
  const Level L = g->lv[level];
  if (ch.kernel == HEXMG_KERNEL_STREAM && !(g->galerkin && level > 0) && !maskin) {
    const HaarCoef<T> q = *reinterpret_cast<const HaarCoef<T>*>(f32 ? (const void*)&g->hq32 : (const void*)&g->hq64);
    const T* E = f32 ? (const T*)g->E32[level] : (const T*)g->E64[level];
    StreamTask<T> task{};
    task.L = L;
    task.E = E;
    task.u = u;
    task.f = f;
    task.wd = wd;
    task.y = y;
    task.act = act;
    task.dotp = dotp;
    task.zchunk = ch.zchunk;
    stream_grid(L, f32, ch.shape, ch.zchunk, &task.gx, &task.gy, &task.nchunks);
    const int shape = ch.shape, zc = ch.zchunk;
    const bool pre = zc == 1, dot = dotp != nullptr;
    emit_task<StreamTask<T>>(
        g, g->stage, s, batch_sig(kBkStream, sizeof(T), mode, shape, pre, dot) | ((unsigned long long)g->rec_class << 48),
        task,
        task.gx * task.gy * task.nchunks * nrhs,
        [=](hipStream_t st) {
          launch_stream<T>(mode, false, shape, L, q, E, u, f, wd, y, zc, nrhs, act, st, LaunchTimer{}, dotp);
        },
        [=](const Batch<StreamTask<T>>& b, hipStream_t st) { launch_stream_batch<T>(mode, shape, pre, dot, b, q, st); });
    return;
  }
  const hexmg_grid::Choice c = ch;
  emit_launch(g, g->stage, s, [=](hipStream_t st) {
    launch_choice_now<T>(g, c, mode, level, u, f, wd, y, nrhs, st, maskin, act, LaunchTimer{}, dotp);
  });
}

// Times the candidate kernels of one level in one precision in each of the
// three modes (K u, damped-Jacobi sweep, residual; zero vectors, the level's
// own scratch buffers) and keeps the fastest per mode.  The streaming kernel
// is kept unless the node-gather is more than 5% faster.
// modes: how many of the three modes to time (1 = K u only; f and wd may then
// be null).
template <typename T>
int tune_level(hexmg_grid* g, int level, T* u, T* f, T* y, const T* wd, std::array<hexmg_grid::Choice, 3>* out,
               hipStream_t s, int modes = 3) {
  const Level& L = g->lv[level];
  const size_t bytes = 3ull * L.nn * sizeof(T);
  HIP_TRY(hipMemsetAsync(u, 0, bytes, s));
  if (f) HIP_TRY(hipMemsetAsync(f, 0, bytes, s));
  const bool f32 = sizeof(T) == 4;
  // the mixed form's binary64 K p reads the binary32 direction: its own kernels are timed
  const bool u32in = !f32 && modes == 1 && g->desc.precision == HEXMG_MIXED;
  if (u32in) HIP_TRY(hipMemsetAsync(g->p32, 0, 3ull * L.nn * sizeof(float), s));
  auto run = [&](const hexmg_grid::Choice& c, int mode) {
    if constexpr (sizeof(T) == 8) {
      if (u32in) {
        const HaarCoef<double> q = *reinterpret_cast<const HaarCoef<double>*>(&g->hq64);
        if (c.kernel == HEXMG_KERNEL_STREAM)
          launch_apply_u32(c.shape, L, q, g->E64[level], g->p32, y, c.zchunk, 1, nullptr, s);
        else
          launch_gather_apply_u32(L, g->Ke64, g->E64[level], g->p32, y, 1, nullptr, s);
        return;
      }
    }
    launch_choice<T>(g, c, mode, level, u, f, wd, y, 1, s);
  };
  std::vector<hexmg_grid::Choice> cand;
  for (int sh = 0; sh < stream_shapes(f32); ++sh)
    for (int zc : {1, 2, 4, 8, 16, 32, 64, 128})
      if ((zc <= L.nzn || zc == 2) && (long long)((L.nzn + zc - 1) / zc) * g->desc.max_nrhs <= 65535)
        cand.push_back({HEXMG_KERNEL_STREAM, zc, sh});
  cand.push_back({HEXMG_KERNEL_GATHER, 0, 0});
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (int mode = 0; mode < modes; ++mode) {
    float best_stream = 1e30f, best_gather = 1e30f;
    hexmg_grid::Choice bs{HEXMG_KERNEL_STREAM, 4, 0};
    // small levels run for a few microseconds per launch: more repetitions
    // keep the timer's noise below the differences between candidates
    const int reps = L.ne < 100000 ? 12 : 3;
    for (const auto& c : cand) {
      run(c, mode);
      HIP_TRY(hipEventRecord(e0, s));
      for (int rep = 0; rep < reps; ++rep) run(c, mode);
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (c.kernel == HEXMG_KERNEL_GATHER) {
        best_gather = ms;
      } else if (ms < best_stream) {
        best_stream = ms;
        bs = c;
      }
    }
    (*out)[mode] = (best_gather < 0.95f * best_stream) ? hexmg_grid::Choice{HEXMG_KERNEL_GATHER, 0, 0} : bs;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 0;
}

// Every level and mode of the precisions whose V-cycle vectors the grid holds
// (they serve as scratch); without binary64 ones, the level-0 binary64 K u
// (outer product and true residual) on the CG vectors p and q.
int tune_kernels(hexmg_grid* g, hipStream_t s) {
  for (int l = 0; l < (g->galerkin ? 1 : g->L); ++l) {
    if (g->vu64[l]) {
      if (int e = tune_level<double>(g, l, g->vu64[l], g->vf64[l], g->vt64[l], g->wd64[l], &g->choice64[l], s))
        return e;
    } else if (l == 0) {
      if (int e = tune_level<double>(g, 0, g->r, nullptr, g->q, nullptr, &g->choice64[0], s, 1)) return e;
    }
    if (g->vu32[l])
      if (int e = tune_level<float>(g, l, g->vu32[l], g->vf32[l], g->vt32[l], g->wd32[l], &g->choice32[l], s))
        return e;
  }
  g->tuned = true;
  return 0;
}

template <typename T>
void gather(hexmg_grid* g, int mode, int level, const T* u, const T* f, const T* wd, T* y, int nrhs,
            hipStream_t s, bool maskin = false, const int* act = nullptr, double* dotp = nullptr) {
  const bool f32 = sizeof(T) == 4;
  hipEvent_t a = nullptr, b = nullptr;
  const bool prof = g->profile && level == 0 && !g->rec;
  if (prof) {
    a = take_event(g);
    b = take_event(g);
  }
  LaunchTimer t;
  if (a && b) t = LaunchTimer{a, b};
  const int cm = mode == kSmoothFirst ? kSmooth : mode;  // the sweep's kernel choice
  launch_choice<T>(g, (f32 ? g->choice32[level] : g->choice64[level])[cm], mode, level, u, f, wd, y, nrhs, s, maskin,
                   act, t, dotp);
  if (a && b) g->recs.push_back({family_of(mode, f32), a, b, g->prof_tag});
}

// y = A u at level 0 in binary64 on u, a binary32 search direction of the
// mixed form (the level's binary64 K u choice; recorded as a batchable task
// while the grid is batched).
void apply_p32(hexmg_grid* g, const float* u, double* y, int nrhs, hipStream_t s, const int* act, double* dotp) {
  const hexmg_grid::Choice ch = g->choice64[0][kApply];
  const Level L = g->lv[0];
  const double* E = g->E64[0];
  const double* Ke = g->Ke64;
  const HaarCoef<double> q = *reinterpret_cast<const HaarCoef<double>*>(&g->hq64);
  if (g->rec) {
    if (ch.kernel == HEXMG_KERNEL_STREAM) {
      StreamTask<double> task{};
      task.L = L;
      task.E = E;
      task.u32 = u;
      task.y = y;
      task.act = act;
      task.dotp = dotp;
      task.zchunk = ch.zchunk;
      stream_grid(L, false, ch.shape, ch.zchunk, &task.gx, &task.gy, &task.nchunks);
      const int shape = ch.shape, zc = ch.zchunk;
      const bool pre = zc == 1, dot = dotp != nullptr;
      emit_task<StreamTask<double>>(
          g, g->stage, s,
          batch_sig(kBkStreamU32, sizeof(double), kApply, shape, pre, dot) | ((unsigned long long)g->rec_class << 48),
          task, task.gx * task.gy * task.nchunks * nrhs,
          [=](hipStream_t st) { launch_apply_u32(shape, L, q, E, u, y, zc, nrhs, act, st, LaunchTimer{}, dotp); },
          [=](const Batch<StreamTask<double>>& b, hipStream_t st) {
            launch_stream_batch<double>(kApply, shape, pre, dot, b, q, st, true);
          });
    } else {
      emit_launch(g, g->stage, s,
                  [=](hipStream_t st) { launch_gather_apply_u32(L, Ke, E, u, y, nrhs, act, st, LaunchTimer{}); });
    }
    return;
  }
  hipEvent_t a = nullptr, b = nullptr;
  if (g->profile) {
    a = take_event(g);
    b = take_event(g);
  }
  LaunchTimer t;
  if (a && b) t = LaunchTimer{a, b};
  if (ch.kernel == HEXMG_KERNEL_STREAM)
    launch_apply_u32(ch.shape, L, q, E, u, y, ch.zchunk, nrhs, act, s, t, dotp);
  else
    launch_gather_apply_u32(L, Ke, E, u, y, nrhs, act, s, t);
  if (a && b) g->recs.push_back({family_of(kApply, false), a, b, g->prof_tag});
}

// drops the records of launches tagged with a CG iteration beyond last_its
void prune_profile(hexmg_grid* g, int last_its) {
  std::vector<hexmg_grid::Rec> keep;
  for (auto& r : g->recs) {
    if (r.tag > last_its) {
      g->event_pool.push_back(r.a);
      g->event_pool.push_back(r.b);
    } else {
      keep.push_back(r);
    }
  }
  g->recs.swap(keep);
}

void drain_profile(hexmg_grid* g) {
  for (auto& r : g->recs) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.b);
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g->prof_ms[r.family] += ms;
      g->prof_count[r.family] += 1;
    }
    g->event_pool.push_back(r.a);
    g->event_pool.push_back(r.b);
  }
  g->recs.clear();
}

// ---- V-cycle (Alg. 3) -----------------------------------------------------
template <typename T>
struct VView {
  std::vector<T*> f, u, t, r;
  std::vector<const T*> wd;
};

VView<double> view64(hexmg_grid* g) {
  VView<double> v{g->vf64, g->vu64, g->vt64, g->vr64, {}};
  for (auto p : g->wd64) v.wd.push_back(p);
  return v;
}
VView<float> view32(hexmg_grid* g) {
  VView<float> v{g->vf32, g->vu32, g->vt32, g->vr32, {}};
  for (auto p : g->wd32) v.wd.push_back(p);
  return v;
}

template <typename T>
CoarseCycle<T> make_cycle(hexmg_grid* g) {
  CoarseCycle<T> a{};
  for (int l = 0; l < g->L; ++l) {
    a.lv[l] = g->lv[l];
    if constexpr (sizeof(T) == 4) {
      a.E[l] = g->E32[l];
      a.wd[l] = g->wd32[l];
      a.u[l] = g->vu32[l];
      a.t[l] = g->vt32[l];
      a.r[l] = g->vr32[l];
      a.f[l] = g->vf32[l];
    } else {
      a.E[l] = g->E64[l];
      a.wd[l] = g->wd64[l];
      a.u[l] = g->vu64[l];
      a.t[l] = g->vt64[l];
      a.r[l] = g->vr64[l];
      a.f[l] = g->vf64[l];
    }
  }
  if constexpr (sizeof(T) == 4)
    a.Ke = g->Ke32;
  else
    a.Ke = g->Ke64;
  a.Ainv = g->Ainv;
  a.nc = g->nc;
  a.L = g->L;
  a.nu = g->desc.smooth_sweeps;
  return a;
}

// Orders stream s after the coarsest inverse of the last hexmg_set_density
// (formed on the auxiliary stream); a no-op once s has waited.
void wait_coarse(hexmg_grid* g, hipStream_t s) {
  if (!g->coarse_pending || (g->coarse_waited_valid && g->coarse_waited == s)) return;
  (void)hipStreamWaitEvent(s, g->ev_coarse, 0);
  g->coarse_waited = s;
  g->coarse_waited_valid = true;
}

// Whether the level-0 pre-smoothing forms the first sweep from zero on load
// (kSmoothFirst: the second sweep reads f and omega/D instead of the first's
// output), so that the CG residual update writes no first sweep: two or more
// sweeps, and a streaming sweep kernel with such a form.
template <typename T>
bool first_fused(const hexmg_grid* g) {
  if (!g->desc.fuse_first || g->L < 2 || g->desc.smooth_sweeps < 2) return false;
  const hexmg_grid::Choice& ch = (sizeof(T) == 4 ? g->choice32 : g->choice64)[0][kSmooth];
  return ch.kernel == HEXMG_KERNEL_STREAM && first_shape_ok(sizeof(T) == 4, ch.shape);
}

// out = V_l(f) from a zero initial guess.  The first sweep writes the level's
// scratch vector and the 2*nu-1 further sweeps alternate, so the result lands
// in `out` without a copy.  f and out must not overlap.  With first_done the
// caller has already written the first sweep (omega D^-1 f) into the scratch
// vector.  act: per right-hand side skip flags (may be null).  maskin: f may be
// non-zero at fixed DOFs, so this level's element products mask their input
// (the deeper levels' right-hand sides come out of the masked restriction).
template <typename T>
void vcycle_level(hexmg_grid* g, VView<T>& v, int l, const T* f, T* out, int nrhs, const int* act, hipStream_t s,
                  bool first_done = false, bool maskin = false, double* dotp = nullptr) {
  const Level& L = g->lv[l];
  if (l == g->L - 1) {
    wait_coarse(g, s);
    const int nc = g->nc;
    const double* Ainv = g->Ainv;
    GemvTask<T> task{nc, Ainv, f, out, act, gemv_blocks(nc)};
    emit_task<GemvTask<T>>(
        g, kStCoarse, s, batch_sig(kBkGemv, sizeof(T)), task, task.gx * nrhs,
        [=](hipStream_t st) { launch_coarse_gemv<T>(nc, Ainv, f, out, nrhs, act, st); },
        [](const Batch<GemvTask<T>>& b, hipStream_t st) { launch_coarse_gemv_batch<T>(b, st); });
    return;
  }
  const long long N = 3ll * L.nn;
  const int nu = g->desc.smooth_sweeps;
  T* buf[2] = {v.t[l], out};
  int cur = 0;
  // level 0: the second sweep may form the first from f (first_fused); the
  // first sweep's output is then neither written nor read
  const bool first = l == 0 && !maskin && first_fused<T>(g);
  if (!first_done && !first) {
    const T* wdl = v.wd[l];
    T* t0 = buf[0];
    emit_launch(g, st_down(l, 0), s,
                [=](hipStream_t st) { launch_jacobi_first<T>(N, wdl, f, t0, nrhs, act, st); });
  }
  for (int it = 1; it < nu; ++it) {
    g->stage = st_down(l, it);
    gather<T>(g, it == 1 && first ? kSmoothFirst : kSmooth, l, buf[cur], f, v.wd[l], buf[1 - cur], nrhs, s, maskin,
              act);
    cur = 1 - cur;
  }
  g->stage = st_down(l, 90);
  gather<T>(g, kResidual, l, buf[cur], f, v.wd[l], v.r[l], nrhs, s, maskin, act);
  // the next level's first sweep is formed inside the restriction (not on the coarsest level)
  const bool fuse = l + 1 < g->L - 1;
  {
    const Level F = L, C = g->lv[l + 1];
    RestrictTask<T> task{F, C, v.r[l], v.f[l + 1], act, fuse ? v.wd[l + 1] : nullptr, fuse ? v.t[l + 1] : nullptr,
                         restrict_blocks(C)};
    emit_task<RestrictTask<T>>(
        g, st_down(l, 95), s, batch_sig(kBkRestrict, sizeof(T)), task, task.gx * nrhs,
        [=](hipStream_t st) { launch_restrict<T>(F, C, task.r, task.fc, nrhs, act, st, task.wdc, task.tc); },
        [](const Batch<RestrictTask<T>>& b, hipStream_t st) { launch_restrict_batch<T>(b, st); });
  }
  int& tail = sizeof(T) == 4 ? g->tail32 : g->tail64;
  const int blocks = sizeof(T) == 4 ? g->tail_blocks32 : g->tail_blocks64;
  bool done = false;
  if (fuse && tail == l + 1) {  // the rest of the cycle as one cooperative launch
    wait_coarse(g, s);
    done = launch_coarse_cycle<T>(make_cycle<T>(g), l + 1, nrhs, act, blocks, s) == hipSuccess;
    if (!done) {
      (void)hipGetLastError();
      tail = 0;  // not launchable here: back to one launch per step from now on
    }
  }
  if (!done) vcycle_level<T>(g, v, l + 1, v.f[l + 1], v.u[l + 1], nrhs, act, s, fuse);
  {
    const Level F = L, C = g->lv[l + 1];
    ProlongTask<T> task{F, C, v.u[l + 1], buf[cur], act, prolong_blocks(F)};
    emit_task<ProlongTask<T>>(
        g, st_up(l, 0), s, batch_sig(kBkProlong, sizeof(T)), task, task.gx * nrhs,
        [=](hipStream_t st) { launch_prolong_add<T>(F, C, task.ec, task.u, nrhs, act, st); },
        [](const Batch<ProlongTask<T>>& b, hipStream_t st) { launch_prolong_add_batch<T>(b, st); });
  }
  for (int it = 0; it < nu; ++it) {
    g->stage = st_up(l, 1 + it);
    gather<T>(g, kSmooth, l, buf[cur], f, v.wd[l], buf[1 - cur], nrhs, s, maskin, act, it == nu - 1 ? dotp : nullptr);
    cur = 1 - cur;
  }
}

// Partials per right-hand side of f . out formed inside the last level-0
// sweep of the V-cycle (its streaming kernel), or 0 where that sweep cannot
// form them (no sweep, the node-gather kernel, too many workgroups).
template <typename T>
int sweep_dot_parts(const hexmg_grid* g) {
  if (g->L < 2) return 0;
  const hexmg_grid::Choice& ch = (sizeof(T) == 4 ? g->choice32 : g->choice64)[0][kSmooth];
  if (ch.kernel != HEXMG_KERNEL_STREAM) return 0;
  const int nb = stream_blocks(g->lv[0], sizeof(T) == 4, ch.shape, ch.zchunk);
  return nb <= kMaxDotParts || nb <= g->big_parts_n ? nb : 0;
}

// Where a level-0 launch with nb workgroups writes its per-workgroup partials:
// straight into the consumer's buffer, or (more than a vector kernel's block
// sums itself) into big_parts, summed by one more small launch (sum_big).
double* parts_target(hexmg_grid* g, int nb, double* consumer) {
  return nb <= kMaxDotParts ? consumer : g->big_parts;
}
// returns the number of partials the consumer then sums per right-hand side
int sum_big(hexmg_grid* g, int nb, double* consumer, int nrhs, const int* act, int stage, hipStream_t s) {
  if (nb <= kMaxDotParts) return nb;
  const double* parts = g->big_parts;
  emit_launch(g, stage, s, [=](hipStream_t st) { launch_sum_parts(parts, nb, consumer, nrhs, act, st); });
  return 1;
}

// Times the rest of the V-cycle from each level ls >= 1 launched step by step
// against the cooperative launch (several workgroup counts) and keeps the
// cooperative launch from the level where it saves the most, if it saves more
// than 5% there.
template <typename T>
int tune_tail(hexmg_grid* g, hipStream_t s) {
  const bool f32 = sizeof(T) == 4;
  int& tail = f32 ? g->tail32 : g->tail64;
  int& tblocks = f32 ? g->tail_blocks32 : g->tail_blocks64;
  tail = 0;
  tblocks = 0;
  const int maxb = coarse_cycle_max_blocks<T>();
  if (g->L < 3 || maxb <= 0 || g->galerkin) return 0;
  if ((f32 ? (const void*)g->vu32[0] : (const void*)g->vu64[0]) == nullptr) return 0;  // precision not held
  VView<T> v = [&] {
    if constexpr (sizeof(T) == 4)
      return view32(g);
    else
      return view64(g);
  }();
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto time3 = [&](auto&& fn, float* ms) -> int {
    fn();
    HIP_TRY(hipEventRecord(e0, s));
    for (int rep = 0; rep < 3; ++rep) fn();
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    return 0;
  };
  float best_gain = 0.f;
  const CoarseCycle<T> cyc = make_cycle<T>(g);
  for (int ls = 1; ls <= g->L - 2; ++ls) {
    const size_t bytes = 3ull * g->lv[ls].nn * sizeof(T);
    HIP_TRY(hipMemsetAsync(v.f[ls], 0, bytes, s));
    HIP_TRY(hipMemsetAsync(v.t[ls], 0, bytes, s));
    float ms_launch = 0.f;
    if (int e = time3([&] { vcycle_level<T>(g, v, ls, v.f[ls], v.u[ls], 1, nullptr, s, true); }, &ms_launch))
      return e;
    int prev = -1;
    for (int b : {64, 128, 256, 512, 1024}) {
      b = b < maxb ? b : maxb;
      if (b == prev) continue;
      prev = b;
      bool ok = true;
      float ms = 0.f;
      wait_coarse(g, s);
      if (int e = time3([&] { ok = ok && launch_coarse_cycle<T>(cyc, ls, 1, nullptr, b, s) == hipSuccess; }, &ms))
        return e;
      if (!ok) {
        (void)hipGetLastError();
        continue;
      }
      const float gain = ms_launch - ms;
      if (gain > 0.05f * ms_launch && gain > best_gain) {
        best_gain = gain;
        tail = ls;
        tblocks = b;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 0;
}

// z = M^{-1} r (the V-cycle in the grid's precision) for nrhs <= max_nrhs
// binary64 right-hand sides, and the partials of r . z; returns how many
// partials each right-hand side has (kReduceBlocks apart from fuse_dot).  In
// mixed precision the binary32 right-hand side is formed inside the first
// sweep, and z is written in binary64 only with write_z; otherwise it stays in
// the binary32 buffer g->vu32[0] (the CG update widens it on the fly).  With
// first_done the first sweep (and in mixed precision the binary32 copy of r)
// was already written by the CG residual update.  With fuse_dot the partials
// come from the last level-0 sweep where it can form them (in mixed precision
// as the binary32 copy of r, which the V-cycle consumes, times z), the
// returned count apart.
int precondition(hexmg_grid* g, const double* r, double* z, double* rz_partials, int nrhs, const int* act,
                 hipStream_t s, bool write_z = true, bool first_done = false, bool fuse_dot = false) {
  const long long N = 3ll * g->lv[0].nn;
  if (g->desc.precision == HEXMG_FP64) {
    VView<double> v = view64(g);
    const int nd = fuse_dot ? sweep_dot_parts<double>(g) : 0;
    vcycle_level<double>(g, v, 0, r, z, nrhs, act, s, first_done, false,
                         nd ? parts_target(g, nd, rz_partials) : nullptr);
    if (nd) return sum_big(g, nd, rz_partials, nrhs, act, kStEnd, s);
    emit_launch(g, kStEnd, s, [=](hipStream_t st) { launch_dot_partial(N, r, z, rz_partials, nrhs, act, st); });
    return kReduceBlocks;
  }
  VView<float> v = view32(g);
  const int nd = fuse_dot && !write_z ? sweep_dot_parts<float>(g) : 0;
  float* f32 = g->vf32[0];
  float* u32 = g->vu32[0];
  if (g->L == 1) {  // the coarsest level is the whole grid: no sweep to fuse into
    if (!first_done)
      emit_launch(g, st_down(0, 0), s, [=](hipStream_t st) { launch_f64_to_f32(N, r, f32, nrhs, act, st); });
    vcycle_level<float>(g, v, 0, f32, u32, nrhs, act, s);
  } else {
    if (!first_done) {
      const float* wd = g->wd32[0];
      float* t32 = g->vt32[0];
      if (first_fused<float>(g))  // the second sweep forms the first: only the binary32 copy of r
        emit_launch(g, st_down(0, 0), s, [=](hipStream_t st) { launch_f64_to_f32(N, r, f32, nrhs, act, st); });
      else
        emit_launch(g, st_down(0, 0), s,
                    [=](hipStream_t st) { launch_jacobi_first_from64(N, wd, r, f32, t32, nrhs, act, st); });
    }
    vcycle_level<float>(g, v, 0, f32, u32, nrhs, act, s, true, false,
                        nd ? parts_target(g, nd, rz_partials) : nullptr);
  }
  if (nd) return sum_big(g, nd, rz_partials, nrhs, act, kStEnd, s);
  if (write_z)
    emit_launch(g, kStEnd, s, [=](hipStream_t st) { launch_to64_dot(N, u32, r, z, rz_partials, nrhs, act, st); });
  else
    emit_launch(g, kStEnd, s, [=](hipStream_t st) { launch_dot_mixed(N, u32, r, rz_partials, nrhs, act, st); });
  return kReduceBlocks;
}

// out[r * kScalars] = x_r . y_r for each right-hand side r
void dot(hexmg_grid* g, long long n, const double* x, const double* y, double* out, int nrhs, hipStream_t s) {
  launch_dot_partial(n, x, y, g->partials, nrhs, nullptr, s);
  launch_reduce_final(g->partials, out, kScalars, nrhs, s);
}

int read_scalars(hexmg_grid* g, int nrhs, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(g->host_scalars, g->scalars, (size_t)kScalars * nrhs * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

}  // namespace

extern "C" {

int hexmg_default_desc(int nx, int ny, int nz, int levels, hexmg_grid_desc* d) {
  if (!d) return fail(HEXMG_ERR_INVALID, "null descriptor");
  std::memset(d, 0, sizeof(*d));
  d->nx = nx;
  d->ny = ny;
  d->nz = nz;
  d->levels = levels;
  d->E0 = 1.0;
  d->Emin = 1e-9;
  d->nu = 0.3;
  d->penal = 3.0;
  d->precision = HEXMG_FP64;
  d->smooth_sweeps = 2;
  d->omega = 0.0;  // automatic: by coarse operator at grid creation
  d->coarse_avg = HEXMG_AVG_DENSITY;
  d->max_nrhs = 1;
  d->kernel = HEXMG_KERNEL_AUTO;
  d->fixed_mask = nullptr;
  d->vcycle_both = 0;
  d->rr_every = 8;
  d->fuse_first = 1;
  return 0;
}

int hexmg_workspace_size(const hexmg_grid_desc* d, size_t* bytes) {
  if (int e = validate(d)) return e;
  if (!bytes) return fail(HEXMG_ERR_INVALID, "null bytes");
  hexmg_grid g;
  g.desc = *d;
  g.L = d->levels;
  make_levels(d, g.lv);
  *bytes = carve(&g, nullptr);
  return 0;
}

int hexmg_grid_create(const hexmg_grid_desc* d, void* workspace, size_t bytes, void* stream,
                      hexmg_grid_t* out) {
  if (int e = validate(d)) return e;
  if (!workspace || !out) return fail(HEXMG_ERR_INVALID, "null workspace or output");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(HEXMG_ERR_INVALID, "workspace must be 256-byte aligned");
  size_t need = 0;
  hexmg_workspace_size(d, &need);
  if (bytes < need) return fail(HEXMG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  hexmg_grid* g = new hexmg_grid();
  g->desc = *d;
  g->L = d->levels;
  make_levels(d, g->lv);
  carve(g, static_cast<char*>(workspace));
  for (int l = 0; l < g->L; ++l) g->lv[l].mask = g->mask[l];
  g->tuned = d->kernel != HEXMG_KERNEL_AUTO;
  g->choice64.assign(g->L, {});
  g->choice32.assign(g->L, {});
  for (int l = 0; l < g->L; ++l) {
    for (int m = 0; m < 3; ++m) {
      if (d->kernel == HEXMG_KERNEL_GATHER) {
        g->choice64[l][m] = {HEXMG_KERNEL_GATHER, 0, 0};
        g->choice32[l][m] = {HEXMG_KERNEL_GATHER, 0, 0};
      } else {
        g->choice64[l][m] = {HEXMG_KERNEL_STREAM, stream_zchunk(g->lv[l], false, 1), 1};
        g->choice32[l][m] = {HEXMG_KERNEL_STREAM, stream_zchunk(g->lv[l], true, 1), 1};
      }
    }
  }
  g->density_set = false;
  g->profile = false;
  g->Ainv = g->Abuf[0];
  g->last_stream = s;
  for (int i = 0; i < 8; ++i) {
    g->prof_ms[i] = 0.0;
    g->prof_count[i] = 0;
  }
  g->host_scalars = nullptr;
  auto cleanup = [&](int code) {
    if (g->host_scalars) (void)hipHostFree(g->host_scalars);
    delete g;
    return code;
  };
  {
    const size_t nsc = (size_t)kScalars * (d->max_nrhs > 8 ? d->max_nrhs : 8);
    const size_t nring = 3ull * kScalars * d->max_nrhs;
    if (hipHostMalloc((void**)&g->host_scalars, (nsc + nring) * sizeof(double), hipHostMallocDefault) != hipSuccess)
      return cleanup(fail(HEXMG_ERR_DEVICE, "pinned host allocation failed"));
    g->host_ring = g->host_scalars + nsc;
  }
  if (!haar_coefficients(d->nu, &g->hq64))
    return cleanup(fail(HEXMG_ERR_INVALID, "element stiffness does not have the expected Haar block pattern"));
  {
    const HaarCoef<double>& q = g->hq64;
    g->hq32 = HaarCoef<float>{(float)q.d1, (float)q.b1, (float)q.g, (float)q.a2,
                              (float)q.b2, (float)q.d3, (float)q.b3, (float)q.a4};
  }
  double Ke[576];
  float Kf[576];
  element_matrix(d->nu, Ke);
  for (int i = 0; i < 576; ++i) Kf[i] = (float)Ke[i];
  if (hipMemcpyAsync(g->Ke64, Ke, sizeof(Ke), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(g->Ke32, Kf, sizeof(Kf), hipMemcpyHostToDevice, s) != hipSuccess)
    return cleanup(fail(HEXMG_ERR_DEVICE, "copy of the element matrix failed"));
  g->Gc_host.resize(8 * 576);
  galerkin_child_matrices(Ke, g->Gc_host.data());
  if (hipMemcpyAsync(g->Gc, g->Gc_host.data(), g->Gc_host.size() * sizeof(double), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return cleanup(fail(HEXMG_ERR_DEVICE, "copy of the Galerkin child matrices failed"));
  if (d->fixed_mask) {
    if (hipMemcpyAsync(g->mask[0], d->fixed_mask, g->lv[0].nn, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return cleanup(fail(HEXMG_ERR_DEVICE, "copy of the support mask failed"));
  } else {
    launch_mask_default(g->lv[0], g->mask[0], s);
  }
  for (int l = 1; l < g->L; ++l) launch_mask_inject(g->lv[l - 1], g->lv[l], g->mask[l - 1], g->mask[l], s);
  g->desc.fixed_mask = nullptr;  // copied; do not keep the caller's pointer
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
    return cleanup(fail(HEXMG_ERR_DEVICE, "grid set-up kernels failed"));
  *out = g;
  return 0;
}

int hexmg_grid_destroy(hexmg_grid_t g) {
  if (!g) return 0;
  // Work queued on the library's own streams (the coarsest inverse on the
  // auxiliary stream, a batched solve's stream) still writes the caller's
  // workspace: let it finish before the caller may reuse that memory.
  if (g->aux_stream) (void)hipStreamSynchronize(g->aux_stream);
  if (g->own_stream) (void)hipStreamSynchronize(g->own_stream);
  if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
  if (g->aux_stream) (void)hipStreamDestroy(g->aux_stream);
  for (hipEvent_t e : {g->ev_fork, g->ev_coarse, g->ev_flag, g->ev_read})
    if (e) (void)hipEventDestroy(e);
  for (auto& r : g->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : g->event_pool) (void)hipEventDestroy(e);
  if (g->host_scalars) (void)hipHostFree(g->host_scalars);
  delete g;
  return 0;
}

int hexmg_set_density(hexmg_grid_t g, const double* rho, void* stream) {
  if (!g || !rho) return fail(HEXMG_ERR_INVALID, "null argument");
  hipStream_t s = (hipStream_t)stream;
  g->last_stream = s;
  const hexmg_grid_desc& d = g->desc;
  if (!g->aux_stream) {
    if (hipStreamCreateWithFlags(&g->aux_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_coarse, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_flag, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_read, hipEventDisableTiming) != hipSuccess)
      return fail(HEXMG_ERR_DEVICE, "stream or event creation failed");
  }
  // the previous coarsest inverse may still be in flight on the auxiliary stream
  if (g->coarse_pending) HIP_TRY(hipStreamWaitEvent(s, g->ev_coarse, 0));
  // Coarsest level on the auxiliary stream: its moduli straight from level 0
  // (or the Galerkin stencil, which needs the levels above), assembly,
  // Gauss-Jordan inverse, symmetrization; everything it reads is final when
  // it is forked.  With density averaging it reads the caller's rho and is
  // forked before the SIMP kernel; the stream then waits for that read before
  // later work (which may overwrite rho) is ordered after this call.
  const int nc = g->nc;
  hipStream_t a = g->aux_stream;
  const bool dens = d.coarse_avg == HEXMG_AVG_DENSITY;
  const bool early = !g->galerkin && g->L > 1 && dens;
  auto fork_coarsest = [&]() -> int {
    HIP_TRY(hipEventRecord(g->ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(a, g->ev_fork, 0));
    const Level& C = g->lv[g->L - 1];
    if (g->galerkin) {
      launch_dense_from_stencil(C, g->S64[g->L - 1], g->Abuf[0], a);
    } else {
      const double* Ec = g->E64[0];
      if (g->L > 1) {
        const double scale = double(1 << (g->L - 1));
        launch_coarsest_moduli(g->lv[0], C, 1 << (g->L - 1), dens ? (early ? rho : g->rho[0]) : g->E64[0], dens,
                               d.E0, d.Emin, d.penal, scale, g->Ecoarse, a);
        if (early) HIP_TRY(hipEventRecord(g->ev_read, a));
        Ec = g->Ecoarse;
      }
      launch_coarse_assemble(C, g->Ke64, Ec, g->Abuf[0], a);
    }
    double* inv = nullptr;
    launch_gj_blocked(nc, g->Abuf[0], g->Abuf[1], g->gjD, &inv, a);
    double* other = (inv == g->Abuf[0]) ? g->Abuf[1] : g->Abuf[0];
    launch_symmetrize(nc, inv, other, a);
    HIP_TRY(hipEventRecord(g->ev_coarse, a));
    g->Ainv = other;
    g->coarse_pending = true;
    g->coarse_waited_valid = false;
    return 0;
  };
  if (early)
    if (int e = fork_coarsest()) return e;
  launch_simp(g->lv[0].ne, rho, d.E0, d.Emin, d.penal, 1.0, g->E64[0], g->E32[0], g->rho[0], g->flags, s);
  if (!g->galerkin && !early)
    if (int e = fork_coarsest()) return e;
  launch_or_flags(kReduceBlocks, g->flags, g->flags + kReduceBlocks, s);
  HIP_TRY(hipMemcpyAsync(g->host_scalars, g->flags + kReduceBlocks, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(g->ev_flag, s));
  for (int l = 1; l < g->L; ++l) {
    launch_homogenize(g->lv[l - 1], g->lv[l], g->rho[l - 1], g->rho[l], s);
    if (d.coarse_avg == HEXMG_AVG_DENSITY)
      launch_modulus_from_density(g->lv[l].ne, g->rho[l], d.E0, d.Emin, d.penal, double(1 << l), g->E64[l],
                                  g->E32[l], s);
    else
      launch_modulus_from_mean(g->lv[l - 1], g->lv[l], g->E64[l - 1], 2.0, g->E64[l], g->E32[l], s);
  }
  if (g->galerkin) {  // Eq. 23 products, level by level, as stencils
    launch_galerkin_first(g->lv[0], g->lv[1], g->E64[0], g->Gc, g->Ke64, g->S64[1], g->S32[1], s);
    for (int l = 1; l + 1 < g->L; ++l)
      launch_galerkin_coarsen(g->lv[l], g->lv[l + 1], g->S64[l], g->S64[l + 1], g->S32[l + 1], s);
    for (int l = 1; l < g->L; ++l)
      if (g->S16[l]) launch_stencil_to16(d.stencil_storage, g->lv[l], g->S64[l], g->S16[l], g->Sexp[l], s);
    if (int e = fork_coarsest()) return e;
  }
  // omega 0 = automatic: 0.6 with re-discretized coarse operators, 0.5 with
  // Galerkin ones (on black-and-white designs the Galerkin hierarchy has
  // lambda_max(D^-1 A) of 4-6, where 0.6 lets damped Jacobi amplify the
  // highest modes)
  const double omega = d.omega > 0.0 ? d.omega : (g->galerkin ? 0.5 : 0.6);
  if (g->galerkin) {
    launch_diag(g->lv[0], g->Ke64, g->E64[0], omega, g->wd64[0], g->wd32[0], s);
    for (int l = 1; l < g->L; ++l) launch_stencil_diag(g->lv[l], g->S64[l], omega, g->wd64[l], g->wd32[l], s);
  } else {
    for (int l = 0; l < g->L; ++l) launch_diag(g->lv[l], g->Ke64, g->E64[l], omega, g->wd64[l], g->wd32[l], s);
  }
  if (early) HIP_TRY(hipStreamWaitEvent(s, g->ev_read, 0));
  HIP_TRY(hipGetLastError());
  // validity of rho: wait only for the flag, not for the set-up queued behind it
  int bad = 0;
  HIP_TRY(hipEventSynchronize(g->ev_flag));
  std::memcpy(&bad, g->host_scalars, sizeof(int));
  if (bad) {
    g->density_set = false;
    return fail(HEXMG_ERR_NONFINITE, "density outside [0,1] or not finite");
  }
  g->density_set = true;
  if (!g->tuned) {
    if (int e = tune_kernels(g, s)) return e;
  }
  if (!g->tail_tuned) {
    if (int e = tune_tail<double>(g, s)) return e;
    if (int e = tune_tail<float>(g, s)) return e;
    g->tail_tuned = true;
  }
  return 0;
}

int hexmg_apply_K(hexmg_grid_t g, int level, int dtype, const void* u, void* y, int nrhs, void* stream) {
  if (!g || !u || !y) return fail(HEXMG_ERR_INVALID, "null argument");
  if (level < 0 || level >= g->L) return fail(HEXMG_ERR_INVALID, "bad level");
  if (nrhs < 1) return fail(HEXMG_ERR_INVALID, "nrhs must be >= 1");
  if (!g->density_set) return fail(HEXMG_ERR_INVALID, "hexmg_set_density has not succeeded");
  hipStream_t s = (hipStream_t)stream;
  g->last_stream = s;
  if (nrhs > 65535) return fail(HEXMG_ERR_INVALID, "nrhs must be <= 65535");
  if (dtype == HEXMG_F32 && g->galerkin && level > 0 && !g->S32[level] && !g->S16[level])
    return fail(HEXMG_ERR_INVALID, "this grid holds no binary32 stencils (16-bit storage needs a binary32 V-cycle)");
  if (dtype == HEXMG_F64)
    gather<double>(g, kApply, level, (const double*)u, nullptr, nullptr, (double*)y, nrhs, s, true);
  else if (dtype == HEXMG_F32)
    gather<float>(g, kApply, level, (const float*)u, nullptr, nullptr, (float*)y, nrhs, s, true);
  else
    return fail(HEXMG_ERR_INVALID, "bad dtype");
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_vcycle(hexmg_grid_t g, int dtype, const void* r, void* z, int nrhs, void* stream) {
  if (!g || !r || !z) return fail(HEXMG_ERR_INVALID, "null argument");
  if (nrhs < 1) return fail(HEXMG_ERR_INVALID, "nrhs must be >= 1");
  if (!g->density_set) return fail(HEXMG_ERR_INVALID, "hexmg_set_density has not succeeded");
  if (r == z) return fail(HEXMG_ERR_INVALID, "r and z must not overlap");
  hipStream_t s = (hipStream_t)stream;
  g->last_stream = s;
  const long long N = 3ll * g->lv[0].nn;
  if (dtype != HEXMG_F64 && dtype != HEXMG_F32) return fail(HEXMG_ERR_INVALID, "bad dtype");
  if ((dtype == HEXMG_F64 ? (const void*)g->vu64[0] : (const void*)g->vu32[0]) == nullptr)
    return fail(HEXMG_ERR_INVALID, "the grid holds no V-cycle vectors of this dtype (create it with vcycle_both = 1)");
  for (int k = 0; k < nrhs; k += g->desc.max_nrhs) {
    const int nb = (nrhs - k) < g->desc.max_nrhs ? (nrhs - k) : g->desc.max_nrhs;
    if (dtype == HEXMG_F64) {
      VView<double> v = view64(g);
      vcycle_level<double>(g, v, 0, (const double*)r + k * N, (double*)z + k * N, nb, nullptr, s, false, true);
    } else {
      VView<float> v = view32(g);
      vcycle_level<float>(g, v, 0, (const float*)r + k * N, (float*)z + k * N, nb, nullptr, s, false, true);
    }
  }
  HIP_TRY(hipGetLastError());
  return 0;
}

}  // extern "C"

namespace {

// PCG (Alg. 1) for nb <= max_nrhs right-hand sides of one grid in lockstep.
// The CG scalars, the convergence test and the iteration counts live on the
// device (see ScalarSlot): every kernel skips right-hand sides whose active
// flag has been cleared, so the host can keep one iteration in flight while it
// reads the state of the previous one from a ring of three pinned slots.  The
// run is a resumable state machine so that several grids can advance together:
// advance() is called once wait_event() has completed.
struct PcgRun {
  hexmg_grid* g = nullptr;
  const double* f = nullptr;
  double* u = nullptr;
  int nb = 0;
  double rtol = 0.0;
  int maxit = 0;
  hipStream_t s = nullptr;
  hexmg_solve_info* info = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr}, t0 = nullptr, t1 = nullptr;
  enum Phase { kIterate, kFinish, kDone } phase = kIterate;
  int issued = 0, target = 0, final_slot = 0, status = 0;
  int limit = 0;    // host iteration number the run may not pass (maxit, moved by restarts)
  int tag_off = 0;  // host iteration number minus the device's, for profile tags after a restart
  int restarts = 0;
  std::vector<int> its_off;  // per right-hand side: host iteration number minus 1 minus its iterations so far
  std::vector<double> prev_rr;  // ||r||^2 of the last iteration read, per right-hand side

  int init() {
    for (auto& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    return 0;
  }
  void release() {
    if (g) g->prof_tag = 0;
    for (auto& e : ev) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    t0 = t1 = nullptr;
  }
  long long N() const { return 3ll * g->lv[0].nn; }
  double* slot(int k) const { return g->host_ring + (size_t)(k % 3) * kScalars * g->desc.max_nrhs; }
  hipEvent_t wait_event() const { return ev[(phase == kFinish ? final_slot : target) % 3]; }
  // the scalars of slot k reach the host by a copy (final phase) or, for a CG
  // iteration, written by the iteration's last kernel itself
  int post(int k, bool copy, int stage) {
    if (copy) {
      double* dst = slot(k);
      const double* src = g->scalars;
      const size_t bytes = (size_t)kScalars * nb * sizeof(double);
      HIP_TRY(emit_api(g, stage, s, [=](hipStream_t st) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
      }));
    }
    hipEvent_t e = ev[k % 3];
    HIP_TRY(emit_api(g, stage + 1, s, [=](hipStream_t st) { return hipEventRecord(e, st); }));
    return 0;
  }
  // iteration k (1-based): q = A p, alpha, the r update (its x update follows
  // in the next p update, or at the end), ||r||^2 and the test
  bool m32() const { return g->desc.precision == HEXMG_MIXED32; }
  // the mixed form's binary32 direction of iteration k (odd: p32, even: p32b)
  float* dir32(int k) const { return (k & 1) ? g->p32 : g->p32b; }
  int issue_iteration(int k) {
    double* sc = g->scalars;
    g->prof_tag = k - tag_off;
    // q = A p, with p . q formed inside the streaming kernel when it is the
    // level-0 choice and its workgroups are few enough; else a separate pass
    const bool f32 = m32();
    const hexmg_grid::Choice& ch = (f32 ? g->choice32 : g->choice64)[0][kApply];
    int npq = 0;
    if (ch.kernel == HEXMG_KERNEL_STREAM) {
      const int nbk = stream_blocks(g->lv[0], f32, ch.shape, ch.zchunk);
      if (nbk <= kMaxDotParts || nbk <= g->big_parts_n) npq = nbk;
    }
    g->stage = kStEnd + 200;
    double* pq_target = npq ? parts_target(g, npq, g->partials) : nullptr;
    if (f32)
      gather<float>(g, kApply, 0, g->p32, nullptr, nullptr, g->q32, nb, s, false, g->active, pq_target);
    else if (!g->p)  // mixed form: binary64 product on the binary32 direction
      apply_p32(g, dir32(k), g->q, nb, s, g->active, pq_target);
    else
      gather<double>(g, kApply, 0, g->p, nullptr, nullptr, g->q, nb, s, false, g->active, pq_target);
    if (npq) npq = sum_big(g, npq, g->partials, nb, g->active, kStEnd + 205, s);
    if (!npq) {
      const long long n = N();
      const int b = nb;
      double *p = g->p, *q = g->q, *parts = g->partials;
      float* q32 = g->q32;
      const float* p32 = f32 ? g->p32 : dir32(k);
      const int* act = g->active;
      if (f32)
        emit_launch(g, kStEnd + 210, s, [=](hipStream_t st) { launch_dot_mixed(n, q32, p, parts, b, act, st); });
      else if (!p)
        emit_launch(g, kStEnd + 210, s, [=](hipStream_t st) { launch_dot_mixed(n, p32, q, parts, b, act, st); });
      else
        emit_launch(g, kStEnd + 210, s, [=](hipStream_t st) { launch_dot_partial(n, p, q, parts, b, act, st); });
      npq = kReduceBlocks;
    }
    // r -= alpha q with the next preconditioner's first sweep (x += alpha p follows in the p update)
    const bool sweep = g->L > 1;
    if (g->desc.precision == HEXMG_FP64) {
      emit_update_r<double, double>(npq, (k - 1) & 1, g->q, g->wd64[0], nullptr,
                                    sweep && !first_fused<double>(g) ? g->vt64[0] : nullptr, nullptr);
    } else if (!f32) {
      emit_update_r<float, double>(npq, (k - 1) & 1, g->q, g->wd32[0], g->vf32[0],
                                   sweep && !first_fused<float>(g) ? g->vt32[0] : nullptr, nullptr);
    } else {
      // binary32 A p; every rr_every-th iteration of a right-hand side its
      // residual is replaced by the binary64 M f - A x (x brought up to date
      // first).  The device decides per right-hand side from its own
      // iteration count (flags in repl); the host launches the replacement
      // kernels only in iterations where some right-hand side may need them.
      const int every = g->desc.rr_every;
      bool replace = false;
      for (int r = 0; r < nb && every > 0; ++r) replace = replace || (k - its_off[r]) % every == 0;
      const int b = nb;
      const long long n = N();
      int* repl = g->repl;
      const int* act = g->active;
      if (replace)
        emit_launch(g, kStEnd + 220, s,
                    [=](hipStream_t st) { launch_replace_flags(sc, act, repl, b, every, st); });
      emit_update_r<float, float>(npq, (k - 1) & 1, g->q32, g->wd32[0], g->vf32[0],
                                  sweep && !first_fused<float>(g) ? g->vt32[0] : nullptr, replace ? g->repl : nullptr);
      if (replace) {
        double* p = g->p;
        double* x = u;
        emit_launch(g, kStEnd + 310, s, [=](hipStream_t st) { launch_flush_x(n, sc, p, x, b, st, repl); });
        g->stage = kStEnd + 320;
        gather<double>(g, kApply, 0, u, nullptr, nullptr, g->q, nb, s, false, g->repl);
        const Level L0 = g->lv[0];
        const double *ff = f, *q = g->q;
        double *r = g->r, *p2 = g->partials2;
        const float* wd = g->wd32[0];
        float *f32v = g->vf32[0], *t32 = sweep ? g->vt32[0] : nullptr;
        emit_launch(g, kStEnd + 330, s, [=](hipStream_t st) {
          launch_replace_r(L0, ff, q, r, p2, wd, f32v, t32, sc, repl, b, st);
        });
      }
    }
    {
      RrCheckTask task{g->partials2, sc, g->active, slot(k)};
      const int b = nb;
      emit_task<RrCheckTask>(
          g, kStEnd + 400, s, batch_sig(kBkRrCheck), task, nb,
          [=](hipStream_t st) { launch_rr_check(task.rr_partials, task.sc, task.active, task.host_slot, b, st); },
          [](const Batch<RrCheckTask>& bt, hipStream_t st) { launch_rr_check_batch(bt, st); });
    }
    issued = k;
    return post(k, false, kStEnd + 500);
  }
  // r -= alpha q (TQ: q's type) fused with the first sweep, as a batchable task
  template <typename TW, typename TQ>
  void emit_update_r(int npq, int parity, const TQ* q, const TW* wd, float* f32, TW* t, const int* repl) {
    UpdateRTask<TW, TQ> task{N(), g->partials, npq, parity, g->scalars, g->active, q, g->r, g->partials2, wd, f32, t,
                             repl};
    const int b = nb;
    emit_task<UpdateRTask<TW, TQ>>(
        g, kStEnd + 300, s, batch_sig(kBkUpdateR, sizeof(TW), sizeof(TQ)), task, kReduceBlocks * nb,
        [=](hipStream_t st) {
          launch_update_r_first<TW, TQ>(task.n, task.pq_partials, task.npq, task.sc, task.active, task.q, task.r,
                                        task.rr_partials, task.parity, task.wdinv, task.f32, task.t, b, st,
                                        task.repl);
        },
        [](const Batch<UpdateRTask<TW, TQ>>& bt, hipStream_t st) { launch_update_r_first_batch<TW, TQ>(bt, st); });
  }
  template <typename TZ>
  void emit_update_px(int nrz, int parity, const TZ* z, float* p32) {
    UpdatePxTask<TZ> task{N(), g->partials, nrz, parity, g->scalars, g->active, z, g->p, u, p32, g->p32b};
    const int b = nb;
    emit_task<UpdatePxTask<TZ>>(
        g, kStEnd + 100, s, batch_sig(kBkUpdatePx, sizeof(TZ)), task, kReduceBlocks * nb,
        [=](hipStream_t st) {
          launch_update_px<TZ>(task.n, task.rz_partials, task.nrz, task.sc, task.active, task.z, task.p, task.x,
                               task.parity, b, st, task.p32, task.p32b);
        },
        [](const Batch<UpdatePxTask<TZ>>& bt, hipStream_t st) { launch_update_px_batch<TZ>(bt, st); });
  }
  // z = M^{-1} r (its first sweep already formed), beta, x += alpha p (iteration k)
  // and p = z + beta p, then iteration k+1
  int issue_next() {
    const int k = issued;
    g->prof_tag = k + 1 - tag_off;
    if (g->desc.precision == HEXMG_FP64) {
      const int nrz = precondition(g, g->r, g->z, g->partials, nb, g->active, s, true, true, true);
      emit_update_px<double>(nrz, (k - 1) & 1, g->z, nullptr);
    } else {
      const int nrz = precondition(g, g->r, g->z, g->partials, nb, g->active, s, false, true, true);
      emit_update_px<float>(nrz, (k - 1) & 1, g->vu32[0], g->p32);  // mixed: the direction itself
    }
    return issue_iteration(k + 1);
  }
  int begin() {
    const Level& L0 = g->lv[0];
    double* sc = g->scalars;
    prev_rr.assign(nb, 0.0);
    its_off.assign(nb, 0);
    limit = maxit;
    {
      hipEvent_t e0 = t0;
      HIP_TRY(emit_api(g, kStStart, s, [=](hipStream_t st) { return hipEventRecord(e0, st); }));
    }
    const int b = nb;
    const long long n = N();
    double *r = g->r, *x = u, *parts = g->partials, *p = g->p;
    float* p32 = g->p32;
    int* act = g->active;
    const double* ff = f;
    const double rt2 = rtol > 0.0 ? rtol * rtol : -1.0;
    emit_launch(g, kStStart + 1, s, [=](hipStream_t st) {
      launch_pcg_start(L0, ff, r, x, parts, b, st);  // r0 = M f, x0 = 0, ||r0||^2 partials
    });
    emit_launch(g, kStInit, s, [=](hipStream_t st) { launch_pcg_init(rt2, parts, sc, act, b, st); });
    if (maxit == 0) return enqueue_finish(0);
    g->prof_tag = 1;
    if (p) {
      precondition(g, g->r, p, g->partials, nb, g->active, s);  // p0 = z0 = M^{-1} r0
    } else {  // mixed form: z0 stays in the binary32 V-cycle output, which p0 copies
      precondition(g, g->r, nullptr, g->partials, nb, g->active, s, false);
      const float* z32 = g->vu32[0];
      const size_t bytes = (size_t)n * b * sizeof(float);
      HIP_TRY(emit_api(g, kStEnd + 20, s,
                       [=](hipStream_t st) { return hipMemcpyAsync(p32, z32, bytes, hipMemcpyDeviceToDevice, st); }));
    }
    emit_launch(g, kStEnd + 10, s, [=](hipStream_t st) { launch_reduce_final(parts, sc + kRz0, kScalars, b, st); });
    if (m32()) emit_launch(g, kStEnd + 20, s, [=](hipStream_t st) { launch_f64_to_f32(n, p, p32, b, act, st); });
    if (int e = issue_iteration(1)) return e;
    if (maxit >= 2)
      if (int e = issue_next()) return e;
    target = 1;
    phase = kIterate;
    return 0;
  }
  // HEXMG_MIXED32: CG restarted from the current iterate for the right-hand
  // sides whose binary64 residual (just computed by the finish, A x in q)
  // misses the test although the recursive one met it: r = M f - A x,
  // z = M^{-1} r, p = z, then iterations continue.  h: the finish's scalars.
  int restart(const double* h) {
    double* sc = g->scalars;
    int its_min = maxit;
    const int k1 = issued + 1;
    for (int k = 0; k < nb; ++k) {
      const double* q = h + k * kScalars;
      if (q[kStatus] == 0.0 && q[kTmp] > q[kStop] && q[kIts] < maxit) {
        its_min = std::min(its_min, (int)q[kIts]);
        its_off[k] = k1 - 1 - (int)q[kIts];
      }
    }
    int last_its = 0;
    for (int k = 0; k < nb; ++k) last_its = std::max(last_its, (int)h[k * kScalars + kIts]);
    ++restarts;
    tag_off = issued - last_its;
    limit = issued + (maxit - its_min);
    const int b = nb, mx = maxit;
    const long long n = N();
    int* act = g->active;
    emit_launch(g, kStRestart, s, [=](hipStream_t st) { launch_pcg_restart(sc, act, b, mx, st); });
    const bool sweep = g->L > 1;
    {
      const Level L0 = g->lv[0];
      const double *ff = f, *q = g->q;
      double *r = g->r, *p2 = g->partials2;
      const float* wd = g->wd32[0];
      float *f32v = g->vf32[0], *t32 = sweep ? g->vt32[0] : nullptr;
      emit_launch(g, kStReplace, s,
                  [=](hipStream_t st) { launch_replace_r(L0, ff, q, r, p2, wd, f32v, t32, sc, act, b, st); });
    }
    g->prof_tag = k1 - tag_off;
    precondition(g, g->r, g->p, g->partials, nb, g->active, s, true, true);  // p = z = M^{-1} r
    double *parts = g->partials, *p = g->p;
    float* p32 = g->p32;
    const int par = (k1 - 1) & 1;
    emit_launch(g, kStEnd + 10, s,
                [=](hipStream_t st) { launch_reduce_final(parts, sc + kRz0 + par, kScalars, b, st); });
    emit_launch(g, kStEnd + 20, s, [=](hipStream_t st) { launch_f64_to_f32(n, p, p32, b, act, st); });
    if (int e = issue_iteration(k1)) return e;
    if (k1 + 1 <= limit)
      if (int e = issue_next()) return e;
    target = k1;
    phase = kIterate;
    for (int k = 0; k < nb; ++k) prev_rr[k] = 0.0;
    return 0;
  }
  int enqueue_finish(int read) {
    const Level L0 = g->lv[0];
    double* sc = g->scalars;
    const int b = nb;
    const long long n = N();
    double *p = g->p, *x = u, *q = g->q, *pa = g->partials, *pb = g->partials2;
    const float *p32 = g->p32, *p32b = g->p32b;
    const double* ff = f;
    emit_launch(g, kStEnd + 600, s, [=](hipStream_t st) {
      launch_flush_x(n, sc, p, x, b, st, nullptr, p32, p32b);  // the x updates still pending
    });
    {
      hipEvent_t e1 = t1;
      HIP_TRY(emit_api(g, kStEnd + 610, s, [=](hipStream_t st) { return hipEventRecord(e1, st); }));
    }
    g->prof_tag = 0;
    g->stage = kStEnd + 620;
    gather<double>(g, kApply, 0, u, nullptr, nullptr, g->q, nb, s);  // true residual in binary64
    emit_launch(g, kStEnd + 630, s, [=](hipStream_t st) {
      launch_pcg_final(L0, ff, q, x, pa, pb, sc, b, st);  // ||M f - A x||^2, f . x
    });
    final_slot = read + 2;  // a slot no result in flight is written to
    phase = kFinish;
    return post(final_slot, true, kStEnd + 640);
  }
  // Whether the iteration after `target` (already in flight) is expected to
  // meet the stop test for every active right-hand side: ||r||^2 shrinking by
  // the last observed factor would reach the threshold.  Speculating one more
  // iteration beyond it would then only queue launches that exit at once.
  bool predict_last(const double* h) {
    bool all = true;
    for (int k = 0; k < nb; ++k) {
      const double* q = h + k * kScalars;
      const double rr = q[kRr], prev = prev_rr[k] > 0.0 ? prev_rr[k] : q[kFf];
      if (q[kActive] != 0.0 && !(prev > 0.0 && rr * (rr / prev) <= q[kStop])) all = false;
    }
    return all;
  }
  int advance() {
    if (phase == kIterate) {
      const double* h = slot(target);
      int nact = 0;
      for (int k = 0; k < nb; ++k) nact += h[k * kScalars + kActive] != 0.0;
      if (nact == 0 || target >= limit) return enqueue_finish(target);
      // keep one iteration in flight beyond the one waited for, unless that
      // one is expected to be the last
      const bool last = predict_last(h);
      while (issued < limit && issued < target + 2 && !(issued == target + 1 && last))
        if (int e = issue_next()) return e;
      for (int k = 0; k < nb; ++k) prev_rr[k] = h[k * kScalars + kRr];
      ++target;
      return 0;
    }
    // kFinish
    const double* h = slot(final_slot);
    HIP_TRY(hipGetLastError());
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    status = 0;
    int last_its = 0;
    for (int k = 0; k < nb; ++k) last_its = std::max(last_its, (int)h[k * kScalars + kIts]);
    prune_profile(g, last_its);
    if (m32() && restarts < 8) {  // binary64 residual short of the test: continue from x
      bool any = false;
      for (int k = 0; k < nb; ++k) {
        const double* q = h + k * kScalars;
        any = any || (q[kStatus] == 0.0 && q[kTmp] > q[kStop] && q[kIts] < maxit);
      }
      if (any) return restart(h);
    }
    for (int k = 0; k < nb; ++k) {
      const double* q = h + k * kScalars;
      const int st = (int)q[kStatus];
      const double ff = q[kFf];
      if (info) {
        hexmg_solve_info& in = info[k];
        in.iterations = (int)q[kIts];
        in.status = st;
        in.rel_res_recursive = ff > 0 ? std::sqrt(q[kRr] / ff) : 0.0;
        in.rel_res_true = ff > 0 ? std::sqrt(q[kTmp] / ff) : 0.0;
        in.compliance = q[kTmp2];
        in.ms_solve = ms;
      }
      if (st == -4) return fail(HEXMG_ERR_NONFINITE, "load vector is not finite");
      if (st < 0)
        status = st;
      else if (status >= 0 && st > status)
        status = st;
    }
    phase = kDone;
    return 0;
  }
};

// Drives a set of runs (distinct grids) to completion: each round waits for
// every pending run's scalars, then lets each run enqueue its next phase.
int drive(std::vector<PcgRun>& runs) {
  for (auto& r : runs)
    if (int e = r.begin()) return e;
  for (;;) {
    bool pending = false;
    for (auto& r : runs) {
      if (r.phase == PcgRun::kDone) continue;
      pending = true;
      HIP_TRY(hipEventSynchronize(r.wait_event()));
      if (int e = r.advance()) return e;
    }
    if (!pending) return 0;
  }
}

// Drives runs of distinct grids on one stream with their launches batched:
// every round records the next launches of every pending run (each run still
// decides on its own, from its own scalars) and then launches them together,
// one launch per place in the iteration and kernel signature for all grids.
int drive_batched(std::vector<PcgRun>& runs, BatchRecorder& rec, hipStream_t s) {
  for (size_t i = 0; i < runs.size(); ++i) {
    runs[i].g->rec = &rec;
    runs[i].g->rec_grid = (int)i;
  }
  int e = 0;
  for (auto& r : runs)
    if (!e) e = r.begin();
  bool pending = true;
  while (!e) {
    const hipError_t he = rec.flush(s);
    if (he != hipSuccess) {
      e = fail(HEXMG_ERR_DEVICE, std::string("batched launch: ") + hipGetErrorString(he));
      break;
    }
    if (!pending) break;
    pending = false;
    for (auto& r : runs) {
      if (r.phase == PcgRun::kDone) continue;
      pending = true;
      if (hipEventSynchronize(r.wait_event()) != hipSuccess) {
        e = fail(HEXMG_ERR_DEVICE, "event wait failed");
        break;
      }
      if ((e = r.advance())) break;
    }
  }
  if (e) rec.recs.clear();
  for (auto& r : runs) r.g->rec = nullptr;
  return e;
}

int combine_status(int worst, int st) {
  if (st < 0) return st;
  if (worst >= 0 && st > worst) return st;
  return worst;
}

}  // namespace

extern "C" {

int hexmg_solve(hexmg_grid_t g, const double* f, double* u, int nrhs, double rtol, int maxit,
                hexmg_solve_info* info, void* stream) {
  if (!g || !f || !u) return fail(HEXMG_ERR_INVALID, "null argument");
  if (nrhs < 1 || maxit < 0) return fail(HEXMG_ERR_INVALID, "bad nrhs or maxit");
  if (!g->density_set) return fail(HEXMG_ERR_INVALID, "hexmg_set_density has not succeeded");
  hipStream_t s = (hipStream_t)stream;
  g->last_stream = s;
  const long long N = 3ll * g->lv[0].nn;
  int worst = 0;
  for (int k = 0; k < nrhs; k += g->desc.max_nrhs) {
    std::vector<PcgRun> runs(1);
    PcgRun& r = runs[0];
    r.g = g;
    r.f = f + k * N;
    r.u = u + k * N;
    r.nb = (nrhs - k) < g->desc.max_nrhs ? (nrhs - k) : g->desc.max_nrhs;
    r.rtol = rtol;
    r.maxit = maxit;
    r.s = s;
    r.info = info ? info + k : nullptr;
    int e = r.init();
    if (!e) e = drive(runs);
    r.release();
    if (e) return e;
    worst = combine_status(worst, r.status);
  }
  if (worst == HEXMG_ERR_BREAKDOWN) return fail(worst, "PCG breakdown (p^T A p <= 0 or non-finite residual)");
  if (worst == HEXMG_NOT_CONVERGED) g_err = "not converged within maxit";
  return worst;
}

int hexmg_batch_solve(hexmg_grid_t* grids, int ngrids, const double* const* f, double* const* u, const int* nrhs,
                      double rtol, int maxit, hexmg_solve_info* infos, void* stream) {
  if (!grids || !f || !u || !nrhs || ngrids < 1) return fail(HEXMG_ERR_INVALID, "null argument");
  if (maxit < 0) return fail(HEXMG_ERR_INVALID, "bad maxit");
  for (int i = 0; i < ngrids; ++i) {
    if (!grids[i] || !f[i] || !u[i]) return fail(HEXMG_ERR_INVALID, "null grid or vector");
    if (nrhs[i] < 1 || nrhs[i] > grids[i]->desc.max_nrhs)
      return fail(HEXMG_ERR_INVALID, "nrhs[i] must be in [1, max_nrhs of grid i]");
    if (!grids[i]->density_set) return fail(HEXMG_ERR_INVALID, "hexmg_set_density has not succeeded on every grid");
    for (int j = 0; j < i; ++j)
      if (grids[j] == grids[i]) return fail(HEXMG_ERR_INVALID, "a grid appears twice in the batch");
  }
  hipStream_t s = (hipStream_t)stream;
  // All grids run on the caller's stream; their launches are batched (see
  // drive_batched).  Batched launches of the streaming kernel share the block
  // coefficients of K0, so grids whose Poisson ratios differ go in separate
  // launches (a class per distinct ratio).  The cooperative coarse-cycle launch
  // is not batched: the coarse part of the cycle is launched step by step.
  struct Saved { int t64, t32; };
  std::vector<Saved> saved(ngrids);
  std::vector<double> nus;
  for (int i = 0; i < ngrids; ++i) {
    hexmg_grid* g = grids[i];
    saved[i] = {g->tail64, g->tail32};
    g->tail64 = g->tail32 = 0;
    g->last_stream = s;
    size_t k = 0;
    while (k < nus.size() && nus[k] != g->desc.nu) ++k;
    if (k == nus.size()) nus.push_back(g->desc.nu);
    g->rec_class = (int)k;
  }
  int worst = 0, e = 0;
  // right-hand sides beyond max_nrhs are not batched: nrhs[i] <= max_nrhs (checked above)
  std::vector<PcgRun> runs(ngrids);
  int off = 0;
  for (int i = 0; i < ngrids && !e; ++i) {
    PcgRun& r = runs[i];
    r.g = grids[i];
    r.f = f[i];
    r.u = u[i];
    r.nb = nrhs[i];
    r.rtol = rtol;
    r.maxit = maxit;
    r.s = s;
    r.info = infos ? infos + off : nullptr;
    off += nrhs[i];
    e = r.init();
  }
  BatchRecorder rec(ngrids);
  if (!e) e = drive_batched(runs, rec, s);
  for (auto& r : runs) worst = combine_status(worst, r.status);
  if (!e) (void)hipStreamSynchronize(s);
  for (auto& r : runs) r.release();
  for (int i = 0; i < ngrids; ++i) {
    grids[i]->tail64 = saved[i].t64;
    grids[i]->tail32 = saved[i].t32;
    grids[i]->batch_launches = rec.launches;
    grids[i]->batch_records = rec.records;
  }
  if (e) return e;
  if (worst == HEXMG_ERR_BREAKDOWN) return fail(worst, "PCG breakdown in the batch");
  if (worst == HEXMG_NOT_CONVERGED) g_err = "not converged within maxit";
  return worst;
}

int hexmg_batch_stats(hexmg_grid_t g, size_t* launches, size_t* recorded) {
  if (!g) return fail(HEXMG_ERR_INVALID, "null grid");
  if (launches) *launches = g->batch_launches;
  if (recorded) *recorded = g->batch_records;
  return 0;
}

int hexmg_compliance_sensitivity(hexmg_grid_t g, const double* f, const double* u, int nrhs,
                                 const double* weights, double* c_host, double* dc, void* stream) {
  if (!g || !f || !u) return fail(HEXMG_ERR_INVALID, "null argument");
  if (nrhs < 1) return fail(HEXMG_ERR_INVALID, "nrhs must be >= 1");
  if (!g->density_set) return fail(HEXMG_ERR_INVALID, "hexmg_set_density has not succeeded");
  hipStream_t s = (hipStream_t)stream;
  g->last_stream = s;
  const Level& L0 = g->lv[0];
  const long long N = 3ll * L0.nn;
  const hexmg_grid_desc& d = g->desc;
  for (int k = 0; k < nrhs; ++k) {
    if (dc) {
      const double w = weights ? weights[k] : 1.0;
      launch_sensitivity_haar(L0, g->hq64, g->rho[0], u + k * N, -d.penal * (d.E0 - d.Emin) * w, d.penal - 1.0,
                              k > 0, dc, s);
    }
    if (c_host) {
      dot(g, N, f + k * N, u + k * N, g->scalars + kTmp, 1, s);
      if (int e = read_scalars(g, 1, s)) return e;
      c_host[k] = g->host_scalars[kTmp];
    }
  }
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_filter(int nx, int ny, int nz, double rmin, int adjoint, const double* in, double* out, double* tmp,
                 void* stream) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(HEXMG_ERR_INVALID, "grid dimensions must be >= 1");
  if (!(rmin > 1.0 && rmin <= 8.0)) return fail(HEXMG_ERR_INVALID, "need 1 < rmin <= 8");
  if (!in || !out || in == out) return fail(HEXMG_ERR_INVALID, "need distinct in and out");
  if (adjoint && (!tmp || tmp == in || tmp == out)) return fail(HEXMG_ERR_INVALID, "the adjoint needs a separate tmp");
  if ((long long)nx * ny * nz >= (1ll << 31)) return fail(HEXMG_ERR_INVALID, "grid too large");
  launch_filter(nx, ny, nz, rmin, adjoint, in, out, tmp, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_filter_noalloc(int nx, int ny, int nz, double rmin, int adjoint, const double* in, double* out,
                         void* stream) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(HEXMG_ERR_INVALID, "grid dimensions must be >= 1");
  if (!(rmin > 1.0 && rmin <= 8.0)) return fail(HEXMG_ERR_INVALID, "need 1 < rmin <= 8");
  if (!in || !out || in == out) return fail(HEXMG_ERR_INVALID, "need distinct in and out");
  const long long n = (long long)nx * ny * nz;
  double* tmp = nullptr;
  if (adjoint) {
    if (n > kFilterScratchElems)
      return fail(HEXMG_ERR_INVALID, "hexmg_filter_noalloc: the adjoint takes at most " +
                                         std::to_string(kFilterScratchElems) + " elements, got " + std::to_string(n));
    const int e = filter_scratch_ptr(&tmp);
    if (e != 0)
      return fail(HEXMG_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(static_cast<hipError_t>(e)));
  } else if (n >= (1ll << 31)) {
    return fail(HEXMG_ERR_INVALID, "grid too large");
  }
  launch_filter(nx, ny, nz, rmin, adjoint, in, out, tmp, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_sensitivity_filter(int nx, int ny, int nz, double rmin, double gamma, const double* x, const double* dc,
                             double* out, void* stream) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(HEXMG_ERR_INVALID, "grid dimensions must be >= 1");
  if (!(rmin > 0.0 && rmin <= 8.0)) return fail(HEXMG_ERR_INVALID, "need 0 < rmin <= 8");
  if (!(gamma > 0.0)) return fail(HEXMG_ERR_INVALID, "need gamma > 0");
  if (!x || !dc || !out || out == x || out == dc) return fail(HEXMG_ERR_INVALID, "out must not overlap x or dc");
  if ((long long)nx * ny * nz >= (1ll << 31)) return fail(HEXMG_ERR_INVALID, "grid too large");
  launch_sens_filter(nx, ny, nz, rmin, gamma, x, dc, out, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_gravity_load(hexmg_grid_t g, double gz, const double* f_ext, double* f, void* stream) {
  if (!g || !f) return fail(HEXMG_ERR_INVALID, "null argument");
  if (f == f_ext) return fail(HEXMG_ERR_INVALID, "f must not overlap f_ext");
  if (!std::isfinite(gz)) return fail(HEXMG_ERR_INVALID, "g must be finite");
  if (!g->density_set) return fail(HEXMG_ERR_INVALID, "hexmg_set_density has not succeeded");
  launch_gravity_load(g->lv[0], g->rho[0], gz, f_ext, f, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_gravity_sensitivity(hexmg_grid_t g, const double* u, double gz, double weight, double* dc, void* stream) {
  if (!g || !u || !dc) return fail(HEXMG_ERR_INVALID, "null argument");
  if (!std::isfinite(gz) || !std::isfinite(weight)) return fail(HEXMG_ERR_INVALID, "g and weight must be finite");
  launch_gravity_sensitivity(g->lv[0], u, 2.0 * weight * (-gz / 8.0), dc, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_apply_passive(long long n, const uint8_t* passive, double* x, void* stream) {
  if (n < 0 || (n > 0 && (!passive || !x))) return fail(HEXMG_ERR_INVALID, "null argument or negative size");
  if (n == 0) return 0;
  launch_apply_passive(n, passive, x, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_volume_weights(hexmg_grid_t g, const uint8_t* passive, double* dv, void* stream) {
  if (!g || !passive || !dv) return fail(HEXMG_ERR_INVALID, "null argument");
  launch_volume_weights(g->lv[0].ne, passive, g->flags, dv, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return 0;
}

int hexmg_oc_update(hexmg_grid_t g, const double* x, const double* dc, const double* dv, double volfrac,
                    double move, double eta, double* x_new, double* lambda_host, double* change_host,
                    double* volume_host, void* stream) {
  if (!g || !x || !dc || !dv || !x_new) return fail(HEXMG_ERR_INVALID, "null argument");
  if (x_new == x || x_new == dc || x_new == dv) return fail(HEXMG_ERR_INVALID, "x_new must not overlap the inputs");
  if (!(volfrac > 0.0 && volfrac < 1.0) || !(move > 0.0 && move <= 1.0) || !(eta > 0.0 && eta <= 1.0))
    return fail(HEXMG_ERR_INVALID, "need 0 < volfrac < 1, 0 < move <= 1, 0 < eta <= 1");
  hipStream_t s = (hipStream_t)stream;
  const long long n = g->lv[0].ne;
  // bisection on log lambda, kOcProbes interior probes per pass
  double lo = std::log(1e-12), hi = std::log(1e12);
  const double rel_tol = 1e-12;
  int passes = 0;
  while (std::exp(hi - lo) - 1.0 > rel_tol && passes < 64) {
    OcProbes pw;
    double lp[kOcProbes];
    for (int p = 0; p < kOcProbes; ++p) {
      lp[p] = lo + (hi - lo) * (p + 1) / (kOcProbes + 1);
      pw.v[p] = std::exp(-eta * lp[p]);
    }
    launch_oc_probe(n, x, dc, dv, eta, move, pw, g->oc_partials, g->oc_vol, s);
    HIP_TRY(hipMemcpyAsync(g->host_scalars, g->oc_vol, kOcProbes * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // the pinned mirror holds 8*kScalars doubles
    static_assert(kOcProbes <= 8 * kScalars, "pinned buffer too small");
    double nlo = lo, nhi = hi;
    for (int p = 0; p < kOcProbes; ++p) {
      if (g->host_scalars[p] > volfrac) {
        nlo = lp[p];
      } else {
        nhi = lp[p];
        break;
      }
    }
    if (!std::isfinite(g->host_scalars[0])) return fail(HEXMG_ERR_NONFINITE, "non-finite OC volume");
    lo = nlo;
    hi = nhi;
    ++passes;
  }
  const double lam = std::exp(0.5 * (lo + hi));
  launch_oc_apply(n, x, dc, dv, eta, move, std::exp(-eta * 0.5 * (lo + hi)), x_new, g->oc_partials, g->oc_vol, s);
  HIP_TRY(hipGetLastError());
  if (change_host || volume_host) {
    HIP_TRY(hipMemcpyAsync(g->host_scalars, g->oc_vol, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (change_host) *change_host = g->host_scalars[0];
    if (volume_host) *volume_host = g->host_scalars[1];
  }
  if (lambda_host) *lambda_host = lam;
  return 0;
}

int hexmg_element_matrix(double nu, double* Ke) {
  if (!Ke) return fail(HEXMG_ERR_INVALID, "null output");
  if (!(nu > -1.0 && nu < 0.5)) return fail(HEXMG_ERR_INVALID, "need -1 < nu < 0.5");
  element_matrix(nu, Ke);
  return 0;
}

int hexmg_kernel_choice(hexmg_grid_t g, int level, int dtype, int mode, int* kernel, int* zchunk, int* shape) {
  if (!g) return fail(HEXMG_ERR_INVALID, "null grid");
  if (level < 0 || level >= g->L) return fail(HEXMG_ERR_INVALID, "bad level");
  if (dtype != HEXMG_F64 && dtype != HEXMG_F32) return fail(HEXMG_ERR_INVALID, "bad dtype");
  if (mode < 0 || mode > 2) return fail(HEXMG_ERR_INVALID, "mode must be 0 (K u), 1 (sweep) or 2 (residual)");
  const hexmg_grid::Choice& c = (dtype == HEXMG_F64 ? g->choice64[level] : g->choice32[level])[mode];
  if (kernel) *kernel = c.kernel;
  if (zchunk) *zchunk = c.zchunk;
  if (shape) *shape = c.shape;
  return 0;
}

int hexmg_set_kernel_choice(hexmg_grid_t g, int level, int dtype, int kernel, int zchunk, int shape) {
  if (!g) return fail(HEXMG_ERR_INVALID, "null grid");
  if (level < 0 || level >= g->L) return fail(HEXMG_ERR_INVALID, "bad level");
  if (dtype != HEXMG_F64 && dtype != HEXMG_F32) return fail(HEXMG_ERR_INVALID, "bad dtype");
  hexmg_grid::Choice c{kernel, zchunk, shape};
  if (kernel == HEXMG_KERNEL_GATHER) {
    c = {HEXMG_KERNEL_GATHER, 0, 0};
  } else if (kernel == HEXMG_KERNEL_STREAM) {
    if (zchunk < 1 || shape < 0 || shape >= stream_shapes(dtype == HEXMG_F32))
      return fail(HEXMG_ERR_INVALID, "bad z-chunk or shape");
    const int nzn = g->lv[level].nzn;
    if ((long long)((nzn + zchunk - 1) / zchunk) * g->desc.max_nrhs > 65535)
      return fail(HEXMG_ERR_INVALID, "z-chunk too small: z-chunks times max_nrhs must be <= 65535");
  } else {
    return fail(HEXMG_ERR_INVALID, "bad kernel");
  }
  (dtype == HEXMG_F64 ? g->choice64 : g->choice32)[level].fill(c);
  g->tuned = true;
  return 0;
}

int hexmg_coarse_cycle_choice(hexmg_grid_t g, int dtype, int* level, int* blocks) {
  if (!g) return fail(HEXMG_ERR_INVALID, "null grid");
  if (dtype != HEXMG_F64 && dtype != HEXMG_F32) return fail(HEXMG_ERR_INVALID, "bad dtype");
  if (level) *level = dtype == HEXMG_F32 ? g->tail32 : g->tail64;
  if (blocks) *blocks = dtype == HEXMG_F32 ? g->tail_blocks32 : g->tail_blocks64;
  return 0;
}

int hexmg_set_coarse_cycle(hexmg_grid_t g, int dtype, int level, int blocks) {
  if (!g) return fail(HEXMG_ERR_INVALID, "null grid");
  if (dtype != HEXMG_F64 && dtype != HEXMG_F32) return fail(HEXMG_ERR_INVALID, "bad dtype");
  if (level != 0 && (level < 1 || level > g->L - 2))
    return fail(HEXMG_ERR_INVALID, "level must be 0 (off) or in [1, levels - 2]");
  if (level != 0 && g->galerkin)
    return fail(HEXMG_ERR_INVALID, "the cooperative coarse cycle is not available with Galerkin coarse operators");
  if (blocks < 0) return fail(HEXMG_ERR_INVALID, "blocks must be >= 0");
  int b = 0;
  if (level) {
    const int maxb = dtype == HEXMG_F32 ? coarse_cycle_max_blocks<float>() : coarse_cycle_max_blocks<double>();
    if (maxb <= 0) return fail(HEXMG_ERR_DEVICE, "cooperative launch not available");
    b = (blocks == 0 || blocks > maxb) ? maxb : blocks;
  }
  (dtype == HEXMG_F32 ? g->tail32 : g->tail64) = level;
  (dtype == HEXMG_F32 ? g->tail_blocks32 : g->tail_blocks64) = b;
  g->tail_tuned = true;
  return 0;
}

int hexmg_profile_enable(hexmg_grid_t g, int enable) {
  if (!g) return fail(HEXMG_ERR_INVALID, "null grid");
  if (!enable) drain_profile(g);
  g->profile = enable != 0;
  if (enable) {
    drain_profile(g);
    for (int i = 0; i < 8; ++i) {
      g->prof_ms[i] = 0.0;
      g->prof_count[i] = 0;
    }
  }
  return 0;
}

int hexmg_profile_query(hexmg_grid_t g, const char* family, int* launches, double* ms) {
  if (!g || !family) return fail(HEXMG_ERR_INVALID, "null argument");
  drain_profile(g);
  for (int i = 0; i < kNumFamilies; ++i)
    if (std::strcmp(family, kFamilies[i]) == 0) {
      if (launches) *launches = g->prof_count[i];
      if (ms) *ms = g->prof_ms[i];
      return 0;
    }
  return fail(HEXMG_ERR_INVALID, std::string("unknown kernel family ") + family);
}

const char* hexmg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
