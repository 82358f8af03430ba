// C ABI and cycle driver of libmgwr (Algorithm 2 of arXiv 1706.07632 on top
// of the gfx950 kernels).  The library never allocates device memory: the
// caller's workspace holds the packed H-matrix and every level's arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "hplan.h"
#include "kernels.h"
#include "mgwr.h"
#include "net.h"
#include "plan_internal.h"

using namespace mgwr;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

namespace mgwr {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace mgwr

namespace {

#define HIP_TRY(...)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (__VA_ARGS__);                                                            \
    if (e_ != hipSuccess) return fail(MGWR_ERR_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kNormParts = 1024;
// Smallest relative tolerance for which solves use zebra defects.
constexpr double kZebraMinTol = 1e-10;

// Carves the workspace: every array starts on a 256-byte boundary.
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

template <typename T>
struct DevOps {  // precision-specific device arrays
  T* dense = nullptr;
  T* dinv = nullptr;
  T* ffA = nullptr;
  T* zuB = nullptr;
  // float32 operations of a MGWR_MIXED_BF16 plan: ffA and zuB hold bfloat16
  // entries (2 bytes each)
  int lr_bf16 = 0;
  std::vector<T*> U, F, R;  // per level
};

}  // namespace

struct mgwr_plan {
  HostPlan hp;
  bool bound = false;
  int device = -1;
  hipStream_t stream = nullptr;
  size_t ws_bytes = 0;
  unsigned char* ws = nullptr;
  // shared index arrays
  LeafDesc* leaves = nullptr;
  int* dn_list = nullptr;
  int* ff_row = nullptr;
  int* zu_row = nullptr;
  double* a1 = nullptr;
  double* tpow = nullptr;             // t_m^alpha, m = 0..M (time variable of the warm-start interpolation)
  double* B0 = nullptr;      // f + a_{.,1} g
  double* part = nullptr;    // norm partials
  double* scal = nullptr;    // device scalar(s)
  DevOps<double> d64;
  DevOps<float> d32;
  bool mixed = false;   // float32 inner cycles (MGWR_MIXED_FP32 or MGWR_MIXED_BF16)
  // 2D grids in colour-split storage inside a solve (MarchArgs::split): the
  // caller's arrays are natural; b is formed split, a given iterate is moved
  // in and the result moved back out (mgwr_plan_set_layout)
  bool split = false;
  int set_layout = MGWR_LAYOUT_AUTO;   // mgwr_plan_set_layout (AUTO: tuned for the shape, else split)
  bool bf16 = false;    // their low-rank factors in bfloat16
  // live timing (mgwr_timing_enable)
  struct Pending { hipEvent_t b, e; int cls; double flops, bytes; };
  bool timing = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  mgwr_timing tacc{};
  // time-pipelined cycles (float64)
  static constexpr int kMaxPipeCycles = 16;
  static_assert(kMaxPipeCycles >= kMaxInnerCycles, "a launch holds one refinement step");
  std::vector<Stage> stages;   // host image for kMaxPipeCycles cycles
  int stages_per_cycle = 0, tasks_per_cycle = 0, norm_chunks = 0;
  const double* stages_f = nullptr;    // level-0 arrays the uploaded image refers to
  const double* stages_u = nullptr;
  Stage* stages_dev = nullptr;
  int* counters = nullptr;
  int* flags_dev = nullptr;            // [0] ticket, [1] abort, [2 .. 2 + kXcdQueues) per-XCD tickets
  int* xq = nullptr;                   // per-XCD task queues of its pipelined launches
  long long xq_cap = 0;                // their capacity (tasks)
  int* xprobe = nullptr;               // 64 ints: the XCD check at binding
  double* norms = nullptr;             // [kMaxPipeCycles][norm_chunks]
  int khint = 0;                       // cycles the last pipelined solve from a zero or given iterate needed
  int khint_warm = 0;                  // the same from a predicted iterate
  int tuned = 0;                       // schedule measured best by mgwr_plan_autotune (0: none)
  // staged schedule knobs: operand prefetch of the marches (0 by mesh length,
  // 1 shallow, 2 deep) and the level the coarse pipelined launch starts at
  // (-1 by rule); set by mgwr_plan_set_staging or mgwr_plan_autotune (else
  // the autotuner's choice for the shape, if any)
  int set_prefetch = 0;
  int set_coarse = -1;
  bool staging_set = false;
  bool side_by_side = false;           // solved beside enough staged instances to busy every batch worker
  int prefetch = 0;                    // in use
  int khint_staged = 0;                // cycles the last staged float64 solve from zero needed
  int khint_staged_warm = 0;           // the same from a predicted iterate
  // average residual factor per cycle of the last converged solve from the
  // zero iterate (0: none yet); the warm-start judge compares a prediction
  // with what the zero iterate reaches in as many cycles
  double rate_zero = 0.0;
  double create_ms = 0.0, bind_ms = 0.0;   // host set-up times (mgwr_stats.setup_ms)
  double cycle_flops = 0.0, cycle_bytes = 0.0;  // algorithmic work of one pipelined cycle
  // staged schedule: from level coarse_l on (0: never) a cycle's levels run as
  // one pipelined launch ([0] float64, [1] float32 stage images)
  int coarse_l = 0;
  unsigned spin_limit = kDefaultSpinLimit;   // polls of a progress wait (mgwr_plan_set_progress_limit)
  std::vector<Stage> coarse_stages[2];
  // Zebra defects (see zebra_defects) in the current solve: only for
  // tolerances of at least kZebraMinTol, since they carry the rounding of
  // the line solves (measured floor about 1e-12 ||b||; 1D n = 127, alpha = 0.7)
  bool zebra = true;
  int coarse_tasks[2] = {0, 0};
  long long coarse_cnt[2] = {0, 0};
  double coarse_flops[2] = {0.0, 0.0}, coarse_bytes[2] = {0.0, 0.0};
  bool coarse_up[2] = {false, false};
  Stage* cstages_dev[2] = {nullptr, nullptr};
  int* ccounters = nullptr;
  int* cflags = nullptr;   // [0] ticket, [1] abort
  // learned initial guess
  static constexpr int kMaxSlices = 64;
  mgwr_net* net = nullptr;
  int nslices = 0;
  int* rows_dev = nullptr;
  // offsets computed by layout()
  struct Off {
    size_t stages, counters, flags, norms, wrows, cstages, ccounters, cflags, xq, xprobe;
    size_t leaves, dn_list, ff_row, zu_row, a1, tm, B0, part, scal;
    size_t dense64, dinv64, ffA64, zuB64, dense32, dinv32, ffA32, zuB32;
    std::vector<size_t> U64, F64, R64, U32, F32, R32;
    size_t total;
  } off;
};

namespace {

// Upper bound of the stages of one pipelined cycle plus what one outer step
// adds to it (its norm defect; in mixed precision also the cast and the
// correction).  A launch holds at most kMaxPipeCycles cycles in all.
long long stages_per_cycle_bound(const HostPlan& hp) {
  const int L = (int)hp.levels.size();
  long long spc = 3, visits = 1;
  for (int l = 0; l < L; ++l) {
    if (l == L - 1) spc += 2 * visits;
    else spc += visits * (2LL * (hp.p.nu1 + hp.p.nu2) + 3);
    visits *= hp.p.gamma;
  }
  return spc;
}

// Work items a pipelined launch of one plan can hold: the stages counted as
// in stages_per_cycle_bound, each with at most one item per 16 points of its
// level, over kMaxPipeCycles cycles.
long long xq_capacity(const HostPlan& hp) {
  const int L = (int)hp.levels.size();
  long long per = 3 * ((hp.levels[0].N + 15) / 16), visits = 1;
  for (int l = 0; l < L; ++l) {
    const long long items = (hp.levels[l].N + 15) / 16;
    if (l == L - 1) per += 2 * visits * items;
    else per += visits * (2LL * (hp.p.nu1 + hp.p.nu2) + 3) * items;
    visits *= hp.p.gamma;
  }
  return per * mgwr_plan::kMaxPipeCycles;
}

void layout(mgwr_plan* pl) {
  const HostPlan& hp = pl->hp;
  const PackedPlan& pk = hp.pk;
  const int M = hp.p.M;
  const int L = (int)hp.levels.size();
  Carver cv;
  auto& o = pl->off;
  o.leaves = cv.take(pk.leaves.size() * sizeof(LeafDesc));
  o.dn_list = cv.take(std::max<size_t>(1, pk.dn_list.size()) * sizeof(int));
  o.ff_row = cv.take(std::max<size_t>(1, pk.ff_row.size()) * sizeof(int));
  o.zu_row = cv.take(std::max<size_t>(1, pk.zu_row.size()) * sizeof(int));
  o.a1 = cv.take((size_t)M * sizeof(double));
  o.tm = cv.take((size_t)(M + 1) * sizeof(double));
  o.part = cv.take(kNormParts * sizeof(double));
  o.scal = cv.take(16 * sizeof(double));
  o.dense64 = cv.take(pk.dense.size() * sizeof(double));
  o.dinv64 = cv.take(pk.dinv.size() * sizeof(double));
  o.ffA64 = cv.take(std::max<size_t>(1, pk.ffA.size()) * sizeof(double));
  o.zuB64 = cv.take(std::max<size_t>(1, pk.zuB.size()) * sizeof(double));
  o.B0 = cv.take((size_t)M * hp.levels[0].N * sizeof(double));
  o.U64.assign(L, 0); o.F64.assign(L, 0); o.R64.assign(L, 0);
  for (int l = 0; l < L; ++l) {
    size_t bytes = (size_t)M * hp.levels[l].N * sizeof(double);
    if (l > 0) { o.U64[l] = cv.take(bytes); o.F64[l] = cv.take(bytes); }
    if (l + 1 < L || l == 0) o.R64[l] = cv.take(bytes);
  }
  pl->mixed = hp.p.precision == MGWR_MIXED_FP32 || hp.p.precision == MGWR_MIXED_BF16;
  pl->bf16 = hp.p.precision == MGWR_MIXED_BF16;
  o.U32.assign(L, 0); o.F32.assign(L, 0); o.R32.assign(L, 0);
  if (pl->mixed) {
    o.dense32 = cv.take(pk.dense.size() * sizeof(float));
    o.dinv32 = cv.take(pk.dinv.size() * sizeof(float));
    // the inner cycles' low-rank factors: float32, or bfloat16 (2 bytes)
    const size_t lr_bytes = pl->bf16 ? 2 : sizeof(float);
    o.ffA32 = cv.take(std::max<size_t>(1, pk.ffA.size()) * lr_bytes);
    o.zuB32 = cv.take(std::max<size_t>(1, pk.zuB.size()) * lr_bytes);
    for (int l = 0; l < L; ++l) {
      size_t bytes = (size_t)M * hp.levels[l].N * sizeof(float);
      o.U32[l] = cv.take(bytes);
      o.F32[l] = cv.take(bytes);
      if (l + 1 < L) o.R32[l] = cv.take(bytes);
    }
  }
  // pipelined schedule: stage table, per-(stage, leaf) counters, norms
  {
    const int nleaf = (int)pk.leaves.size();
    // stages per cycle: per non-coarsest level 2(nu1+nu2) half-sweeps + defect +
    // restriction + prolongation, times gamma^depth visits; coarsest 2; plus the norm defect
    const long long S = stages_per_cycle_bound(hp) * mgwr_plan::kMaxPipeCycles;
    o.stages = cv.take((size_t)S * sizeof(Stage));
    o.counters = cv.take((size_t)S * nleaf * sizeof(int));
    o.flags = cv.take((2 + kXcdQueues) * sizeof(int));
    o.norms = cv.take((size_t)mgwr_plan::kMaxPipeCycles * ((hp.levels[0].N + 15) / 16) * sizeof(double));
    // a launch's tasks: at most every stage with the largest work-item count
    o.xq = cv.take((size_t)xq_capacity(hp) * sizeof(int));
    o.xprobe = cv.take(64 * sizeof(int));
    // the coarse part of a staged cycle (one cycle from level >= 1)
    const long long C = stages_per_cycle_bound(hp);
    o.cstages = cv.take((size_t)2 * C * sizeof(Stage));
    o.ccounters = cv.take((size_t)C * nleaf * sizeof(int));
    o.cflags = cv.take(2 * sizeof(int));
  }
  o.wrows = cv.take(mgwr_plan::kMaxSlices * sizeof(int));
  o.total = cv.off;
}

hipEvent_t pool_event(mgwr_plan* pl) {
  if (!pl->event_pool.empty()) {
    hipEvent_t e = pl->event_pool.back();
    pl->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when timing is on.
struct Timed {
  mgwr_plan* pl;
  int cls;
  double flops, bytes;
  hipEvent_t b = nullptr;
  Timed(mgwr_plan* p, int c, double f, double by) : pl(p), cls(c), flops(f), bytes(by) {
    if (pl->timing && (b = pool_event(pl))) (void)hipEventRecord(b, pl->stream);
  }
  ~Timed() {
    if (!b) return;
    hipEvent_t e = pool_event(pl);
    if (!e) { pl->event_pool.push_back(b); return; }
    (void)hipEventRecord(e, pl->stream);
    pl->pending.push_back({b, e, cls, flops, bytes});
  }
};

// Accumulates finished event pairs (the stream has been synchronised).
void drain_timing(mgwr_plan* pl) {
  for (auto& q : pl->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, q.b, q.e) == hipSuccess) {
      pl->tacc.launches[q.cls] += 1;
      pl->tacc.ms[q.cls] += ms;
      pl->tacc.flops[q.cls] += q.flops;
      pl->tacc.bytes[q.cls] += q.bytes;
    }
    pl->event_pool.push_back(q.b);
    pl->event_pool.push_back(q.e);
  }
  pl->pending.clear();
}

template <typename T>
MarchArgs<T> base_args(mgwr_plan* pl, const DevOps<T>& ops, int level) {
  const HostPlan& hp = pl->hp;
  MarchArgs<T> a{};
  a.leaves = pl->leaves;
  a.nleaf = (int)hp.pk.leaves.size();
  a.dn_list = pl->dn_list;
  a.dense = ops.dense;
  a.dinv = ops.dinv + (size_t)level * a.nleaf * 256;
  a.dinv_hi = sizeof(T) == 4 ? pl->d64.dinv + (size_t)level * a.nleaf * 256 : nullptr;
  a.ff_row = pl->ff_row;
  a.ffA = ops.ffA;
  a.zu_row = pl->zu_row;
  a.zuB = ops.zuB;
  a.lr_bf16 = ops.lr_bf16;
  a.prefetch = pl->prefetch;
  a.k = hp.p.k;
  a.nslots = hp.nslots;
  a.split = pl->split && hp.p.dim == 2 ? 1 : 0;
  a.n0 = (hp.levels[level].N + 1) / 2;
  a.ring = std::max(hp.window + 2, 3);  // leaves written while older ones are still read
  return a;
}

// Grid transfers fused into the marches (1D only; the cycle is the same in
// exact arithmetic).  Restriction: after a second-colour half-sweep the
// defect lives on the first colour, the coarse points q = 2p + 1, where full
// weighting reduces to r[q] / 2: the defect march writes it straight into
// the coarse right-hand side.  Prolongation: the first-colour half-sweep that
// follows the coarse-grid correction reads the iterate only at its
// second-colour neighbours (its own lines are solved afresh), and the second-
// colour half-sweep after it reads only first-colour values, so the corrected
// iterate is needed nowhere else; the half-sweep adds the interpolated
// correction to the neighbours it reads.
struct TransferFusion {
  bool restrict_in_defect, prolong_in_smooth;
};
TransferFusion transfer_fusion(const HostPlan& hp) {
  TransferFusion f;
  f.restrict_in_defect = hp.p.dim == 1 && hp.p.nu1 >= 1;
  f.prolong_in_smooth = hp.p.dim == 1 && hp.p.nu2 >= 1;
  return f;
}

// Zebra-in-time line relaxation of one colour on one level: every line of
// the colour is solved with (R~ + c_l I) by the H-forward substitution.
// Colour 0 is updated first: the coarse-grid points (1-based even in 1D,
// i + j even in 2D), which are the flat indices q with q % 2 == par0.
// Ec (1D, colour 0 only): coarse correction whose interpolation the
// half-sweep applies to the neighbours it reads (see MarchArgs).
// Dout: see MarchArgs (the changes of the solved entries).
template <typename T>
int smooth(mgwr_plan* pl, DevOps<T>& ops, int l, int colour, T* F, T* U, const T* Ec = nullptr,
           T* Dout = nullptr) {
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[l];
  int par0 = hp.p.dim == 1 ? 1 : 0;
  int par = colour == 0 ? par0 : 1 - par0;
  int ncols = (lv.N - par + 1) / 2;
  MarchArgs<T> a = base_args<T>(pl, ops, l);
  a.F = F; a.U = U; a.Out = nullptr;
  a.ld = lv.N; a.ncols = ncols; a.cstride = 2; a.coff = par;
  if (a.split) { a.cstride = 1; a.coff = par ? (int)a.n0 : 0; }   // the colour's contiguous block
  a.dim = hp.p.dim; a.n = lv.n; a.inv_h2 = (T)(1.0 / (lv.h * lv.h));
  if (Ec) { a.Ec = Ec; a.nc = hp.levels[l + 1].n; }
  a.Dout = Dout;
  Timed tm(pl, sizeof(T) == 8 ? MGWR_K_SMOOTH64 : MGWR_K_SMOOTH32, 2.0 * hp.stored * ncols,
           (Dout ? 5.0 : 3.0) * hp.p.M * ncols * sizeof(T));
  HIP_TRY(launch_march<T>(MODE_SMOOTH, a, pl->stream));
  return MGWR_OK;
}

// Defect b - A u on level l.  red_only: on the first colour only.  Right
// after a half-sweep of the second colour the defect there is zero (each of
// its lines was just solved exactly with the same operator), so a defect
// that only feeds the restriction needs the first colour alone.
template <typename T>
// Inj / Inj0 (1D, red_only): the restriction is fused, see MarchArgs.
// natural: the arrays are in natural order whatever the plan's storage (the
// defect entry point).
int defect(mgwr_plan* pl, DevOps<T>& ops, int l, const T* F, T* U, T* Out, bool red_only = false,
           T* Inj = nullptr, T* Inj0 = nullptr, bool natural = false) {
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[l];
  MarchArgs<T> a = base_args<T>(pl, ops, l);
  if (natural) a.split = 0;
  a.F = F; a.U = U; a.Out = Out;
  a.ld = lv.N; a.ncols = lv.N; a.cstride = 1; a.coff = 0;
  if (red_only) {
    const int par0 = hp.p.dim == 1 ? 1 : 0;
    a.ncols = (lv.N - par0 + 1) / 2; a.cstride = 2; a.coff = par0;
    if (a.split) { a.cstride = 1; a.coff = 0; }   // the first colour is the first block
  }
  a.dim = hp.p.dim; a.n = lv.n; a.inv_h2 = (T)(1.0 / (lv.h * lv.h));
  if (Inj) { a.Inj = Inj; a.Inj0 = Inj0; a.nc = hp.levels[l + 1].n; }
  Timed tm(pl, sizeof(T) == 8 ? MGWR_K_DEFECT64 : MGWR_K_DEFECT32, 2.0 * hp.stored * a.ncols,
           3.0 * hp.p.M * a.ncols * sizeof(T));
  HIP_TRY(launch_march<T>(MODE_RESID, a, pl->stream));
  return MGWR_OK;
}

// The float64 defect b - A u of a mixed-precision refinement step on level
// 0, written rounded to float32 as the next inner right-hand side, with each
// chain's max |r| in norms[chunk] (one pass instead of the defect, a cast and
// a norm over the float64 array).
int defect_rhs32(mgwr_plan* pl, const double* F, double* U, float* rhs32, double* norms) {
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[0];
  MarchArgs<double> a = base_args<double>(pl, pl->d64, 0);
  a.F = F; a.U = U; a.Out = nullptr; a.Out32 = rhs32; a.norm_out = norms;
  a.ld = lv.N; a.ncols = lv.N; a.cstride = 1; a.coff = 0;
  a.dim = hp.p.dim; a.n = lv.n; a.inv_h2 = 1.0 / (lv.h * lv.h);
  Timed tm(pl, MGWR_K_DEFECT64, 2.0 * hp.stored * a.ncols, 2.5 * hp.p.M * a.ncols * sizeof(double));
  HIP_TRY(launch_march<double>(MODE_RESID, a, pl->stream));
  return MGWR_OK;
}

int read_scalar(mgwr_plan* pl, double* host);

// The norm ||b - A u||_inf on level 0 (float64) without storing the defect:
// each chain's max |r| goes to norms[chunk], reduced into pl->scal and read.
int defect_norm(mgwr_plan* pl, const double* F, double* U, double* norms, double* host) {
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[0];
  MarchArgs<double> a = base_args<double>(pl, pl->d64, 0);
  a.F = F; a.U = U; a.Out = nullptr; a.norm_out = norms;
  a.ld = lv.N; a.ncols = lv.N; a.cstride = 1; a.coff = 0;
  a.dim = hp.p.dim; a.n = lv.n; a.inv_h2 = 1.0 / (lv.h * lv.h);
  {
    Timed tm(pl, MGWR_K_DEFECT64, 2.0 * hp.stored * a.ncols, 2.0 * hp.p.M * a.ncols * sizeof(double));
    HIP_TRY(launch_march<double>(MODE_RESID, a, pl->stream));
  }
  HIP_TRY(launch_maxabs_parts(norms, (int)((lv.N + 15) / 16), pl->scal, pl->stream));
  return read_scalar(pl, host);
}

// The same norm right after a cycle whose last half-sweep wrote its changes
// to d (zebra_stopping_test): the defect is zero on the second colour and a
// stencil of d on the first.
int zebra_norm(mgwr_plan* pl, const double* d, double* norms, double* host) {
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[0];
  int nparts = (int)std::min<long long>(4096, (long long)mgwr_plan::kMaxPipeCycles * ((lv.N + 15) / 16));
  {
    Timed tm(pl, MGWR_K_DEFECT64, 0.0, 2.5 * hp.p.M * lv.N * sizeof(double));
    HIP_TRY(launch_zebra_norm(d, lv.n, hp.p.M, 1.0 / (lv.h * lv.h), norms, &nparts, pl->stream));
  }
  HIP_TRY(launch_maxabs_parts(norms, nparts, pl->scal, pl->stream));
  return read_scalar(pl, host);
}

template <typename T>
int coarse_cycle(mgwr_plan* pl, int l);

// Zebra defects (2D, colour-split storage, at least one pre-smoothing sweep):
// the defect that feeds the restriction is formed from the changes the last
// second-colour half-sweep made (see MarchArgs::Dout) instead of by a defect
// march, which saves the H-matrix product of the first colour.  The result
// equals the defect b - A u up to the rounding of the line solves.
bool zebra_defects(const mgwr_plan* pl) {
  const HostPlan& hp = pl->hp;
  return pl->zebra && hp.p.dim == 2 && pl->split && hp.p.nu1 >= 1 &&
         (long long)hp.levels[0].n * hp.levels[0].n < (1ll << 31);
}
// ... and the stopping test's norm from the last post-smoothing sweep's
// changes on level 0 (the second colour's defect is zero after it).
bool zebra_stopping_test(const mgwr_plan* pl) {
  const HostPlan& hp = pl->hp;
  return pl->zebra && hp.p.dim == 2 && pl->split && hp.p.nu2 >= 1 && hp.levels.size() >= 2 &&
         (long long)hp.levels[0].n * hp.levels[0].n < (1ll << 31);
}

// One cycle of Algorithm 2 on level l: ops.F[l] is the right-hand side,
// ops.U[l] the iterate (level 0 arrays are supplied through F0/U0).  From
// level coarse_l on, where a half-sweep has too few chains to fill the GPU,
// the whole remaining cycle is one pipelined launch.
// dlast: when set, the last post-smoothing half-sweep writes its changes
// there (for a zebra stopping test on level 0).
template <typename T>
int cycle(mgwr_plan* pl, DevOps<T>& ops, int l, T* dlast = nullptr) {
  const HostPlan& hp = pl->hp;
  const int L = (int)hp.levels.size();
  const int M = hp.p.M;
  T* F = ops.F[l];
  T* U = ops.U[l];
  int rc;
  if (l >= 1 && l == pl->coarse_l) return coarse_cycle<T>(pl, l);
  if (l == L - 1) {  // coarsest grid (one point): the line solve is the direct solve
    if ((rc = smooth<T>(pl, ops, l, 0, F, U))) return rc;
    if ((rc = smooth<T>(pl, ops, l, 1, F, U))) return rc;
    return MGWR_OK;
  }
  const TransferFusion fz = transfer_fusion(hp);
  const bool zebra = !fz.restrict_in_defect && zebra_defects(pl);
  for (int s = 0; s < hp.p.nu1; ++s) {
    if ((rc = smooth<T>(pl, ops, l, 0, F, U))) return rc;
    if ((rc = smooth<T>(pl, ops, l, 1, F, U, nullptr, (zebra && s == hp.p.nu1 - 1) ? ops.R[l] : nullptr)))
      return rc;
  }
  const bool red_only = hp.p.nu1 >= 1;   // the pre-smoothing ended with a second-colour half-sweep
  if (zebra) {
    {
      Timed tm(pl, MGWR_K_RESTRICT, 0.0, (double)M * (0.5 * hp.levels[l].N + 2.0 * hp.levels[l + 1].N) * sizeof(T));
      const T inv_h2 = (T)(1.0 / (hp.levels[l].h * hp.levels[l].h));
      HIP_TRY(launch_restrict_zebra<T>(ops.R[l], ops.F[l + 1], hp.levels[l].n, M, inv_h2, pl->stream));
    }
    HIP_TRY(launch_fill<T>(ops.U[l + 1], (long long)M * hp.levels[l + 1].N, (T)0, pl->stream));
  } else if (fz.restrict_in_defect) {
    if ((rc = defect<T>(pl, ops, l, F, U, nullptr, true, ops.F[l + 1], ops.U[l + 1]))) return rc;
  } else {
    if ((rc = defect<T>(pl, ops, l, F, U, ops.R[l], red_only))) return rc;
    {
      Timed tm(pl, MGWR_K_RESTRICT, 0.0,
               (double)M * ((red_only ? 0.5 : 1.0) * hp.levels[l].N + 2.0 * hp.levels[l + 1].N) * sizeof(T));
      HIP_TRY(launch_restrict<T>(ops.R[l], ops.F[l + 1], hp.p.dim, hp.levels[l].n, M, red_only, pl->split,
                                 pl->stream));
    }
    HIP_TRY(launch_fill<T>(ops.U[l + 1], (long long)M * hp.levels[l + 1].N, (T)0, pl->stream));
  }
  for (int gm = 0; gm < hp.p.gamma; ++gm)
    if ((rc = cycle<T>(pl, ops, l + 1))) return rc;
  if (!fz.prolong_in_smooth) {
    Timed tm(pl, MGWR_K_PROLONG, 0.0,
             (double)M * ((hp.p.nu2 >= 1 ? 1.0 : 2.0) * hp.levels[l].N + hp.levels[l + 1].N) * sizeof(T));
    HIP_TRY(launch_prolong<T>(ops.U[l + 1], U, hp.p.dim, hp.levels[l].n, M, hp.p.nu2 >= 1, pl->split, pl->stream));
  }
  for (int s = 0; s < hp.p.nu2; ++s) {
    const T* Ec = (fz.prolong_in_smooth && s == 0) ? ops.U[l + 1] : nullptr;
    if ((rc = smooth<T>(pl, ops, l, 0, F, U, Ec))) return rc;
    if ((rc = smooth<T>(pl, ops, l, 1, F, U, nullptr, s == hp.p.nu2 - 1 ? dlast : nullptr))) return rc;
  }
  return MGWR_OK;
}


// ---- time-pipelined cycles ------------------------------------------------
// Stage list of one cycle of Algorithm 2 on level l (float64), appended to
// `out`; `prev` is the index of the stage whose output the first new stage
// consumes.  Returns the index of the last stage appended.
int append_cycle_stages(mgwr_plan* pl, int l, int prev, std::vector<Stage>& out, bool f32 = false) {
  const HostPlan& hp = pl->hp;
  const int L = (int)hp.levels.size();
  const Level& lv = hp.levels[l];
  DevOps<double>& ops = pl->d64;
  DevOps<float>& o32 = pl->d32;
  const int kofs = f32 ? STG_SMOOTH32 : 0;  // float32 kinds follow the float64 ones
  auto base = [&](int kind) {
    Stage st{};
    st.kind = kind;
    st.prev = prev;
    st.nleaf = (int)hp.pk.leaves.size();
    st.leaves = pl->leaves;
    return st;
  };
  auto push = [&](Stage& st) {
    out.push_back(st);
    prev = (int)out.size() - 1;
  };
  auto smooth_stage = [&](int colour, bool with_ec = false, bool dout = false) {
    int par0 = hp.p.dim == 1 ? 1 : 0;
    int par = colour == 0 ? par0 : 1 - par0;
    int ncols = (lv.N - par + 1) / 2;
    if (ncols <= 0) return;
    Stage st = base(STG_SMOOTH + kofs);
    if (!f32) {
      st.m = base_args<double>(pl, ops, l);
      st.m.F = ops.F[l]; st.m.U = ops.U[l]; st.m.Out = nullptr;
      st.m.ld = lv.N; st.m.ncols = ncols; st.m.cstride = 2; st.m.coff = par;
      if (st.m.split) { st.m.cstride = 1; st.m.coff = par ? (int)st.m.n0 : 0; }
      st.m.dim = hp.p.dim; st.m.n = lv.n; st.m.inv_h2 = 1.0 / (lv.h * lv.h);
      if (with_ec) { st.m.Ec = ops.U[l + 1]; st.m.nc = hp.levels[l + 1].n; }
      if (dout) st.m.Dout = ops.R[l];
    } else {
      st.mf = base_args<float>(pl, o32, l);
      st.mf.F = o32.F[l]; st.mf.U = o32.U[l]; st.mf.Out = nullptr;
      st.mf.ld = lv.N; st.mf.ncols = ncols; st.mf.cstride = 2; st.mf.coff = par;
      if (st.mf.split) { st.mf.cstride = 1; st.mf.coff = par ? (int)st.mf.n0 : 0; }
      st.mf.dim = hp.p.dim; st.mf.n = lv.n; st.mf.inv_h2 = (float)(1.0 / (lv.h * lv.h));
      if (with_ec) { st.mf.Ec = o32.U[l + 1]; st.mf.nc = hp.levels[l + 1].n; }
      if (dout) st.mf.Dout = o32.R[l];
    }
    st.nchunks = (ncols + 15) / 16;
    push(st);
  };
  const TransferFusion fz = transfer_fusion(hp);
  if (l == L - 1) {
    smooth_stage(0);
    smooth_stage(1);
    return prev;
  }
  // Zebra restriction: the last pre-smoothing half-sweep (second colour)
  // writes its changes d, and the restriction of the first-colour defect
  // (1/h^2 times the sum of d over a point's neighbours) is formed from them:
  // no defect stage (see zebra_defects for the staged form)
  const bool zebra1 = pl->zebra && hp.p.nu1 >= 1 &&
                      (hp.p.dim == 1 || (long long)lv.n * lv.n < (1ll << 31));
  for (int s2 = 0; s2 < hp.p.nu1; ++s2) { smooth_stage(0); smooth_stage(1, false, zebra1 && s2 == hp.p.nu1 - 1); }
  // after a second-colour half-sweep the defect vanishes on that colour: the
  // defect stage covers the first colour and the restriction reads only it
  const bool red_only = hp.p.nu1 >= 1;
  if (zebra1) {
    const Level& lc1 = hp.levels[l + 1];
    Stage st = base(STG_RESTRICT + kofs);
    if (!f32) { st.src = ops.R[l]; st.dst = ops.F[l + 1]; st.zero = ops.U[l + 1]; }
    else { st.src = o32.R[l]; st.dst = o32.F[l + 1]; st.zero = o32.U[l + 1]; }
    st.dim = hp.p.dim; st.nf = lv.n; st.nc = lc1.n;
    st.red_only = 1;
    st.split = pl->split && hp.p.dim == 2 ? 1 : 0;
    st.zebra = 1;
    st.zscale = 1.0 / (lv.h * lv.h);
    st.nchunks = (lc1.N + kStencilCols - 1) / kStencilCols;
    push(st);
  } else {
    const int par0 = hp.p.dim == 1 ? 1 : 0;
    const int ncols = red_only ? (lv.N - par0 + 1) / 2 : lv.N;
    // colour-split storage: the first colour is the first block (coff 0)
    const bool split = pl->split && hp.p.dim == 2;
    const int cstride = red_only && !split ? 2 : 1, coff = red_only && !split ? par0 : 0;
    Stage st = base(STG_RESID + kofs);
    if (!f32) {
      st.m = base_args<double>(pl, ops, l);
      st.m.F = ops.F[l]; st.m.U = ops.U[l]; st.m.Out = ops.R[l];
      st.m.ld = lv.N; st.m.ncols = ncols; st.m.cstride = cstride; st.m.coff = coff;
      st.m.dim = hp.p.dim; st.m.n = lv.n; st.m.inv_h2 = 1.0 / (lv.h * lv.h);
      if (fz.restrict_in_defect) {
        st.m.Out = nullptr; st.m.Inj = ops.F[l + 1]; st.m.Inj0 = ops.U[l + 1]; st.m.nc = hp.levels[l + 1].n;
      }
    } else {
      st.mf = base_args<float>(pl, o32, l);
      st.mf.F = o32.F[l]; st.mf.U = o32.U[l]; st.mf.Out = o32.R[l];
      st.mf.ld = lv.N; st.mf.ncols = ncols; st.mf.cstride = cstride; st.mf.coff = coff;
      st.mf.dim = hp.p.dim; st.mf.n = lv.n; st.mf.inv_h2 = (float)(1.0 / (lv.h * lv.h));
      if (fz.restrict_in_defect) {
        st.mf.Out = nullptr; st.mf.Inj = o32.F[l + 1]; st.mf.Inj0 = o32.U[l + 1]; st.mf.nc = hp.levels[l + 1].n;
      }
    }
    st.nchunks = (ncols + 15) / 16;
    push(st);
  }
  const Level& lc = hp.levels[l + 1];
  if (!fz.restrict_in_defect && !zebra1) {
    Stage st = base(STG_RESTRICT + kofs);
    if (!f32) { st.src = ops.R[l]; st.dst = ops.F[l + 1]; st.zero = ops.U[l + 1]; }
    else { st.src = o32.R[l]; st.dst = o32.F[l + 1]; st.zero = o32.U[l + 1]; }
    st.dim = hp.p.dim; st.nf = lv.n; st.nc = lc.n;
    st.red_only = red_only ? 1 : 0;
    st.split = pl->split && hp.p.dim == 2 ? 1 : 0;
    st.nchunks = (lc.N + kStencilCols - 1) / kStencilCols;
    push(st);
  }
  for (int gm = 0; gm < hp.p.gamma; ++gm) prev = append_cycle_stages(pl, l + 1, prev, out, f32);
  if (!fz.prolong_in_smooth) {
    Stage st = base(STG_PROLONG + kofs);
    st.prev = prev;
    if (!f32) { st.src = ops.U[l + 1]; st.dst = ops.U[l]; }
    else { st.src = o32.U[l + 1]; st.dst = o32.U[l]; }
    st.dim = hp.p.dim; st.nf = lv.n; st.nc = lc.n;
    st.black_only = hp.p.nu2 >= 1 ? 1 : 0;   // a first-colour half-sweep follows
    st.split = pl->split && hp.p.dim == 2 ? 1 : 0;
    const long long nq = st.black_only ? (lv.N - (hp.p.dim == 1 ? 0 : 1) + 1) / 2 : lv.N;
    st.nchunks = (int)((nq + kStencilCols - 1) / kStencilCols);
    push(st);
  }
  for (int s2 = 0; s2 < hp.p.nu2; ++s2) { smooth_stage(0, fz.prolong_in_smooth && s2 == 0); smooth_stage(1); }
  return prev;
}

// Algorithmic work of one stage, added to flops / bytes: a march 2 S flops
// and 3 M words per column; a restriction reads the fine defect (first colour
// only: half) and writes the coarse right-hand side and iterate; a
// prolongation reads the coarse correction and reads and writes the fine
// iterate (second colour only: half); the precision hand-overs read and
// write one row each.
void stage_work(const mgwr_plan* pl, const Stage& x, double& flops, double& bytes) {
  const HostPlan& hp = pl->hp;
  if (x.kind == STG_SMOOTH || x.kind == STG_RESID) {
    flops += 2.0 * hp.stored * x.m.ncols;
    bytes += 3.0 * hp.p.M * x.m.ncols * sizeof(double);
  } else if (x.kind == STG_SMOOTH32 || x.kind == STG_RESID32) {
    flops += 2.0 * hp.stored * x.mf.ncols;
    bytes += 3.0 * hp.p.M * x.mf.ncols * sizeof(float);
  } else if (x.kind == STG_CAST || x.kind == STG_CORRECT) {
    bytes += (x.kind == STG_CAST ? 16.0 : 20.0) * hp.p.M * x.npoints;
  } else {
    const double Nf = hp.p.dim == 1 ? x.nf : (double)x.nf * x.nf;
    const double Nc = hp.p.dim == 1 ? x.nc : (double)x.nc * x.nc;
    const double w = (x.kind == STG_RESTRICT || x.kind == STG_PROLONG) ? 8.0 : 4.0;
    const double words = (x.kind == STG_RESTRICT || x.kind == STG_RESTRICT32)
                             ? (x.red_only ? 0.5 : 1.0) * Nf + 2 * Nc
                             : Nc + 2 * (x.black_only ? 0.5 : 1.0) * Nf;
    bytes += words * hp.p.M * w;
  }
}

// Appends K cycles of plan pl.  The defect of the full system (whose
// per-work-item norms go to norms[c * chunks + item]) follows every cycle
// when `every` is set, else only the last one.  Stage indices (prev) are
// relative to the first stage appended.
void build_plan_stages(mgwr_plan* pl, const double* b, double* u, int K, double* norms,
                       std::vector<Stage>& out, bool every = true, bool first_src_is_b = true) {
  const HostPlan& hp = pl->hp;
  const int nleaf = (int)hp.pk.leaves.size();
  pl->d64.F[0] = const_cast<double*>(b);
  pl->d64.U[0] = u;
  std::vector<Stage> st;
  int prev = -1;
  int per_cycle = -1;
  const long long N0 = hp.levels[0].N;
  for (int c = 0; c < K; ++c) {
    if (!pl->mixed) {
      prev = append_cycle_stages(pl, 0, prev, st);
    } else {
      // one refinement step: float32 right-hand side from the float64 defect
      // (b itself before the first correction of a zero iterate), inner
      // float32 cycles on A e = r from e = 0, u += e, float64 defect
      Stage cs{};
      cs.kind = STG_CAST;
      cs.prev = prev;
      cs.nleaf = nleaf;
      cs.leaves = pl->leaves;
      cs.src = (c == 0 && first_src_is_b) ? (const void*)b : (const void*)pl->d64.R[0];
      cs.dst = pl->d32.F[0];
      cs.zero = pl->d32.U[0];
      cs.npoints = N0;
      cs.nchunks = (int)((N0 + kStencilCols - 1) / kStencilCols);
      st.push_back(cs);
      prev = (int)st.size() - 1;
      for (int ic = 0; ic < hp.p.inner_cycles; ++ic) prev = append_cycle_stages(pl, 0, prev, st, true);
      Stage co{};
      co.kind = STG_CORRECT;
      co.prev = prev;
      co.nleaf = nleaf;
      co.leaves = pl->leaves;
      co.src = pl->d32.U[0];
      co.dst = u;
      co.npoints = N0;
      co.nchunks = cs.nchunks;
      st.push_back(co);
      prev = (int)st.size() - 1;
      every = true;  // the next step's right-hand side is this defect
    }
    if (per_cycle < 0) per_cycle = (int)st.size() + 1;
    if (!every && c + 1 < K) continue;
    Stage nd{};
    nd.kind = STG_RESID;
    nd.prev = prev;
    nd.nleaf = nleaf;
    nd.leaves = pl->leaves;
    nd.m = base_args<double>(pl, pl->d64, 0);
    const Level& lv = hp.levels[0];
    nd.m.F = b; nd.m.U = u; nd.m.Out = pl->d64.R[0];
    nd.m.ld = lv.N; nd.m.ncols = lv.N; nd.m.cstride = 1; nd.m.coff = 0;
    nd.m.dim = hp.p.dim; nd.m.n = lv.n; nd.m.inv_h2 = 1.0 / (lv.h * lv.h);
    nd.nchunks = (lv.N + 15) / 16;
    nd.norm_out = norms + (size_t)(every ? c : 0) * nd.nchunks;
    st.push_back(nd);
    prev = (int)st.size() - 1;
  }
  pl->stages_per_cycle = per_cycle;
  pl->norm_chunks = (hp.levels[0].N + 15) / 16;
  pl->cycle_flops = pl->cycle_bytes = 0.0;
  for (int i = 0; i < per_cycle; ++i) stage_work(pl, st[i], pl->cycle_flops, pl->cycle_bytes);
  out.insert(out.end(), st.begin(), st.end());
}

// Task offsets (stage order) and counter offsets.
void assign_offsets(std::vector<Stage>& st) {
  int task = 0;
  long long cnt = 0;
  for (auto& x : st) {
    x.task0 = task;
    task += x.nchunks;
    x.cnt_off = (int)cnt;
    cnt += x.nleaf;
  }
}

// Schedule choice: a staged launch of the finest smoother has N/32 chains of
// 16 columns; below kAutoPipelineChains of them the GPU is mostly idle and the
// pipelined schedule wins (measured: 1D n=1023 pipelines 9x faster, 2D n=255
// with 2032 chains is faster staged).
constexpr int kAutoPipelineChains = 256;

// In a staged cycle, the levels from the first one whose half-sweeps have at
// most kCoarsePipelineChains chains run as one pipelined launch.  Measured on
// 2D n = 255, M = 1024: from level 3 (n = 31, 31 chains) 60.4 ms per solve,
// from level 2 (125 chains) 62.9 ms, from level 1 (505 chains) 66.6 ms, from
// level 4 (8 chains) 67.0 ms; batches of uneven 2D instances 3 % faster than
// from level 2.
constexpr int kCoarsePipelineChains = 64;

// Solved side by side with enough other staged instances to keep every
// worker busy, a plan's coarse launch starts one level below the rule's
// (when that level exists): the small staged launches it then keeps fill
// the gaps the other instances leave, and its own latency-bound coarse
// launch is shorter.  Measured on the 64-instance batch (40 staged): 2D
// n = 127 and 255 from n = 15 instead of 31, 937 against 953 ms per batch
// solve; two levels below 960 ms, one above 1,059 ms, no coarse launch
// 1,001 ms.  Two instances side by side do not fill the GPU and keep the
// rule (pairs of 2D n = 255, M = 1024 instances: mixed 69.9 ms with the
// shift against 65.8, mixed with warm starts 57.5 against 55.3, float64
// with warm starts 67.9 against 66.5, float64 76.1 against 77.0).
constexpr int kSideCoarseShift = 1;

// First level below the finest whose half-sweeps have at most
// kCoarsePipelineChains chains (0: none).
int coarse_switch_level(const HostPlan& hp) {
  const int L = (int)hp.levels.size();
  for (int l = 1; l < L; ++l)
    if ((hp.levels[l].N + 31) / 32 <= kCoarsePipelineChains) return l;
  return 0;
}

// The coarse part of a staged cycle as one pipelined launch on the plan's
// own table, counters and flags.  The stage image depends only on the plan's
// internal arrays, so it is built and uploaded once per binding.  The abort
// flag is cleared when a staged solve starts and read when it ends.
template <typename T>
int coarse_cycle(mgwr_plan* pl, int l) {
  const int w = sizeof(T) == 4 ? 1 : 0;
  std::vector<Stage>& st = pl->coarse_stages[w];
  if (st.empty()) {
    // with defect stages: these latency-bound levels ran 2 % slower with
    // zebra restriction stages (2D n = 255, levels 3-7)
    const bool zebra = pl->zebra;
    pl->zebra = false;
    append_cycle_stages(pl, l, -1, st, w == 1);
    pl->zebra = zebra;
    assign_offsets(st);
    if ((long long)st.size() > stages_per_cycle_bound(pl->hp)) {
      st.clear();
      return fail(MGWR_ERR_STATE, "internal error: coarse stage table exceeds its workspace");
    }
    long long cnt = 0;
    int tasks = 0;
    double flops = 0.0, bytes = 0.0;
    for (const Stage& x : st) {
      cnt += x.nleaf;
      tasks = x.task0 + x.nchunks;
      const int nc = w ? x.mf.ncols : x.m.ncols;
      if (x.kind == STG_SMOOTH + (w ? STG_SMOOTH32 : 0) || x.kind == STG_RESID + (w ? STG_SMOOTH32 : 0)) {
        flops += 2.0 * pl->hp.stored * nc;
        bytes += 3.0 * pl->hp.p.M * nc * sizeof(T);
      }
    }
    pl->coarse_cnt[w] = cnt;
    pl->coarse_tasks[w] = tasks;
    pl->coarse_flops[w] = flops;
    pl->coarse_bytes[w] = bytes;
    pl->coarse_up[w] = false;
  }
  if (!pl->coarse_up[w]) {
    HIP_TRY(hipMemcpyAsync(pl->cstages_dev[w], st.data(), st.size() * sizeof(Stage), hipMemcpyHostToDevice,
                           pl->stream));
    pl->coarse_up[w] = true;
  }
  PipeArgs pa{};   // every field zero (no per-XCD queues unless set)
  pa.stages = pl->cstages_dev[w];
  pa.nstages = (int)st.size();
  pa.ntasks = pl->coarse_tasks[w];
  pa.counters = pl->ccounters;
  pa.ticket = pl->cflags;
  pa.abortf = pl->cflags + 1;
  pa.spin_limit = pl->spin_limit;
  size_t lds = march_lds_bytes<double>(base_args<double>(pl, pl->d64, 0));
  if (pl->mixed) lds = std::max(lds, march_lds_bytes<float>(base_args<float>(pl, pl->d32, 0)));
  Timed tm(pl, MGWR_K_COARSE, pl->coarse_flops[w], pl->coarse_bytes[w]);
  HIP_TRY(launch_fill_int(pl->ccounters, pl->coarse_cnt[w], 0, pl->stream));
  HIP_TRY(launch_fill_int(pl->cflags, 1, 0, pl->stream));
  HIP_TRY(launch_pipeline(pa, lds, pl->stream));
  return MGWR_OK;
}
// Choices measured by mgwr_plan_autotune, shared by every plan of the same
// shape in the process: (dim, n, M, precision, inner cycles, k) -> schedule,
// and for the staged schedule the march prefetch and the coarse level.
using TuneKey = std::tuple<int, int, int, int, int, int>;
struct TuneChoice {
  int sched = 0, prefetch = 0, coarse = -1;
  int layout = MGWR_LAYOUT_AUTO;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tuned;

TuneKey tune_key(const mgwr_plan* pl) {
  const mgwr_params& p = pl->hp.p;
  return TuneKey(p.dim, p.n, p.M, p.precision, p.inner_cycles, p.k);
}

bool use_pipeline(const mgwr_plan* pl) {
  const int sched = pl->hp.p.schedule;
  if (sched == MGWR_SCHED_PIPELINED) return true;
  if (sched == MGWR_SCHED_STAGED) return false;
  if (pl->tuned) return pl->tuned == MGWR_SCHED_PIPELINED;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(pl));
    if (it != g_tuned.end()) return it->second.sched == MGWR_SCHED_PIPELINED;
  }
  return (pl->hp.levels[0].N + 31) / 32 <= kAutoPipelineChains;
}

// Prefetch and coarse level a staged solve of `pl` uses: set on the plan,
// else measured for its shape (AUTO schedule), else the rules.
void staging_choice(const mgwr_plan* pl, int* prefetch, int* coarse) {
  *prefetch = 0;
  *coarse = -1;
  if (pl->staging_set) {
    *prefetch = pl->set_prefetch;
    *coarse = pl->set_coarse;
  } else if (pl->hp.p.schedule == MGWR_SCHED_AUTO) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(pl));
    if (it != g_tuned.end() && it->second.sched == MGWR_SCHED_STAGED) {
      *prefetch = it->second.prefetch;
      *coarse = it->second.coarse;
    }
  }
  if (*coarse < 0) {
    *coarse = coarse_switch_level(pl->hp);
    if (pl->side_by_side && *coarse > 0 && *coarse + kSideCoarseShift < (int)pl->hp.levels.size())
      *coarse += kSideCoarseShift;
  }
}

// Storage of a 2D solve: set on the plan, else measured for its shape (AUTO
// schedule), else colour-split.  1D is natural.
bool split_choice(const mgwr_plan* pl) {
  if (pl->hp.p.dim != 2) return false;
  if (pl->set_layout != MGWR_LAYOUT_AUTO) return pl->set_layout == MGWR_LAYOUT_SPLIT;
  if (pl->hp.p.schedule == MGWR_SCHED_AUTO) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(pl));
    if (it != g_tuned.end() && it->second.layout != MGWR_LAYOUT_AUTO) return it->second.layout == MGWR_LAYOUT_SPLIT;
  }
  return true;
}

// Puts the storage choice in force; stage images built for the other one
// are dropped (they hold the storage flag and column offsets).
void apply_layout(mgwr_plan* pl) {
  const bool sp = split_choice(pl);
  if (sp == pl->split) return;
  pl->split = sp;
  pl->stages_f = nullptr;
  pl->stages_u = nullptr;
  for (int w = 0; w < 2; ++w) {
    pl->coarse_stages[w].clear();
    pl->coarse_up[w] = false;
  }
}

// Puts the staged knobs in force; a new coarse level rebuilds the coarse
// stage images (their workspace holds a whole cycle's stages).
void apply_staging(mgwr_plan* pl) {
  int prefetch, coarse;
  staging_choice(pl, &prefetch, &coarse);
  pl->prefetch = prefetch;
  if (coarse != pl->coarse_l) {
    pl->coarse_l = coarse;
    for (int w = 0; w < 2; ++w) {
      pl->coarse_stages[w].clear();
      pl->coarse_up[w] = false;
    }
  }
}

int read_scalar(mgwr_plan* pl, double* host) {
  HIP_TRY(hipMemcpyAsync(host, pl->scal, sizeof(double), hipMemcpyDeviceToHost, pl->stream));
  HIP_TRY(hipStreamSynchronize(pl->stream));
  if (!pl->pending.empty()) drain_timing(pl);
  return MGWR_OK;
}

template <typename T>
int norm_inf(mgwr_plan* pl, const T* x, long long count, double* host) {
  HIP_TRY(launch_maxabs<T>(x, count, pl->part, kNormParts, pl->scal, pl->stream));
  return read_scalar(pl, host);
}

int check_bound(const mgwr_plan* pl) {
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "null plan");
  if (!pl->bound) return fail(MGWR_ERR_STATE, "plan is not bound to a workspace");
  return MGWR_OK;
}

// Device of the calling thread must be the plan's device.
int use_device(mgwr_plan* pl) {
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != pl->device) HIP_TRY(hipSetDevice(pl->device));
  return MGWR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// batched solves

struct mgwr_batch {
  std::vector<mgwr_plan*> plans;
  bool bound = false;
  int device = -1;
  hipStream_t stream = nullptr;
  size_t off_stages = 0, off_counters = 0, off_flags = 0, off_norms = 0, off_xq = 0, total = 0;
  int* xq = nullptr;          // per-XCD task queues of the merged launch
  long long xq_cap = 0;
  bool graph_xq = false;      // the captured graph uses them
  std::vector<size_t> norm_off;  // per plan, in doubles
  Stage* stages_dev = nullptr;
  int* counters = nullptr;
  int* flags_dev = nullptr;
  double* norms = nullptr;
  std::vector<Stage> stages;
  size_t lds = 0;
  bool timing = false;
  mgwr_timing tacc{};
  unsigned spin_limit = kDefaultSpinLimit;   // the smallest bound of its plans
  // replay of an unchanged launch (stage table, counters, grid) as a HIP graph
  bool use_graph = false;
  std::vector<Stage> graph_stages;     // the table the captured graph runs
  long long graph_ncnt = 0;
  int graph_ntasks = 0;
  unsigned graph_spin = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;  // private (the caller's may be the legacy stream, which cannot capture)
  long long graph_replays = 0;
  std::vector<hipStream_t> worker_streams;  // staged instances solved side by side (default priority)
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
    graph_stages.clear();
  }
  ~mgwr_batch() {
    drop_graph();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (hipStream_t s : worker_streams) (void)hipStreamDestroy(s);
  }
};

namespace {

// Prepares an instance: b = f + a_1 g, the initial iterate (zero, given, or
// predicted by the warm-start network), ||b||, res0.  `flags` returns with
// MGWR_GUESS_IN_U set iff u holds a non-zero iterate whose defect is in R64_0.
// A prediction's float64 defect is always evaluated (stats.warm_res0); one
// whose defect is not finite is dropped for the zero iterate here, a finite
// one is judged after its first cycles (see fall_back_to_zero).
int prepare_solve(mgwr_plan* pl, const double* f, const double* g, double tol, double* u, unsigned& flags,
                  mgwr_stats& s, const double*& b, int& status) {
  int rc;
  pl->zebra = tol >= kZebraMinTol;
  const HostPlan& hp = pl->hp;
  const long long N = hp.levels[0].N;
  const long long MN = (long long)hp.p.M * N;
  s = mgwr_stats{};
  s.warm_res0 = std::nan("");
  s.setup_ms = pl->create_ms + pl->bind_ms;
  apply_layout(pl);
  b = f;
  if (pl->split) {
    // colour-split storage: b is formed in it, a given iterate is moved in
    // (through the level-0 defect array, free until the first defect)
    HIP_TRY(launch_rhs0_split(f, g, pl->a1, pl->B0, hp.p.M, N, pl->stream));
    b = pl->B0;
    if ((flags & MGWR_GUESS_IN_U) && !(flags & MGWR_WARM_START)) {
      HIP_TRY(launch_relayout(u, pl->d64.R[0], hp.p.M, N, true, pl->stream));
      HIP_TRY(hipMemcpyAsync(u, pl->d64.R[0], MN * sizeof(double), hipMemcpyDeviceToDevice, pl->stream));
    }
  } else if (g) {
    HIP_TRY(launch_rhs0(f, g, pl->a1, pl->B0, hp.p.M, N, pl->stream));
    b = pl->B0;
  }
  if (!(flags & (MGWR_GUESS_IN_U | MGWR_WARM_START))) HIP_TRY(launch_fill<double>(u, MN, 0.0, pl->stream));
  if ((rc = norm_inf<double>(pl, b, MN, &s.bnorm))) return rc;
  status = MGWR_ERR_NOT_CONVERGED;
  if (!std::isfinite(s.bnorm)) { status = MGWR_ERR_NONFINITE; return MGWR_OK; }
  if (flags & MGWR_WARM_START) {
    if (!pl->net) return fail(MGWR_ERR_STATE, "MGWR_WARM_START needs a network (mgwr_plan_set_warm_start)");
    flags &= ~(unsigned)MGWR_GUESS_IN_U;
    if (s.bnorm > 0.0) {
      const int ns = pl->nslices;
      const int H = hp.p.dim == 1 ? 1 : hp.levels[0].n, W = hp.levels[0].n;
      {
        // gather, inference and interpolation hold the network (its buffers
        // and stream are shared by every plan it is attached to)
        std::lock_guard<std::mutex> lk(net_mutex(pl->net));
        float* xin = net_input_stage(pl->net);
        HIP_TRY(launch_gather_slices(b, pl->rows_dev, ns, N, s.bnorm, (float)hp.p.alpha, (float)(hp.p.r / 10.0),
                                     xin, pl->split, pl->stream));
        HIP_TRY(hipStreamSynchronize(pl->stream));
        const float* y = nullptr;
        if ((rc = net_infer(pl->net, xin, H, W, hp.levels[0].h, &y))) return rc;
        HIP_TRY(hipStreamSynchronize(net_stream(pl->net)));
        HIP_TRY(launch_time_interp(y, pl->rows_dev, ns, pl->tpow, g, hp.p.M, N, s.bnorm, u, pl->split, pl->stream));
        HIP_TRY(hipStreamSynchronize(pl->stream));
      }
      // the prediction's true residual (reported, and the right-hand side of
      // a first refinement step)
      if ((rc = defect<double>(pl, pl->d64, 0, b, u, pl->d64.R[0]))) return rc;
      if ((rc = norm_inf<double>(pl, pl->d64.R[0], MN, &s.warm_res0))) return rc;
      if (std::isfinite(s.warm_res0)) {
        s.used_warm_start = 1;
        flags |= MGWR_GUESS_IN_U;
      }
    }
    if (!(flags & MGWR_GUESS_IN_U)) HIP_TRY(launch_fill<double>(u, MN, 0.0, pl->stream));
  }
  if (flags & MGWR_GUESS_IN_U) {
    if (!s.used_warm_start) {
      if ((rc = defect<double>(pl, pl->d64, 0, b, u, pl->d64.R[0]))) return rc;
      if ((rc = norm_inf<double>(pl, pl->d64.R[0], MN, &s.res0))) return rc;
    } else {
      s.res0 = s.warm_res0;
    }
  } else {
    s.res0 = s.bnorm;
  }
  s.res = s.res0;
  if (!std::isfinite(s.res0)) {
    status = MGWR_ERR_NONFINITE;
  } else if (s.res0 <= tol * s.bnorm) {
    status = MGWR_OK;
  }
  return MGWR_OK;
}

// The end of a solve: a colour-split iterate goes back to the caller's
// natural order (through the level-0 defect array), on stream s.
int finish_solve(mgwr_plan* pl, double* u, hipStream_t s) {
  if (!pl->split) return MGWR_OK;
  const long long N = pl->hp.levels[0].N, M = pl->hp.p.M;
  HIP_TRY(launch_relayout(u, pl->d64.R[0], M, N, false, s));
  HIP_TRY(hipMemcpyAsync(u, pl->d64.R[0], M * N * sizeof(double), hipMemcpyDeviceToDevice, s));
  return MGWR_OK;
}

int batch_fail(int code, const std::string& m) { return fail(code, m); }

// The true-residual judge of a predicted iterate: after the first outer step
// from it (`cycles` cycles), its residual is compared with the one the zero
// iterate reaches in as many cycles, ||b|| rho0^cycles, rho0 the plan's
// average factor of its last converged solve from zero (||b|| itself before
// there is one).  More than kJudgeMargin times that means the prediction did
// worse than no prediction at all; the solve then restarts from zero (the
// cycles spent stay counted).  The margin absorbs the spread of single-cycle
// factors around their mean (a prediction no better than zero, e.g. the zero
// network, is kept: restarting would only repeat its cycles).  A prediction
// that has already met the tolerance is kept.  Returns 1 when it restarted.
constexpr double kJudgeMargin = 2.0;
int fall_back_to_zero(mgwr_plan* pl, const double* b, double* u, mgwr_stats& s, int cycles, double tol, int* rc) {
  *rc = MGWR_OK;
  if (!s.used_warm_start) return 0;
  const double expect = s.bnorm * (pl->rate_zero > 0.0 ? std::pow(pl->rate_zero, (double)cycles) : 1.0);
  if (s.res <= kJudgeMargin * expect || s.res <= tol * s.bnorm) return 0;
  const long long MN = (long long)pl->hp.p.M * pl->hp.levels[0].N;
  s.used_warm_start = 0;
  s.res = s.res0 = s.bnorm;
  hipError_t e = launch_fill<double>(u, MN, 0.0, pl->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(pl->d64.R[0], b, MN * sizeof(double), hipMemcpyDeviceToDevice, pl->stream);
  if (e != hipSuccess) *rc = fail(MGWR_ERR_HIP, std::string("warm-start fall back: ") + hipGetErrorString(e));
  return 1;
}

}  // namespace

// Pipelined solve of plans[0..n) (float64) with the stage table, counters,
// flags and norms of `bt` (a batch, or one plan's own regions).
// Launch of the merged stage table: counters and flags cleared, then the
// pipeline kernel; replayed from a captured graph when the table, counter
// count and grid equal those of the graph (batches with graphs enabled).
namespace {
// Per-XCD work queues of pipelined launches (PipeArgs::xq): off by default
// (mgwr_set_xcd_queues; measured slower, see the header), used on a device
// once a probe launch has shown that workgroup b runs on XCD b mod
// kXcdQueues.
std::atomic<int> g_xcd_queues{0};
std::mutex g_xcd_mu;
std::map<int, bool> g_xcd_ok;   // device -> round-robin dispatch confirmed

// Runs the probe once per device, on `scratch` (64 ints of the caller's
// workspace); the result is kept for the process.
int check_xcd_dispatch(int device, int* scratch, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_xcd_mu);
  if (g_xcd_ok.count(device)) return MGWR_OK;
  int h[64];
  HIP_TRY(launch_xcc_probe(scratch, 64, s));
  HIP_TRY(hipMemcpyAsync(h, scratch, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  bool ok = true;
  for (int b = 0; b < 64; ++b) ok = ok && h[b] == b % kXcdQueues;
  g_xcd_ok[device] = ok;
  return MGWR_OK;
}

bool xcd_dispatch_ok(int device) {
  std::lock_guard<std::mutex> lk(g_xcd_mu);
  auto it = g_xcd_ok.find(device);
  return it != g_xcd_ok.end() && it->second;
}

// Per-XCD queues of a stage table with ntasks work items.  Each round (the
// stages at one position of the merged instances' lists) is cut into
// kXcdQueues contiguous blocks of nearly equal size, block x to queue x: an
// instance's work items of every round land on the same XCDs, whose L2 then
// holds its H-matrix rows for all its stages.  The queues are then brought
// to the lengths the dispatch gives each XCD (workgroup b on XCD b mod
// kXcdQueues) by moving the latest tasks of longer queues, and sorted, so
// each lists its tasks in stage order.
void build_xcd_queues(const std::vector<Stage>& st, int ntasks, std::vector<int>& q, int* off, int* len) {
  std::vector<std::vector<int>> lists(kXcdQueues);
  for (size_t i = 0; i < st.size();) {
    size_t j = i;
    long long n = 0;
    while (j < st.size() && st[j].round == st[i].round) n += st[j++].nchunks;
    long long pos = 0;
    for (size_t k = i; k < j; ++k)
      for (int c = 0; c < st[k].nchunks; ++c, ++pos) lists[(int)(pos * kXcdQueues / n)].push_back(st[k].task0 + c);
    i = j;
  }
  std::vector<int> want(kXcdQueues);
  for (int x = 0; x < kXcdQueues; ++x) want[x] = ntasks > x ? (ntasks - x + kXcdQueues - 1) / kXcdQueues : 0;
  std::vector<int> spare;
  for (int x = 0; x < kXcdQueues; ++x)
    while ((int)lists[x].size() > want[x]) {
      spare.push_back(lists[x].back());
      lists[x].pop_back();
    }
  for (int x = 0; x < kXcdQueues; ++x)
    while ((int)lists[x].size() < want[x] && !spare.empty()) {
      lists[x].push_back(spare.back());
      spare.pop_back();
    }
  q.clear();
  for (int x = 0; x < kXcdQueues; ++x) {
    std::sort(lists[x].begin(), lists[x].end());
    off[x] = (int)q.size();
    len[x] = (int)lists[x].size();
    q.insert(q.end(), lists[x].begin(), lists[x].end());
  }
}
}  // namespace

int launch_batch_table(mgwr_batch* bt, long long ncnt, int ntasks) {
  bt->spin_limit = kDefaultSpinLimit;
  for (const mgwr_plan* p : bt->plans) bt->spin_limit = std::min(bt->spin_limit, p->spin_limit);
  PipeArgs pa{};   // every field zero (no per-XCD queues unless set)
  pa.stages = bt->stages_dev;
  pa.nstages = (int)bt->stages.size();
  pa.ntasks = ntasks;
  pa.counters = bt->counters;
  pa.ticket = bt->flags_dev;
  pa.abortf = bt->flags_dev + 1;
  pa.spin_limit = bt->spin_limit;
  pa.xq = nullptr;
  pa.xq_ticket = bt->flags_dev + 2;
  const bool use_xq = g_xcd_queues.load() != 0 && bt->xq && ntasks <= bt->xq_cap && xcd_dispatch_ok(bt->device);
  std::vector<int> q;
  if (use_xq) {
    build_xcd_queues(bt->stages, ntasks, q, pa.xq_off, pa.xq_len);
    if ((int)q.size() != ntasks) return fail(MGWR_ERR_STATE, "internal error: XCD queues do not hold every task");
    pa.xq = bt->xq;
  }
  const bool same = bt->graph_exec && bt->graph_ncnt == ncnt && bt->graph_ntasks == ntasks &&
                    bt->graph_spin == bt->spin_limit && bt->graph_xq == use_xq &&
                    bt->graph_stages.size() == bt->stages.size() &&
                    std::memcmp(bt->graph_stages.data(), bt->stages.data(), bt->stages.size() * sizeof(Stage)) == 0;
  if (same) {
    HIP_TRY(hipGraphLaunch(bt->graph_exec, bt->stream));
    bt->graph_replays++;
    return MGWR_OK;
  }
  HIP_TRY(hipMemcpyAsync(bt->stages_dev, bt->stages.data(), bt->stages.size() * sizeof(Stage),
                         hipMemcpyHostToDevice, bt->stream));
  if (use_xq) HIP_TRY(hipMemcpyAsync(bt->xq, q.data(), q.size() * sizeof(int), hipMemcpyHostToDevice, bt->stream));
  if (!bt->use_graph) {
    HIP_TRY(launch_fill_int(bt->counters, ncnt, 0, bt->stream));
    HIP_TRY(launch_fill_int(bt->flags_dev, 2 + kXcdQueues, 0, bt->stream));
    HIP_TRY(launch_pipeline(pa, bt->lds, bt->stream));
    return MGWR_OK;
  }
  // capture on the private stream (nothing runs while capturing): fill
  // kernels (no memset nodes) and the pipeline kernel; the graph is then
  // launched on the batch's stream after the table upload above
  bt->drop_graph();
  if (!bt->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&bt->capture_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(bt->capture_stream, hipStreamCaptureModeRelaxed));
  hipError_t e1 = launch_fill_int(bt->counters, ncnt, 0, bt->capture_stream);
  hipError_t e2 = launch_fill_int(bt->flags_dev, 2 + kXcdQueues, 0, bt->capture_stream);
  hipError_t e3 = launch_pipeline(pa, bt->lds, bt->capture_stream);
  hipGraph_t gr = nullptr;
  hipError_t e4 = hipStreamEndCapture(bt->capture_stream, &gr);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return fail(MGWR_ERR_HIP, "capturing the batched launch failed");
  }
  bt->graph = gr;
  HIP_TRY(hipGraphInstantiate(&bt->graph_exec, bt->graph, nullptr, nullptr, 0));
  bt->graph_stages = bt->stages;
  bt->graph_ncnt = ncnt;
  bt->graph_ntasks = ntasks;
  bt->graph_spin = bt->spin_limit;
  bt->graph_xq = use_xq;
  HIP_TRY(hipGraphLaunch(bt->graph_exec, bt->stream));
  return MGWR_OK;
}

int solve_pipelined(mgwr_batch* bt, const double* const* f, const double* const* g, double tol,
                    double* const* u, unsigned flags, mgwr_stats* stats, const std::vector<int>& sel) {
  const auto t_start = std::chrono::steady_clock::now();
  const int n = (int)bt->plans.size();
  int rc;
  const bool from_zero = !(flags & (MGWR_GUESS_IN_U | MGWR_WARM_START));
  std::vector<mgwr_stats> st(n);
  std::vector<const double*> b(n);
  std::vector<int> status(n), K(n), conv_at(n, -1), base(n, 0), judged(n, 0), zero_start(n, 0);
  std::vector<unsigned> fl_i(n, flags);
  for (int i : sel) {
    mgwr_plan* pl = bt->plans[i];
    if (!f[i] || !u[i]) return batch_fail(MGWR_ERR_INVALID_ARG, "null array in batch");
    if ((rc = use_device(pl))) return rc;
    if ((rc = prepare_solve(pl, f[i], g ? g[i] : nullptr, tol, u[i], fl_i[i], st[i], b[i], status[i]))) return rc;
    const int hint = st[i].used_warm_start ? (pl->khint_warm > 0 ? pl->khint_warm : pl->khint) : pl->khint;
    K[i] = hint > 0 ? hint : 8;
    zero_start[i] = !(fl_i[i] & MGWR_GUESS_IN_U);
  }
  // the plans' streams must be complete before the batch stream uses their arrays
  for (int i : sel) HIP_TRY(hipStreamSynchronize(bt->plans[i]->stream));
  while (true) {
    std::vector<int> act;
    for (int i : sel)
      if (status[i] == MGWR_ERR_NOT_CONVERGED &&
          st[i].cycles + (bt->plans[i]->mixed ? bt->plans[i]->hp.p.inner_cycles : 1) <= bt->plans[i]->hp.p.max_cycles)
        act.push_back(i);
    if (act.empty()) break;
    // per-instance stage lists, then interleaved by position
    std::vector<std::vector<Stage>> lists(act.size());
    std::vector<char> norms_every(act.size(), 1);
    size_t maxlen = 0;
    double flops = 0.0, bytes = 0.0;
    for (size_t a = 0; a < act.size(); ++a) {
      const int i = act[a];
      mgwr_plan* pl = bt->plans[i];
      const int per = pl->mixed ? pl->hp.p.inner_cycles : 1;  // cycles per outer step
      K[i] = std::max(1, std::min({K[i], mgwr_plan::kMaxPipeCycles / per, (pl->hp.p.max_cycles - st[i].cycles) / per}));
      // with a learned step count only the last step's defect is needed (float64
      // cycles); refinement steps need every defect as the next right-hand side
      const int hint = st[i].used_warm_start ? pl->khint_warm : pl->khint;
      const bool every = pl->mixed || !(hint > 0 && st[i].cycles == 0);
      norms_every[a] = every;
      build_plan_stages(pl, b[i], u[i], K[i], bt->norms + bt->norm_off[i], lists[a], every, zero_start[i] != 0);
      zero_start[i] = 0;
      pl->stages_f = nullptr;  // the plan's own uploaded table no longer matches its level-0 pointers
      maxlen = std::max(maxlen, lists[a].size());
      flops += pl->cycle_flops * K[i];
      bytes += pl->cycle_bytes * K[i];
    }
    bt->stages.clear();
    std::vector<std::vector<int>> gidx(act.size());
    for (size_t a = 0; a < act.size(); ++a) gidx[a].assign(lists[a].size(), -1);
    for (size_t pos = 0; pos < maxlen; ++pos)
      for (size_t a = 0; a < act.size(); ++a) {
        if (pos >= lists[a].size()) continue;
        Stage x = lists[a][pos];
        x.prev = x.prev >= 0 ? gidx[a][x.prev] : -1;
        x.round = (int)pos;
        gidx[a][pos] = (int)bt->stages.size();
        bt->stages.push_back(x);
      }
    assign_offsets(bt->stages);
    long long ncnt = 0;
    int ntasks = 0;
    for (auto& x : bt->stages) { ncnt += x.nleaf; ntasks = x.task0 + x.nchunks; }
    if ((size_t)bt->stages.size() * sizeof(Stage) > bt->off_counters - bt->off_stages)
      return batch_fail(MGWR_ERR_STATE, "internal error: batch stage table exceeds its workspace");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (bt->timing) {
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      HIP_TRY(hipEventRecord(e0, bt->stream));
    }
    if ((rc = launch_batch_table(bt, ncnt, ntasks))) return rc;
    if (bt->timing) HIP_TRY(hipEventRecord(e1, bt->stream));
    int fl[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(fl, bt->flags_dev, sizeof(fl), hipMemcpyDeviceToHost, bt->stream));
    std::vector<std::vector<double>> nh(act.size());
    for (size_t a = 0; a < act.size(); ++a) {
      const int i = act[a];
      nh[a].resize((size_t)(norms_every[a] ? K[i] : 1) * bt->plans[i]->norm_chunks);
      HIP_TRY(hipMemcpyAsync(nh[a].data(), bt->norms + bt->norm_off[i], nh[a].size() * sizeof(double),
                             hipMemcpyDeviceToHost, bt->stream));
    }
    HIP_TRY(hipStreamSynchronize(bt->stream));
    if (bt->timing) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      bt->tacc.launches[MGWR_K_PIPE64] += 1;
      bt->tacc.ms[MGWR_K_PIPE64] += ms;
      bt->tacc.flops[MGWR_K_PIPE64] += flops;
      bt->tacc.bytes[MGWR_K_PIPE64] += bytes;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    if (fl[1]) return batch_fail(MGWR_ERR_HIP, "pipelined cycles stalled (a progress wait exceeded its bound)");
    for (size_t a = 0; a < act.size(); ++a) {
      const int i = act[a];
      mgwr_plan* pl = bt->plans[i];
      mgwr_stats& s = st[i];
      const double target = tol * s.bnorm;
      const double first = s.cycles == 0 ? s.res0 : s.res;
      const int nn = norms_every[a] ? K[i] : 1;
      for (int c = 0; c < nn; ++c) {
        double m = 0.0;
        bool bad = false;
        for (int j = 0; j < pl->norm_chunks; ++j) {
          const double v = nh[a][(size_t)c * pl->norm_chunks + j];
          if (v != v) bad = true;
          else m = std::max(m, v);
        }
        const double r = bad ? std::nan("") : m;
        const int done_steps = pl->mixed ? s.refinements : s.cycles;
        const int cyc = norms_every[a] ? done_steps + c : done_steps + K[i] - 1;  // 0-based step of this norm
        if (cyc < 64) s.history[cyc] = r;
        if (conv_at[i] < 0 && r <= target) conv_at[i] = cyc + 1 - base[i];
        s.res = r;
      }
      if (pl->mixed) {
        s.refinements += K[i];
        s.cycles += K[i] * pl->hp.p.inner_cycles;
      } else {
        s.cycles += K[i];
      }
      if (!judged[i]) {
        judged[i] = 1;
        int frc;
        if (fall_back_to_zero(pl, b[i], u[i], s, s.cycles, tol, &frc)) {
          if (frc) return frc;
          HIP_TRY(hipStreamSynchronize(pl->stream));
          base[i] = pl->mixed ? s.refinements : s.cycles;
          conv_at[i] = -1;
          zero_start[i] = 1;
          K[i] = pl->khint > 0 ? pl->khint : 8;
          continue;
        }
      }
      if (!std::isfinite(s.res)) { status[i] = MGWR_ERR_NONFINITE; continue; }
      if (s.res <= target) { status[i] = MGWR_OK; continue; }
      const double rate = std::pow(std::max(s.res / first, 1e-300), 1.0 / K[i]);
      K[i] = (rate < 0.99 && rate > 0) ? (int)std::ceil(std::log(target / s.res) / std::log(rate)) : K[i];
    }
  }
  int ret = MGWR_OK;
  for (int i : sel)
    if ((rc = finish_solve(bt->plans[i], u[i], bt->stream))) return rc;
  HIP_TRY(hipStreamSynchronize(bt->stream));
  const double solve_ms = ms_since(t_start);
  for (int i : sel) {
    mgwr_stats& s = st[i];
    if (conv_at[i] > 0) (s.used_warm_start ? bt->plans[i]->khint_warm : bt->plans[i]->khint) = conv_at[i];
    s.avg_factor = (s.cycles > 0 && s.res0 > 0) ? std::pow(s.res / s.res0, 1.0 / s.cycles) : 0.0;
    s.solve_ms = solve_ms;
    if (from_zero && status[i] == MGWR_OK && s.cycles > 0) bt->plans[i]->rate_zero = s.avg_factor;
    if (stats) stats[i] = s;
    if (ret == MGWR_OK && status[i] != MGWR_OK) ret = status[i];
  }
  if (ret == MGWR_ERR_NOT_CONVERGED) return batch_fail(ret, "an instance reached max_cycles before the tolerance");
  if (ret == MGWR_ERR_NONFINITE) return batch_fail(ret, "an instance's residual norm is not finite");
  return MGWR_OK;
}

extern "C" {

void mgwr_params_default(mgwr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dim = 1;
  p->n = 63;
  p->length = 1.0;
  p->M = 128;
  p->T = 1.0;
  p->alpha = 0.5;
  p->r = 1.0;
  p->k = 10;
  p->leaf = 16;
  p->nu1 = 1;
  p->nu2 = 1;
  p->gamma = 1;
  p->max_cycles = 50;
  p->precision = MGWR_FP64;
  p->inner_cycles = 1;
  p->eta = 1.0;
  p->cluster = MGWR_CLUSTER_INDEX;
}

int mgwr_plan_create(const mgwr_params* p, const double* t_host, mgwr_plan** out) {
  if (!p || !out) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  mgwr_plan* pl = new (std::nothrow) mgwr_plan();
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "out of host memory");
  std::string e;
  try {
    e = build_host_plan(*p, t_host, pl->hp);
  } catch (const std::exception& ex) {
    e = std::string("host setup failed: ") + ex.what();
  }
  if (!e.empty()) {
    delete pl;
    return fail(MGWR_ERR_INVALID_ARG, e);
  }
  layout(pl);
  pl->create_ms = ms_since(t_start);
  *out = pl;
  return MGWR_OK;
}

int mgwr_plan_workspace_bytes(const mgwr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  *bytes = plan->off.total;
  return MGWR_OK;
}

}  // extern "C"

namespace mgwr {

// Points every device array of the plan into the workspace w (no device
// work); the per-binding caches (uploaded stage images) are reset.
void assign_pointers(mgwr_plan* pl, unsigned char* w, size_t bytes, hipStream_t stream) {
  pl->stream = stream;
  pl->ws = w;
  pl->ws_bytes = bytes;
  const HostPlan& hp = pl->hp;
  const auto& o = pl->off;
  pl->leaves = (LeafDesc*)(w + o.leaves);
  pl->dn_list = (int*)(w + o.dn_list);
  pl->ff_row = (int*)(w + o.ff_row);
  pl->zu_row = (int*)(w + o.zu_row);
  pl->a1 = (double*)(w + o.a1);
  pl->tpow = (double*)(w + o.tm);
  pl->part = (double*)(w + o.part);
  pl->scal = (double*)(w + o.scal);
  pl->B0 = (double*)(w + o.B0);
  pl->rows_dev = (int*)(w + o.wrows);
  pl->stages_dev = (Stage*)(w + o.stages);
  pl->counters = (int*)(w + o.counters);
  pl->flags_dev = (int*)(w + o.flags);
  pl->norms = (double*)(w + o.norms);
  pl->xq = (int*)(w + o.xq);
  pl->xq_cap = xq_capacity(hp);
  pl->xprobe = (int*)(w + o.xprobe);
  {
    const long long C = stages_per_cycle_bound(hp);
    pl->cstages_dev[0] = (Stage*)(w + o.cstages);
    pl->cstages_dev[1] = pl->cstages_dev[0] + C;
    pl->ccounters = (int*)(w + o.ccounters);
    pl->cflags = (int*)(w + o.cflags);
    for (int i = 0; i < 2; ++i) {
      pl->coarse_stages[i].clear();
      pl->coarse_up[i] = false;
    }
    pl->coarse_l = coarse_switch_level(hp);
  }
  pl->stages.clear();
  pl->stages_f = nullptr;
  pl->stages_u = nullptr;
  pl->d64.dense = (double*)(w + o.dense64);
  pl->d64.dinv = (double*)(w + o.dinv64);
  pl->d64.ffA = (double*)(w + o.ffA64);
  pl->d64.zuB = (double*)(w + o.zuB64);
  const int L = (int)hp.levels.size();
  pl->d64.U.assign(L, nullptr); pl->d64.F.assign(L, nullptr); pl->d64.R.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    if (l > 0) { pl->d64.U[l] = (double*)(w + o.U64[l]); pl->d64.F[l] = (double*)(w + o.F64[l]); }
    if (l + 1 < L || l == 0) pl->d64.R[l] = (double*)(w + o.R64[l]);
  }
  if (pl->mixed) {
    pl->d32.dense = (float*)(w + o.dense32);
    pl->d32.dinv = (float*)(w + o.dinv32);
    pl->d32.ffA = (float*)(w + o.ffA32);
    pl->d32.zuB = (float*)(w + o.zuB32);
    pl->d32.lr_bf16 = pl->bf16 ? 1 : 0;
    pl->d32.U.assign(L, nullptr); pl->d32.F.assign(L, nullptr); pl->d32.R.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
      pl->d32.U[l] = (float*)(w + o.U32[l]);
      pl->d32.F[l] = (float*)(w + o.F32[l]);
      if (l + 1 < L) pl->d32.R[l] = (float*)(w + o.R32[l]);
    }
  }
}

PlanBinding plan_binding(const mgwr_plan* pl) {
  return PlanBinding{pl->bound, pl->device, pl->ws, pl->ws_bytes, pl->stream, pl->net};
}

void restore_binding(mgwr_plan* pl, const PlanBinding& b) {
  if (b.bound) assign_pointers(pl, b.ws, b.bytes, b.stream);
  pl->bound = b.bound;
  pl->device = b.device;
  pl->net = b.net;
  if (!b.net) pl->nslices = 0;
}

void detach_network(mgwr_plan* pl) {
  pl->net = nullptr;
  pl->nslices = 0;
}

size_t plan_workspace_bytes(const mgwr_plan* pl) { return pl->off.total; }

}  // namespace mgwr

extern "C" {

int mgwr_plan_bind(mgwr_plan* pl, void* ws, size_t bytes, void* stream) {
  if (!pl || !ws) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  if (bytes < pl->off.total) return fail(MGWR_ERR_STATE, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return fail(MGWR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const auto t_start = std::chrono::steady_clock::now();
  HIP_TRY(hipGetDevice(&pl->device));
  assign_pointers(pl, (unsigned char*)ws, bytes, (hipStream_t)stream);
  const HostPlan& hp = pl->hp;
  const PackedPlan& pk = hp.pk;
  const auto& o = pl->off;
  unsigned char* w = pl->ws;
  // one packed host image, one copy
  std::vector<unsigned char> img(o.total > 0 ? std::min(o.total, o.B0) : 0);
  auto put = [&](size_t off, const void* src, size_t n) {
    if (n) std::memcpy(img.data() + off, src, n);
  };
  put(o.leaves, pk.leaves.data(), pk.leaves.size() * sizeof(LeafDesc));
  put(o.dn_list, pk.dn_list.data(), pk.dn_list.size() * sizeof(int));
  put(o.ff_row, pk.ff_row.data(), pk.ff_row.size() * sizeof(int));
  put(o.zu_row, pk.zu_row.data(), pk.zu_row.size() * sizeof(int));
  put(o.a1, pk.a1.data(), pk.a1.size() * sizeof(double));
  {
    std::vector<double> tp(hp.t.size());
    for (size_t m = 0; m < tp.size(); ++m) tp[m] = std::pow(hp.t[m], hp.p.alpha);
    put(o.tm, tp.data(), tp.size() * sizeof(double));
  }
  put(o.dense64, pk.dense.data(), pk.dense.size() * sizeof(double));
  put(o.dinv64, pk.dinv.data(), pk.dinv.size() * sizeof(double));
  put(o.ffA64, pk.ffA.data(), pk.ffA.size() * sizeof(double));
  put(o.zuB64, pk.zuB.data(), pk.zuB.size() * sizeof(double));
  HIP_TRY(hipMemcpyAsync(w, img.data(), img.size(), hipMemcpyHostToDevice, pl->stream));
  if (pl->mixed) {
    // float copies are rounded on the device from the float64 image
    HIP_TRY(launch_cast<double, float>(pl->d64.dense, pl->d32.dense, (long long)pk.dense.size(), pl->stream));
    HIP_TRY(launch_cast<double, float>(pl->d64.dinv, pl->d32.dinv, (long long)pk.dinv.size(), pl->stream));
    if (pl->bf16) {
      HIP_TRY(launch_cast_bf16(pl->d64.ffA, (unsigned short*)pl->d32.ffA, (long long)pk.ffA.size(), pl->stream));
      HIP_TRY(launch_cast_bf16(pl->d64.zuB, (unsigned short*)pl->d32.zuB, (long long)pk.zuB.size(), pl->stream));
    } else {
      HIP_TRY(launch_cast<double, float>(pl->d64.ffA, pl->d32.ffA, (long long)pk.ffA.size(), pl->stream));
      HIP_TRY(launch_cast<double, float>(pl->d64.zuB, pl->d32.zuB, (long long)pk.zuB.size(), pl->stream));
    }
  }
  // LDS of the marching kernel
  MarchArgs<double> a64 = base_args<double>(pl, pl->d64, 0);
  size_t lds = march_lds_bytes<double>(a64);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, pl->device));
  size_t cap = prop.sharedMemPerBlock;
  if (lds + 64 > cap) return fail(MGWR_ERR_STATE, "H-matrix accumulators need " + std::to_string(lds) +
                                                 " bytes of LDS, device allows " + std::to_string(cap));
  // The attribute is a per-kernel ceiling shared by every plan in the process:
  // raise it to the device limit once so no later bind can lower it below an
  // earlier plan's need; each launch still requests exactly its own size.
  HIP_TRY(set_march_lds_limit<double>(cap));
  HIP_TRY(set_march_lds_limit<float>(cap));
  HIP_TRY(set_pipeline_lds_limit(cap));
  {
    const int xrc = check_xcd_dispatch(pl->device, pl->xprobe, pl->stream);
    if (xrc) return xrc;
  }
  HIP_TRY(hipStreamSynchronize(pl->stream));
  pl->bound = true;
  pl->bind_ms = ms_since(t_start);
  return MGWR_OK;
}

int mgwr_residual(mgwr_plan* pl, const double* f, const double* g, const double* u, double* out, double* norm) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!f || !u) return fail(MGWR_ERR_INVALID_ARG, "null array");
  if ((rc = use_device(pl))) return rc;
  const HostPlan& hp = pl->hp;
  const long long MN = (long long)hp.p.M * hp.levels[0].N;
  const double* b = f;
  if (g) {
    HIP_TRY(launch_rhs0(f, g, pl->a1, pl->B0, hp.p.M, hp.levels[0].N, pl->stream));
    b = pl->B0;
  }
  double* dst = out ? out : pl->d64.R[0];
  if ((rc = defect<double>(pl, pl->d64, 0, b, const_cast<double*>(u), dst, false, nullptr, nullptr, true))) return rc;
  if (norm) return norm_inf<double>(pl, dst, MN, norm);
  return MGWR_OK;
}

int mgwr_solve(mgwr_plan* pl, const double* f, const double* g, double tol, double* u, unsigned flags,
               mgwr_stats* st) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!f || !u) return fail(MGWR_ERR_INVALID_ARG, "null array");
  if (!(tol > 0.0)) return fail(MGWR_ERR_INVALID_ARG, "tol must be > 0");
  if ((rc = use_device(pl))) return rc;
  const auto t_start = std::chrono::steady_clock::now();
  if (use_pipeline(pl)) {
    // the pipelined solve of a batch of one, on the plan's own regions
    mgwr_batch one;
    one.plans = {pl};
    one.bound = true;
    one.device = pl->device;
    one.stream = pl->stream;
    one.off_stages = pl->off.stages;
    one.off_counters = pl->off.counters;
    one.norm_off = {0};
    one.stages_dev = pl->stages_dev;
    one.counters = pl->counters;
    one.flags_dev = pl->flags_dev;
    one.xq = pl->xq;
    one.xq_cap = pl->xq_cap;
    one.norms = pl->norms;
    one.lds = march_lds_bytes<double>(base_args<double>(pl, pl->d64, 0));
    if (pl->mixed) one.lds = std::max(one.lds, march_lds_bytes<float>(base_args<float>(pl, pl->d32, 0)));
    one.timing = pl->timing;
    const double* fp[1] = {f};
    const double* gp[1] = {g};
    double* up[1] = {u};
    mgwr_stats s1{};
    int rc2 = solve_pipelined(&one, fp, gp, tol, up, flags, &s1, std::vector<int>{0});
    s1.solve_ms = ms_since(t_start);
    if (pl->timing)
      for (int c = 0; c < MGWR_K_CLASSES; ++c) {
        pl->tacc.launches[c] += one.tacc.launches[c];
        pl->tacc.ms[c] += one.tacc.ms[c];
        pl->tacc.flops[c] += one.tacc.flops[c];
        pl->tacc.bytes[c] += one.tacc.bytes[c];
      }
    if (st) *st = s1;
    return rc2;
  }
  apply_staging(pl);
  const HostPlan& hp = pl->hp;
  const int M = hp.p.M;
  const long long MN = (long long)M * hp.levels[0].N;
  const unsigned flags0 = flags;
  mgwr_stats s{};
  const double* b = f;
  int status = MGWR_ERR_NOT_CONVERGED;
  if ((rc = prepare_solve(pl, f, g, tol, u, flags, s, b, status))) return rc;
  if (!std::isfinite(s.bnorm)) {
    if ((rc = finish_solve(pl, u, pl->stream))) return rc;
    if (st) *st = s;
    return fail(MGWR_ERR_NONFINITE, "right-hand side is not finite");
  }
  const double target = tol * s.bnorm;
  if (pl->coarse_l > 0) HIP_TRY(launch_fill_int(pl->cflags + 1, 1, 0, pl->stream));

  if (status == MGWR_ERR_NOT_CONVERGED && !pl->mixed) {
    pl->d64.F[0] = const_cast<double*>(b);
    pl->d64.U[0] = u;
    // with a cycle count learned from the last solve from zero, the stopping
    // test (a float64 defect, its norm and a host read) is first evaluated
    // after that many cycles
    // (a predicted iterate is still judged after its first cycle)
    int skip_to = 0;
    if (!(flags & MGWR_GUESS_IN_U)) skip_to = pl->khint_staged;
    else if (s.used_warm_start) skip_to = pl->khint_staged_warm;
    const bool zt = zebra_stopping_test(pl);
    while (s.cycles < hp.p.max_cycles) {
      // whether this cycle is followed by a stopping test
      const bool tested = (s.used_warm_start && s.cycles == 0) || s.cycles + 1 >= skip_to;
      if ((rc = cycle<double>(pl, pl->d64, 0, zt && tested ? pl->d64.R[0] : nullptr))) return rc;
      s.cycles++;
      const bool judge = s.used_warm_start && s.cycles == 1;
      if (!judge && s.cycles < skip_to) continue;
      if (zt) {
        if ((rc = zebra_norm(pl, pl->d64.R[0], pl->norms, &s.res))) return rc;
      } else if ((rc = defect_norm(pl, b, u, pl->norms, &s.res))) {
        return rc;
      }
      if (s.cycles <= 64) s.history[s.cycles - 1] = s.res;
      if (s.cycles == 1 && fall_back_to_zero(pl, b, u, s, 1, tol, &rc)) {
        if (rc) return rc;
        skip_to = 0;
        continue;
      }
      if (!std::isfinite(s.res)) { status = MGWR_ERR_NONFINITE; break; }
      if (s.res <= target) { status = MGWR_OK; break; }
    }
    if (status == MGWR_OK && !(flags & MGWR_GUESS_IN_U)) pl->khint_staged = s.cycles;
    if (status == MGWR_OK && s.used_warm_start) pl->khint_staged_warm = s.cycles;
  } else if (status == MGWR_ERR_NOT_CONVERGED) {
    // float64 outer residual and correction; float32 inner cycles on A e = r
    if (!(flags & MGWR_GUESS_IN_U)) {
      // zero iterate: the first defect is b itself
      HIP_TRY(launch_cast<double, float>(b, pl->d32.F[0], MN, pl->stream));
    } else {
      HIP_TRY(launch_cast<double, float>(pl->d64.R[0], pl->d32.F[0], MN, pl->stream));
    }
    while (s.cycles < hp.p.max_cycles) {
      HIP_TRY(launch_fill<float>(pl->d32.U[0], MN, 0.0f, pl->stream));
      for (int ic = 0; ic < hp.p.inner_cycles && s.cycles < hp.p.max_cycles; ++ic) {
        if ((rc = cycle<float>(pl, pl->d32, 0))) return rc;
        s.cycles++;
      }
      HIP_TRY(launch_add_correction(u, pl->d32.U[0], MN, pl->stream));
      s.refinements++;
      // the defect is the next float32 right-hand side; its norm from the
      // chains' partial maxima
      if ((rc = defect_rhs32(pl, b, u, pl->d32.F[0], pl->norms))) return rc;
      HIP_TRY(launch_maxabs_parts(pl->norms, (int)((hp.levels[0].N + 15) / 16), pl->scal, pl->stream));
      if ((rc = read_scalar(pl, &s.res))) return rc;
      if (s.refinements <= 64) s.history[s.refinements - 1] = s.res;
      if (s.refinements == 1 && fall_back_to_zero(pl, b, u, s, s.cycles, tol, &rc)) {
        if (rc) return rc;
        HIP_TRY(launch_cast<double, float>(b, pl->d32.F[0], MN, pl->stream));
        continue;
      }
      if (!std::isfinite(s.res)) { status = MGWR_ERR_NONFINITE; break; }
      if (s.res <= target) { status = MGWR_OK; break; }
    }
  }
  if (pl->coarse_l > 0 && s.cycles > 0) {
    int stalled = 0;
    HIP_TRY(hipMemcpyAsync(&stalled, pl->cflags + 1, sizeof(int), hipMemcpyDeviceToHost, pl->stream));
    HIP_TRY(hipStreamSynchronize(pl->stream));
    if (stalled) return fail(MGWR_ERR_HIP, "pipelined coarse cycles stalled (a progress wait exceeded its bound)");
  }
  s.avg_factor = (s.cycles > 0 && s.res0 > 0) ? std::pow(s.res / s.res0, 1.0 / s.cycles) : 0.0;
  if (status == MGWR_OK && s.cycles > 0 && !(flags0 & (MGWR_GUESS_IN_U | MGWR_WARM_START)))
    pl->rate_zero = s.avg_factor;
  if ((rc = finish_solve(pl, u, pl->stream))) return rc;
  s.solve_ms = ms_since(t_start);
  if (st) *st = s;
  if (status == MGWR_ERR_NOT_CONVERGED) return fail(status, "max_cycles reached before the tolerance");
  if (status == MGWR_ERR_NONFINITE) return fail(status, "residual norm is not finite");
  return MGWR_OK;
}

int mgwr_hmatvec(mgwr_plan* pl, const double* x, double* y, int ncols) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!x || !y || ncols < 0) return fail(MGWR_ERR_INVALID_ARG, "bad argument");
  if ((rc = use_device(pl))) return rc;
  MarchArgs<double> a = base_args<double>(pl, pl->d64, 0);
  a.F = nullptr; a.U = const_cast<double*>(x); a.Out = y;
  a.ld = ncols; a.ncols = ncols; a.cstride = 1; a.coff = 0; a.dim = 0; a.n = 0; a.inv_h2 = 0.0; a.split = 0;
  HIP_TRY(launch_march<double>(MODE_MATVEC, a, pl->stream));
  return MGWR_OK;
}

int mgwr_apply_A(mgwr_plan* pl, const double* u, double* out) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!u || !out) return fail(MGWR_ERR_INVALID_ARG, "null array");
  if ((rc = use_device(pl))) return rc;
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[0];
  const long long MN = (long long)hp.p.M * lv.N;
  if (u < out + MN && out < u + MN) return fail(MGWR_ERR_INVALID_ARG, "u and out must not overlap");
  // the product march with the stencil: out = R~ u + A_h u
  MarchArgs<double> a = base_args<double>(pl, pl->d64, 0);
  a.F = nullptr; a.U = const_cast<double*>(u); a.Out = out;
  a.ld = lv.N; a.ncols = lv.N; a.cstride = 1; a.coff = 0; a.split = 0;   // the caller's natural order
  a.dim = hp.p.dim; a.n = lv.n; a.inv_h2 = 1.0 / (lv.h * lv.h);
  HIP_TRY(launch_march<double>(MODE_MATVEC, a, pl->stream));
  return MGWR_OK;
}

int mgwr_htrsm(mgwr_plan* pl, int level, const double* b, double* x, int ncols) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!b || !x || ncols < 0 || level < 0 || level >= (int)pl->hp.levels.size())
    return fail(MGWR_ERR_INVALID_ARG, "bad argument");
  if ((rc = use_device(pl))) return rc;
  MarchArgs<double> a = base_args<double>(pl, pl->d64, level);
  a.F = b; a.U = x; a.Out = nullptr;
  a.ld = ncols; a.ncols = ncols; a.cstride = 1; a.coff = 0; a.dim = 0; a.n = 0; a.inv_h2 = 0.0; a.split = 0;
  HIP_TRY(launch_march<double>(MODE_TRSM, a, pl->stream));
  return MGWR_OK;
}

int mgwr_timing_enable(mgwr_plan* pl, int enable) {
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "null plan");
  if (!pl->pending.empty()) {
    if (pl->bound) HIP_TRY(hipStreamSynchronize(pl->stream));
    drain_timing(pl);
  }
  pl->timing = enable != 0;
  if (enable) pl->tacc = mgwr_timing{};
  return MGWR_OK;
}

int mgwr_timing_get(mgwr_plan* pl, mgwr_timing* out) {
  if (!pl || !out) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  if (pl->bound) HIP_TRY(hipStreamSynchronize(pl->stream));
  drain_timing(pl);
  *out = pl->tacc;
  return MGWR_OK;
}

int mgwr_plan_set_warm_start(mgwr_plan* pl, mgwr_net* net, int nslices, const int* rows) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!net) {
    pl->net = nullptr;
    pl->nslices = 0;
    return MGWR_OK;
  }
  const HostPlan& hp = pl->hp;
  if (nslices < 1 || nslices > mgwr_plan::kMaxSlices || !rows)
    return fail(MGWR_ERR_INVALID_ARG, "nslices must lie in [1, 64] with a row list");
  if (net_signal_channels(net) != nslices || net_input_channels(net) != nslices + 2 || net_out_channels(net) != nslices)
    return fail(MGWR_ERR_INVALID_ARG, "the network must take nslices signal + 2 extra channels and give nslices");
  const int n0 = hp.levels[0].n;
  if (((n0 + 1) & n0) != 0 || n0 < 3)
    return fail(MGWR_ERR_INVALID_ARG, "a warm start needs n = 2^p - 1 points per side");
  if (net_capacity(net) < hp.levels[0].N) return fail(MGWR_ERR_STATE, "the network must be bound for >= N points");
  for (int i = 0; i < nslices; ++i)
    if (rows[i] < 0 || rows[i] >= hp.p.M || (i > 0 && rows[i] <= rows[i - 1]))
      return fail(MGWR_ERR_INVALID_ARG, "slice rows must increase within [0, M)");
  std::vector<int> rv(rows, rows + nslices);
  HIP_TRY(hipMemcpyAsync(pl->rows_dev, rv.data(), nslices * sizeof(int), hipMemcpyHostToDevice, pl->stream));
  HIP_TRY(hipStreamSynchronize(pl->stream));
  pl->net = net;
  pl->nslices = nslices;
  return MGWR_OK;
}

}  // extern "C"

namespace {

// 64-bit FNV-1a of a byte range (the weight blob's checksum).
unsigned long long fnv1a64(const unsigned char* p, size_t n) {
  unsigned long long h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

// Parses and checks a weight blob (layout in mgwr.h); on success *params
// points at its nparam float32 weights inside the blob.
int parse_model(const void* blob, size_t bytes, mgwr_model_info* info, const float** params) {
  if (!blob || bytes == 0) return fail(MGWR_ERR_MODEL, "no learned weights (empty blob)");
  const unsigned char* p = static_cast<const unsigned char*>(blob);
  size_t off = 0;
  auto take = [&](void* dst, size_t n) -> bool {
    if (off + n > bytes) return false;
    std::memcpy(dst, p + off, n);
    off += n;
    return true;
  };
  char magic[8];
  int version = 0;
  mgwr_model_info mi{};
  if (!take(magic, 8) || std::memcmp(magic, "MGWRNET1", 8) != 0)
    return fail(MGWR_ERR_MODEL, "weight blob: bad magic");
  if (!take(&version, 4) || version != 1) return fail(MGWR_ERR_MODEL, "weight blob: unsupported version");
  if (!take(&mi.layers, 4) || mi.layers < 1 || mi.layers > 16)
    return fail(MGWR_ERR_MODEL, "weight blob: layer count outside [1, 16]");
  for (int l = 0; l <= mi.layers; ++l)
    if (!take(&mi.channels[l], 4) || mi.channels[l] < 1 || mi.channels[l] > 1024)
      return fail(MGWR_ERR_MODEL, "weight blob: channel count outside [1, 1024]");
  if (!take(&mi.nsignal, 4) || mi.nsignal < 1 || mi.nsignal > mi.channels[0] - 1)
    return fail(MGWR_ERR_MODEL, "weight blob: bad signal channel count");
  if (!take(&mi.nslices, 4) || mi.nslices < 1 || mi.nslices > 64)
    return fail(MGWR_ERR_MODEL, "weight blob: slice count outside [1, 64]");
  for (int i = 0; i < mi.nslices; ++i)
    if (!take(&mi.rows[i], 4) || mi.rows[i] < 0 || (i > 0 && mi.rows[i] <= mi.rows[i - 1]))
      return fail(MGWR_ERR_MODEL, "weight blob: slice rows must increase from 0");
  if (!take(&mi.h_min, 8) || !(mi.h_min >= 0.0) || !std::isfinite(mi.h_min))
    return fail(MGWR_ERR_MODEL, "weight blob: bad h_min");
  long long expect = 0;
  for (int l = 0; l < mi.layers; ++l) expect += (long long)mi.channels[l + 1] * mi.channels[l] * 9 + mi.channels[l + 1];
  if (!take(&mi.nparam, 8) || mi.nparam != expect)
    return fail(MGWR_ERR_MODEL, "weight blob: parameter count does not match the layer shapes");
  const size_t pbytes = (size_t)mi.nparam * sizeof(float);
  const size_t poff = off;
  if (off + pbytes + 8 != bytes) return fail(MGWR_ERR_MODEL, "weight blob: wrong size");
  off += pbytes;
  unsigned long long sum = 0;
  std::memcpy(&sum, p + off, 8);
  if (sum != fnv1a64(p, off)) return fail(MGWR_ERR_MODEL, "weight blob: checksum mismatch");
  for (long long i = 0; i < mi.nparam; ++i) {
    float v;
    std::memcpy(&v, p + poff + (size_t)i * 4, 4);
    if (!std::isfinite(v)) return fail(MGWR_ERR_MODEL, "weight blob: non-finite weight");
  }
  if (info) *info = mi;
  if (params) *params = reinterpret_cast<const float*>(p + poff);
  return MGWR_OK;
}

}  // namespace

extern "C" {

int mgwr_model_describe(const void* blob, size_t bytes, mgwr_model_info* info) {
  return parse_model(blob, bytes, info, nullptr);
}

int mgwr_model_load(mgwr_plan* pl, mgwr_net* net, const void* blob, size_t bytes) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!net) return fail(MGWR_ERR_INVALID_ARG, "null network");
  if (!net_is_bound(net)) return fail(MGWR_ERR_STATE, "network is not bound");
  mgwr_model_info mi{};
  const float* w = nullptr;
  if ((rc = parse_model(blob, bytes, &mi, &w))) return rc;
  if (!net_same_shape(net, mi.layers, mi.channels, mi.nsignal) || (size_t)mi.nparam != net_param_count(net))
    return fail(MGWR_ERR_MODEL, "weight blob: network shape differs from the bound network's");
  for (int i = 0; i < mi.nslices; ++i)
    if (mi.rows[i] >= pl->hp.p.M) return fail(MGWR_ERR_MODEL, "weight blob: slice row beyond the plan's mesh");
  if (mi.nsignal != mi.nslices || mi.channels[0] - 1 != mi.nslices + 2 || mi.channels[mi.layers] != mi.nslices)
    return fail(MGWR_ERR_MODEL, "weight blob: the network must map nslices slices plus 2 extra channels to nslices");
  // attach first (it checks the plan's grid and the net's capacity), then copy
  if ((rc = mgwr_plan_set_warm_start(pl, net, mi.nslices, mi.rows))) return rc;
  std::vector<float> host((size_t)mi.nparam);   // the blob's weights may be unaligned
  std::memcpy(host.data(), w, host.size() * sizeof(float));
  HIP_TRY(hipMemcpyAsync(net_params(net), host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice,
                         net_stream(net)));
  HIP_TRY(hipStreamSynchronize(net_stream(net)));
  if ((rc = mgwr_net_sync_weights(net))) return rc;
  if ((rc = mgwr_net_set_finest(net, mi.h_min))) return rc;
  HIP_TRY(hipStreamSynchronize(net_stream(net)));
  return MGWR_OK;
}

int mgwr_plan_get_info(const mgwr_plan* pl, mgwr_plan_info* info) {
  if (!pl || !info) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  const HostPlan& hp = pl->hp;
  info->M = hp.p.M;
  info->nleaf = (int)hp.pk.leaves.size();
  info->nclusters = (int)hp.clusters.size();
  info->ndense = (int)hp.dense_blocks.size();
  info->nrk = (int)hp.rk_blocks.size();
  info->nzclusters = hp.nzclusters;
  info->nslots = hp.nslots;
  info->window = hp.window;
  info->levels = (int)hp.levels.size();
  info->k = hp.p.k;
  info->stored_entries = hp.stored;
  info->shift0 = hp.levels[0].shift;
  info->layout = split_choice(pl) ? MGWR_LAYOUT_SPLIT : MGWR_LAYOUT_NATURAL;
  info->nf64leaves = 0;
  for (const LeafDesc& d : hp.pk.leaves) info->nf64leaves += d.f64solve;
  return MGWR_OK;
}

int mgwr_plan_get_mesh(const mgwr_plan* pl, double* t, double* a1) {
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "null plan");
  if (t) std::memcpy(t, pl->hp.t.data(), pl->hp.t.size() * sizeof(double));
  if (a1) std::memcpy(a1, pl->hp.pk.a1.data(), pl->hp.pk.a1.size() * sizeof(double));
  return MGWR_OK;
}

int mgwr_plan_export_dense(const mgwr_plan* pl, double* Rt) {
  if (!pl || !Rt) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  export_dense(pl->hp, Rt);
  return MGWR_OK;
}

int mgwr_plan_set_progress_limit(mgwr_plan* pl, unsigned polls) {
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "null plan");
  pl->spin_limit = polls;
  return MGWR_OK;
}

int mgwr_plan_destroy(mgwr_plan* pl) {
  if (!pl) return MGWR_OK;
  if (pl->bound && !pl->pending.empty()) {
    (void)hipStreamSynchronize(pl->stream);
    drain_timing(pl);
  }
  for (hipEvent_t e : pl->event_pool) (void)hipEventDestroy(e);
  delete pl;
  return MGWR_OK;
}

const char* mgwr_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

extern "C" {

int mgwr_batch_create(int count, mgwr_plan* const* plans, mgwr_batch** out) {
  if (!out || count < 1 || !plans) return batch_fail(MGWR_ERR_INVALID_ARG, "bad batch arguments");
  *out = nullptr;
  mgwr_batch* bt = new (std::nothrow) mgwr_batch();
  if (!bt) return batch_fail(MGWR_ERR_INVALID_ARG, "out of host memory");
  Carver cv;
  long long nst = 0, ncnt = 0, nnorm = 0;
  for (int i = 0; i < count; ++i) {
    mgwr_plan* pl = plans[i];
    if (!pl || !pl->bound) { delete bt; return batch_fail(MGWR_ERR_STATE, "every plan of a batch must be bound"); }
    if (i > 0 && pl->device != plans[0]->device) { delete bt; return batch_fail(MGWR_ERR_INVALID_ARG, "plans on different devices"); }
    const long long spc = stages_per_cycle_bound(pl->hp) * mgwr_plan::kMaxPipeCycles;
    nst += spc;
    ncnt += spc * (long long)pl->hp.pk.leaves.size();
    bt->norm_off.push_back((size_t)nnorm);
    nnorm += (long long)mgwr_plan::kMaxPipeCycles * ((pl->hp.levels[0].N + 15) / 16);
    bt->plans.push_back(pl);
    bt->lds = std::max(bt->lds, march_lds_bytes<double>(base_args<double>(pl, pl->d64, 0)));
    if (pl->mixed) bt->lds = std::max(bt->lds, march_lds_bytes<float>(base_args<float>(pl, pl->d32, 0)));
  }
  long long nxq = 0;
  for (int i = 0; i < count; ++i) nxq += xq_capacity(plans[i]->hp);
  bt->off_stages = cv.take((size_t)nst * sizeof(Stage));
  bt->off_counters = cv.take((size_t)ncnt * sizeof(int));
  bt->off_flags = cv.take((2 + kXcdQueues) * sizeof(int));
  bt->off_norms = cv.take((size_t)nnorm * sizeof(double));
  bt->off_xq = cv.take((size_t)nxq * sizeof(int));
  bt->xq_cap = nxq;
  bt->total = cv.off;
  *out = bt;
  return MGWR_OK;
}

int mgwr_batch_workspace_bytes(const mgwr_batch* bt, size_t* bytes) {
  if (!bt || !bytes) return batch_fail(MGWR_ERR_INVALID_ARG, "null argument");
  *bytes = bt->total;
  return MGWR_OK;
}

int mgwr_batch_bind(mgwr_batch* bt, void* ws, size_t bytes, void* stream) {
  if (!bt || !ws) return batch_fail(MGWR_ERR_INVALID_ARG, "null argument");
  if (bytes < bt->total) return batch_fail(MGWR_ERR_STATE, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return batch_fail(MGWR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  HIP_TRY(hipGetDevice(&bt->device));
  if (bt->device != bt->plans[0]->device) return batch_fail(MGWR_ERR_INVALID_ARG, "batch bound to another device");
  unsigned char* w = (unsigned char*)ws;
  bt->stream = (hipStream_t)stream;
  bt->stages_dev = (Stage*)(w + bt->off_stages);
  bt->counters = (int*)(w + bt->off_counters);
  bt->flags_dev = (int*)(w + bt->off_flags);
  bt->norms = (double*)(w + bt->off_norms);
  bt->xq = (int*)(w + bt->off_xq);
  bt->bound = true;
  return MGWR_OK;
}

}  // extern "C"

namespace {

// Staged instances of a batch are solved by up to kStagedWorkers host
// threads, each with a stream of its own: a staged solve waits on the host
// for its stopping tests, and its coarse levels run as latency-bound launches
// that leave most of the GPU idle, so solving several side by side fills it.
// Not done when two entries share a plan (one workspace).  Warm-started
// instances run side by side too: their predictions take turns on the
// network they share (net_mutex), their cycles overlap.  Measured on 64
// uneven 2D instances: one by one 9.6e8 unknowns/s; 2-4 workers 1.15e9, 8
// workers 1.22e9, 12 or 16 no faster.
constexpr int kStagedWorkers = 8;

bool staged_side_by_side(const mgwr_batch* bt, const std::vector<int>& staged, unsigned flags) {
  (void)flags;   // warm starts too: each prediction holds its network's lock
  if (staged.size() < 2) return false;
  std::set<const mgwr_plan*> seen;
  for (int i : staged)
    if (!seen.insert(bt->plans[i]).second) return false;
  return true;
}

// rcs / msgs: status and error text of each staged entry, in the order of
// `staged`.  The return value reports a failure of the set-up itself.
int solve_staged_side_by_side(mgwr_batch* bt, const std::vector<int>& staged, const double* const* f,
                              const double* const* g, double tol, double* const* u, unsigned flags,
                              mgwr_stats* stats, std::vector<int>& rcs, std::vector<std::string>& msgs) {
  const int nw = std::min<int>(kStagedWorkers, (int)staged.size());
  const bool full = (int)staged.size() >= kStagedWorkers;   // every worker busy: coarse launches one level lower
  while ((int)bt->worker_streams.size() < nw) {
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    bt->worker_streams.push_back(s);
  }
  // work already queued on the plans' own streams (their inputs, earlier
  // solves) completes before another stream touches their arrays
  for (int i : staged) HIP_TRY(hipStreamSynchronize(bt->plans[i]->stream));
  // Per-launch event timing stays on the calling thread: a plan's events and
  // its pending list are not touched by the workers (timing is suspended for
  // the phase and restored after it; the batch times the phase as a whole).
  std::vector<char> timed(staged.size(), 0);
  for (size_t j = 0; j < staged.size(); ++j) {
    mgwr_plan* pl = bt->plans[staged[j]];
    if (!pl->pending.empty()) drain_timing(pl);
    timed[j] = pl->timing ? 1 : 0;
    pl->timing = false;
  }
  const auto t_start = std::chrono::steady_clock::now();
  rcs.assign(staged.size(), MGWR_OK);
  msgs.assign(staged.size(), std::string());
  std::vector<mgwr_stats> sts(staged.size());
  std::atomic<int> next(0);
  auto work = [&](int w) {
    const hipError_t e = hipSetDevice(bt->device);
    for (int j = next.fetch_add(1); j < (int)staged.size(); j = next.fetch_add(1)) {
      const int i = staged[j];
      if (e != hipSuccess) {
        rcs[j] = MGWR_ERR_HIP;
        msgs[j] = std::string("hipSetDevice: ") + hipGetErrorString(e);
        continue;
      }
      mgwr_plan* pl = bt->plans[i];
      hipStream_t own = pl->stream;
      pl->stream = bt->worker_streams[w];
      pl->side_by_side = full;
      mgwr_stats si{};
      int rc = mgwr_solve(pl, f[i], g ? g[i] : nullptr, tol, u[i], flags, &si);
      if (rc != MGWR_OK) msgs[j] = mgwr_last_error();
      const hipError_t se = hipStreamSynchronize(pl->stream);   // all of it done before the plan's stream returns
      pl->stream = own;
      pl->side_by_side = false;
      if (rc == MGWR_OK && se != hipSuccess) {
        rc = MGWR_ERR_HIP;
        msgs[j] = std::string("hipStreamSynchronize: ") + hipGetErrorString(se);
      }
      rcs[j] = rc;
      sts[j] = si;
    }
  };
  std::vector<std::thread> threads;
  try {
    for (int w = 1; w < nw; ++w) threads.emplace_back(work, w);
  } catch (...) {
    // fewer threads: the remaining entries are taken by those that started
  }
  work(0);
  for (std::thread& t : threads) t.join();
  const double wall_ms = ms_since(t_start);
  double flops = 0.0, bytes = 0.0;
  for (size_t j = 0; j < staged.size(); ++j) {
    mgwr_plan* pl = bt->plans[staged[j]];
    pl->timing = timed[j] != 0;
    if (stats) stats[staged[j]] = sts[j];
    if (bt->timing) {
      // one cycle's stages plus one float64 defect of the full system; with
      // zebra defects the defect marches above the pipelined coarse levels
      // and the stopping-test march are not run
      // (the stage list of a cycle with defect stages, as the coarse launch
      // runs them; the staged levels' are dropped below with zebra defects)
      const bool zd = zebra_defects(pl), zt = !pl->mixed && zebra_stopping_test(pl);
      std::vector<Stage> one;
      const bool zebra = pl->zebra;
      pl->zebra = false;
      append_cycle_stages(pl, 0, -1, one, pl->mixed);
      pl->zebra = zebra;
      const int ncoarse = pl->coarse_l > 0 ? pl->hp.levels[pl->coarse_l].n : 0;
      double cf = zt ? 0.0 : 2.0 * pl->hp.stored * pl->hp.levels[0].N;
      double cb = (zt ? 2.5 : 3.0) * pl->hp.p.M * pl->hp.levels[0].N * 8.0;
      for (const Stage& x : one) {
        const bool resid = x.kind == STG_RESID || x.kind == STG_RESID32;
        const int nlev = x.kind == STG_RESID32 ? x.mf.n : x.m.n;
        if (zd && resid && nlev > ncoarse) continue;
        stage_work(pl, x, cf, cb);
      }
      flops += cf * sts[j].cycles;
      bytes += cb * sts[j].cycles;
    }
  }
  if (bt->timing) {
    bt->tacc.launches[MGWR_K_SIDE] += 1;
    bt->tacc.ms[MGWR_K_SIDE] += wall_ms;
    bt->tacc.flops[MGWR_K_SIDE] += flops;
    bt->tacc.bytes[MGWR_K_SIDE] += bytes;
  }
  return MGWR_OK;
}

}  // namespace

extern "C" {

int mgwr_batch_solve(mgwr_batch* bt, const double* const* f, const double* const* g, double tol, double* const* u,
                     unsigned flags, mgwr_stats* stats) {
  if (!bt || !bt->bound) return batch_fail(MGWR_ERR_STATE, "batch is not bound");
  if (!f || !u || !(tol > 0.0)) return batch_fail(MGWR_ERR_INVALID_ARG, "bad arguments");
  // instances whose schedule is pipelined share one launch; the others are
  // solved with their staged schedule, side by side where that is safe
  std::vector<int> pipe, staged;
  for (int i = 0; i < (int)bt->plans.size(); ++i) (use_pipeline(bt->plans[i]) ? pipe : staged).push_back(i);
  int ret = MGWR_OK;
  std::string msg;
  if (!pipe.empty()) {
    ret = solve_pipelined(bt, f, g, tol, u, flags, stats, pipe);
    if (ret) msg = mgwr_last_error();
    if (ret != MGWR_OK && ret != MGWR_ERR_NOT_CONVERGED && ret != MGWR_ERR_NONFINITE) return ret;
  }
  if (staged_side_by_side(bt, staged, flags)) {
    std::vector<int> rcs;
    std::vector<std::string> msgs;
    const int rc = solve_staged_side_by_side(bt, staged, f, g, tol, u, flags, stats, rcs, msgs);
    if (rc) return rc;
    for (size_t j = 0; j < staged.size(); ++j) {   // reported as the one-by-one loop below would
      if (rcs[j] != MGWR_OK && rcs[j] != MGWR_ERR_NOT_CONVERGED && rcs[j] != MGWR_ERR_NONFINITE)
        return batch_fail(rcs[j], msgs[j]);
      if (rcs[j] != MGWR_OK && ret == MGWR_OK) {
        ret = rcs[j];
        msg = msgs[j];
      }
    }
  } else {
    for (int i : staged) {
      mgwr_stats si{};
      const int rc = mgwr_solve(bt->plans[i], f[i], g ? g[i] : nullptr, tol, u[i], flags, &si);
      if (stats) stats[i] = si;
      if (rc != MGWR_OK && rc != MGWR_ERR_NOT_CONVERGED && rc != MGWR_ERR_NONFINITE) return rc;
      if (rc != MGWR_OK && ret == MGWR_OK) {
        ret = rc;
        msg = mgwr_last_error();
      }
    }
  }
  if (ret != MGWR_OK) return batch_fail(ret, msg);
  return MGWR_OK;
}

int mgwr_set_xcd_queues(int enable, int* previous) {
  const int old = g_xcd_queues.exchange(enable ? 1 : 0);
  if (previous) *previous = old;
  return MGWR_OK;
}

int mgwr_xcd_queues_in_use(const mgwr_plan* pl, int* in_use) {
  if (!pl || !in_use) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  if (!pl->bound) return fail(MGWR_ERR_STATE, "plan is not bound to a workspace");
  *in_use = g_xcd_queues.load() != 0 && xcd_dispatch_ok(pl->device) ? 1 : 0;
  return MGWR_OK;
}

int mgwr_batch_set_graph(mgwr_batch* bt, int enable) {
  if (!bt) return batch_fail(MGWR_ERR_INVALID_ARG, "null batch");
  bt->use_graph = enable != 0;
  if (!bt->use_graph) bt->drop_graph();
  return MGWR_OK;
}

int mgwr_batch_graph_replays(const mgwr_batch* bt, long long* replays) {
  if (!bt || !replays) return batch_fail(MGWR_ERR_INVALID_ARG, "null argument");
  *replays = bt->graph_replays;
  return MGWR_OK;
}

int mgwr_plan_autotune(mgwr_plan* pl, const double* f, const double* g, double tol, double* u, int* chosen) {
  int rc = check_bound(pl);
  if (rc) return rc;
  if (!f || !u || !(tol > 0.0)) return fail(MGWR_ERR_INVALID_ARG, "bad arguments");
  // candidates: the pipelined schedule, and the staged one with either march
  // prefetch and the coarse launch from the rule's level or one level either
  // side of it
  struct Cand { int sched, prefetch, coarse, layout; };
  const int lay0 = pl->hp.p.dim == 2 ? MGWR_LAYOUT_SPLIT : MGWR_LAYOUT_NATURAL;
  std::vector<Cand> cands = {{MGWR_SCHED_PIPELINED, 0, -1, lay0}};
  const int L = (int)pl->hp.levels.size();
  const int c0 = coarse_switch_level(pl->hp);
  std::vector<int> levels;
  if (c0 == 0) levels = {0};
  for (int c = c0 - 1; c0 > 0 && c <= c0 + 1; ++c)
    if (c >= 1 && c < L) levels.push_back(c);
  for (int pf : {1, 2})
    for (int c : levels) cands.push_back({MGWR_SCHED_STAGED, pf, c, lay0});
  const int saved = pl->tuned;
  const bool saved_set = pl->staging_set;
  const int saved_pf = pl->set_prefetch, saved_c = pl->set_coarse, saved_lay = pl->set_layout;
  const int keep = pl->hp.p.schedule;
  double best = 1e300;
  Cand pick = cands[0];
  // the last round times the best candidate in the other storage (2D)
  const size_t nbase = cands.size();
  for (size_t ci = 0; ci <= nbase; ++ci) {
    if (ci == nbase) {
      if (pl->hp.p.dim != 2) break;
      cands.push_back(pick);
      cands.back().layout = pick.layout == MGWR_LAYOUT_SPLIT ? MGWR_LAYOUT_NATURAL : MGWR_LAYOUT_SPLIT;
    }
    const Cand cd = cands[ci];
    pl->tuned = cd.sched;
    pl->staging_set = true;
    pl->set_prefetch = cd.prefetch;
    pl->set_coarse = cd.coarse;
    pl->set_layout = cd.layout;
    pl->hp.p.schedule = MGWR_SCHED_AUTO;
    double secs = 0.0;
    // the second solve runs with what the first one learned (cycle count)
    for (int rep = 0; rep < 2 && !rc; ++rep) {
      auto t0 = std::chrono::steady_clock::now();
      rc = mgwr_solve(pl, f, g, tol, u, 0u, nullptr);
      if (rc == MGWR_OK) {
        if (hipStreamSynchronize(pl->stream) != hipSuccess) rc = fail(MGWR_ERR_HIP, "synchronise failed");
        secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      }
    }
    pl->hp.p.schedule = keep;
    if (rc) {
      pl->tuned = saved;
      pl->staging_set = saved_set;
      pl->set_prefetch = saved_pf;
      pl->set_coarse = saved_c;
      pl->set_layout = saved_lay;
      return rc;
    }
    if (secs < best) {
      best = secs;
      pick = cd;
    }
  }
  // the plan keeps the choice as set knobs; later AUTO plans of the shape find it in the table
  pl->tuned = pick.sched;
  pl->staging_set = pick.sched == MGWR_SCHED_STAGED;
  pl->set_prefetch = pick.sched == MGWR_SCHED_STAGED ? pick.prefetch : 0;
  pl->set_coarse = pick.sched == MGWR_SCHED_STAGED ? pick.coarse : -1;
  pl->set_layout = pl->hp.p.dim == 2 ? pick.layout : MGWR_LAYOUT_AUTO;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneChoice& tc = g_tuned[tune_key(pl)];
    tc.sched = pick.sched;
    tc.prefetch = pick.prefetch;
    tc.coarse = pick.coarse;
    tc.layout = pl->hp.p.dim == 2 ? pick.layout : MGWR_LAYOUT_AUTO;
  }
  if (chosen) *chosen = pick.sched;
  return MGWR_OK;
}

int mgwr_plan_set_staging(mgwr_plan* pl, int prefetch, int coarse_level) {
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "null plan");
  const int L = (int)pl->hp.levels.size();
  if (prefetch < 0 || prefetch > 2) return fail(MGWR_ERR_INVALID_ARG, "prefetch must be 0, 1 or 2");
  if (coarse_level < -1 || coarse_level >= L)
    return fail(MGWR_ERR_INVALID_ARG, "coarse_level must be -1 (rule), 0 (none) or 1 .. " + std::to_string(L - 1));
  pl->staging_set = !(prefetch == 0 && coarse_level == -1);
  pl->set_prefetch = prefetch;
  pl->set_coarse = coarse_level;
  return MGWR_OK;
}

int mgwr_plan_set_layout(mgwr_plan* pl, int layout) {
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "null plan");
  if (layout != MGWR_LAYOUT_AUTO && layout != MGWR_LAYOUT_NATURAL && layout != MGWR_LAYOUT_SPLIT)
    return fail(MGWR_ERR_INVALID_ARG, "layout must be MGWR_LAYOUT_AUTO, MGWR_LAYOUT_NATURAL or MGWR_LAYOUT_SPLIT");
  pl->set_layout = layout;
  return MGWR_OK;
}

int mgwr_plan_tuned(const mgwr_plan* pl, int* schedule, int* prefetch, int* coarse_level) {
  if (!pl) return fail(MGWR_ERR_INVALID_ARG, "null plan");
  int pf, c;
  staging_choice(pl, &pf, &c);
  if (schedule) *schedule = use_pipeline(pl) ? MGWR_SCHED_PIPELINED : MGWR_SCHED_STAGED;
  if (prefetch) *prefetch = pf;
  if (coarse_level) *coarse_level = c;
  return MGWR_OK;
}

int mgwr_batch_timing(mgwr_batch* bt, int enable, mgwr_timing* out) {
  if (!bt) return batch_fail(MGWR_ERR_INVALID_ARG, "null batch");
  if (bt->bound) HIP_TRY(hipStreamSynchronize(bt->stream));
  if (out) *out = bt->tacc;
  if (enable >= 0) {
    bt->timing = enable != 0;
    if (enable) bt->tacc = mgwr_timing{};
  }
  return MGWR_OK;
}

int mgwr_batch_destroy(mgwr_batch* bt) {
  delete bt;
  return MGWR_OK;
}

}  // extern "C"
