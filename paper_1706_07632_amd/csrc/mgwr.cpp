// C ABI and cycle driver of libmgwr (Algorithm 2 of arXiv 1706.07632 on top
// of the gfx950 kernels).  The library never allocates device memory: the
// caller's workspace holds the packed H-matrix and every level's arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hplan.h"
#include "kernels.h"
#include "mgwr.h"

using namespace mgwr;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(...)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (__VA_ARGS__);                                                            \
    if (e_ != hipSuccess) return fail(MGWR_ERR_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kNormParts = 1024;

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
  double* B0 = nullptr;      // f + a_{.,1} g
  double* part = nullptr;    // norm partials
  double* scal = nullptr;    // device scalar(s)
  DevOps<double> d64;
  DevOps<float> d32;
  bool mixed = false;
  // live timing (mgwr_timing_enable)
  struct Pending { hipEvent_t b, e; int cls; double flops, bytes; };
  bool timing = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  mgwr_timing tacc{};
  // time-pipelined cycles (float64)
  static constexpr int kMaxPipeCycles = 16;
  std::vector<Stage<double>> stages;   // host image for kMaxPipeCycles cycles
  int stages_per_cycle = 0, tasks_per_cycle = 0, norm_chunks = 0;
  const double* stages_f = nullptr;    // level-0 arrays the uploaded image refers to
  const double* stages_u = nullptr;
  Stage<double>* stages_dev = nullptr;
  int* counters = nullptr;
  int* flags_dev = nullptr;            // [0] ticket, [1] abort
  double* norms = nullptr;             // [kMaxPipeCycles][norm_chunks]
  int khint = 0;                       // cycles the last pipelined solve needed
  double cycle_flops = 0.0, cycle_bytes = 0.0;  // algorithmic work of one pipelined cycle
  // offsets computed by layout()
  struct Off {
    size_t stages, counters, flags, norms;
    size_t leaves, dn_list, ff_row, zu_row, a1, B0, part, scal;
    size_t dense64, dinv64, ffA64, zuB64, dense32, dinv32, ffA32, zuB32;
    std::vector<size_t> U64, F64, R64, U32, F32, R32;
    size_t total;
  } off;
};

namespace {

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
  pl->mixed = hp.p.precision == MGWR_MIXED_FP32;
  o.U32.assign(L, 0); o.F32.assign(L, 0); o.R32.assign(L, 0);
  if (pl->mixed) {
    o.dense32 = cv.take(pk.dense.size() * sizeof(float));
    o.dinv32 = cv.take(pk.dinv.size() * sizeof(float));
    o.ffA32 = cv.take(std::max<size_t>(1, pk.ffA.size()) * sizeof(float));
    o.zuB32 = cv.take(std::max<size_t>(1, pk.zuB.size()) * sizeof(float));
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
    long long spc = 1, visits = 1;
    for (int l = 0; l < L; ++l) {
      if (l == L - 1) spc += 2 * visits;
      else spc += visits * (2LL * (hp.p.nu1 + hp.p.nu2) + 3);
      visits *= hp.p.gamma;
    }
    const long long S = spc * mgwr_plan::kMaxPipeCycles;
    o.stages = cv.take((size_t)S * sizeof(Stage<double>));
    o.counters = cv.take((size_t)S * nleaf * sizeof(int));
    o.flags = cv.take(2 * sizeof(int));
    o.norms = cv.take((size_t)mgwr_plan::kMaxPipeCycles * ((hp.levels[0].N + 15) / 16) * sizeof(double));
  }
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
    if (pl->timing && (b = pool_event(pl))) hipEventRecord(b, pl->stream);
  }
  ~Timed() {
    if (!b) return;
    hipEvent_t e = pool_event(pl);
    if (!e) { pl->event_pool.push_back(b); return; }
    hipEventRecord(e, pl->stream);
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
  a.ff_row = pl->ff_row;
  a.ffA = ops.ffA;
  a.zu_row = pl->zu_row;
  a.zuB = ops.zuB;
  a.k = hp.p.k;
  a.nslots = hp.nslots;
  a.ring = std::max(hp.window + 2, 3);  // leaves written while older ones are still read
  return a;
}

// Zebra-in-time line relaxation of one colour on one level: every line of
// the colour is solved with (R~ + c_l I) by the H-forward substitution.
// Colour 0 is updated first: the coarse-grid points (1-based even in 1D,
// i + j even in 2D), which are the flat indices q with q % 2 == par0.
template <typename T>
int smooth(mgwr_plan* pl, DevOps<T>& ops, int l, int colour, T* F, T* U) {
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[l];
  int par0 = hp.p.dim == 1 ? 1 : 0;
  int par = colour == 0 ? par0 : 1 - par0;
  int ncols = (lv.N - par + 1) / 2;
  MarchArgs<T> a = base_args<T>(pl, ops, l);
  a.F = F; a.U = U; a.Out = nullptr;
  a.ld = lv.N; a.ncols = ncols; a.cstride = 2; a.coff = par;
  a.dim = hp.p.dim; a.n = lv.n; a.inv_h2 = (T)(1.0 / (lv.h * lv.h));
  Timed tm(pl, sizeof(T) == 8 ? MGWR_K_SMOOTH64 : MGWR_K_SMOOTH32, 2.0 * hp.stored * ncols,
           3.0 * hp.p.M * ncols * sizeof(T));
  HIP_TRY(launch_march<T>(MODE_SMOOTH, a, pl->stream));
  return MGWR_OK;
}

template <typename T>
int defect(mgwr_plan* pl, DevOps<T>& ops, int l, const T* F, T* U, T* Out) {
  const HostPlan& hp = pl->hp;
  const Level& lv = hp.levels[l];
  MarchArgs<T> a = base_args<T>(pl, ops, l);
  a.F = F; a.U = U; a.Out = Out;
  a.ld = lv.N; a.ncols = lv.N; a.cstride = 1; a.coff = 0;
  a.dim = hp.p.dim; a.n = lv.n; a.inv_h2 = (T)(1.0 / (lv.h * lv.h));
  Timed tm(pl, sizeof(T) == 8 ? MGWR_K_DEFECT64 : MGWR_K_DEFECT32, 2.0 * hp.stored * lv.N,
           3.0 * hp.p.M * lv.N * sizeof(T));
  HIP_TRY(launch_march<T>(MODE_RESID, a, pl->stream));
  return MGWR_OK;
}

// One cycle of Algorithm 2 on level l: ops.F[l] is the right-hand side,
// ops.U[l] the iterate (level 0 arrays are supplied through F0/U0).
template <typename T>
int cycle(mgwr_plan* pl, DevOps<T>& ops, int l) {
  const HostPlan& hp = pl->hp;
  const int L = (int)hp.levels.size();
  const int M = hp.p.M;
  T* F = ops.F[l];
  T* U = ops.U[l];
  int rc;
  if (l == L - 1) {  // coarsest grid (one point): the line solve is the direct solve
    if ((rc = smooth<T>(pl, ops, l, 0, F, U))) return rc;
    if ((rc = smooth<T>(pl, ops, l, 1, F, U))) return rc;
    return MGWR_OK;
  }
  for (int s = 0; s < hp.p.nu1; ++s) {
    if ((rc = smooth<T>(pl, ops, l, 0, F, U))) return rc;
    if ((rc = smooth<T>(pl, ops, l, 1, F, U))) return rc;
  }
  if ((rc = defect<T>(pl, ops, l, F, U, ops.R[l]))) return rc;
  {
    Timed tm(pl, MGWR_K_RESTRICT, 0.0, (double)M * (hp.levels[l].N + hp.levels[l + 1].N) * sizeof(T));
    HIP_TRY(launch_restrict<T>(ops.R[l], ops.F[l + 1], hp.p.dim, hp.levels[l].n, M, pl->stream));
  }
  HIP_TRY(launch_fill<T>(ops.U[l + 1], (long long)M * hp.levels[l + 1].N, (T)0, pl->stream));
  for (int gm = 0; gm < hp.p.gamma; ++gm)
    if ((rc = cycle<T>(pl, ops, l + 1))) return rc;
  {
    Timed tm(pl, MGWR_K_PROLONG, 0.0, (double)M * (2.0 * hp.levels[l].N + hp.levels[l + 1].N) * sizeof(T));
    HIP_TRY(launch_prolong<T>(ops.U[l + 1], U, hp.p.dim, hp.levels[l].n, M, pl->stream));
  }
  for (int s = 0; s < hp.p.nu2; ++s) {
    if ((rc = smooth<T>(pl, ops, l, 0, F, U))) return rc;
    if ((rc = smooth<T>(pl, ops, l, 1, F, U))) return rc;
  }
  return MGWR_OK;
}


// ---- time-pipelined cycles ------------------------------------------------
// Stage list of one cycle of Algorithm 2 on level l (float64), appended to
// `out`; `prev` is the index of the stage whose output the first new stage
// consumes.  Returns the index of the last stage appended.
int append_cycle_stages(mgwr_plan* pl, int l, int prev, std::vector<Stage<double>>& out) {
  const HostPlan& hp = pl->hp;
  const int L = (int)hp.levels.size();
  const Level& lv = hp.levels[l];
  DevOps<double>& ops = pl->d64;
  auto base = [&](int kind) {
    Stage<double> st{};
    st.kind = kind;
    st.prev = prev;
    st.nleaf = (int)hp.pk.leaves.size();
    st.leaves = pl->leaves;
    return st;
  };
  auto push = [&](Stage<double>& st) {
    out.push_back(st);
    prev = (int)out.size() - 1;
  };
  auto smooth_stage = [&](int colour) {
    int par0 = hp.p.dim == 1 ? 1 : 0;
    int par = colour == 0 ? par0 : 1 - par0;
    int ncols = (lv.N - par + 1) / 2;
    if (ncols <= 0) return;
    Stage<double> st = base(STG_SMOOTH);
    st.m = base_args<double>(pl, ops, l);
    st.m.F = ops.F[l]; st.m.U = ops.U[l]; st.m.Out = nullptr;
    st.m.ld = lv.N; st.m.ncols = ncols; st.m.cstride = 2; st.m.coff = par;
    st.m.dim = hp.p.dim; st.m.n = lv.n; st.m.inv_h2 = 1.0 / (lv.h * lv.h);
    st.nchunks = (ncols + 15) / 16;
    push(st);
  };
  if (l == L - 1) {
    smooth_stage(0);
    smooth_stage(1);
    return prev;
  }
  for (int s2 = 0; s2 < hp.p.nu1; ++s2) { smooth_stage(0); smooth_stage(1); }
  {
    Stage<double> st = base(STG_RESID);
    st.m = base_args<double>(pl, ops, l);
    st.m.F = ops.F[l]; st.m.U = ops.U[l]; st.m.Out = ops.R[l];
    st.m.ld = lv.N; st.m.ncols = lv.N; st.m.cstride = 1; st.m.coff = 0;
    st.m.dim = hp.p.dim; st.m.n = lv.n; st.m.inv_h2 = 1.0 / (lv.h * lv.h);
    st.nchunks = (lv.N + 15) / 16;
    push(st);
  }
  const Level& lc = hp.levels[l + 1];
  {
    Stage<double> st = base(STG_RESTRICT);
    st.src = ops.R[l]; st.dst = ops.F[l + 1]; st.zero = ops.U[l + 1];
    st.dim = hp.p.dim; st.nf = lv.n; st.nc = lc.n;
    st.nchunks = (lc.N + kStencilCols - 1) / kStencilCols;
    push(st);
  }
  for (int gm = 0; gm < hp.p.gamma; ++gm) prev = append_cycle_stages(pl, l + 1, prev, out);
  {
    Stage<double> st = base(STG_PROLONG);
    st.prev = prev;
    st.src = ops.U[l + 1]; st.dst = ops.U[l];
    st.dim = hp.p.dim; st.nf = lv.n; st.nc = lc.n;
    st.nchunks = (lv.N + kStencilCols - 1) / kStencilCols;
    push(st);
  }
  for (int s2 = 0; s2 < hp.p.nu2; ++s2) { smooth_stage(0); smooth_stage(1); }
  return prev;
}

// Builds and uploads the stage table of kMaxPipeCycles cycles for level-0
// arrays (f, u); task and counter offsets are assigned in stage order.
int upload_stages(mgwr_plan* pl, const double* b, double* u) {
  if (pl->stages_f == b && pl->stages_u == u && !pl->stages.empty()) return MGWR_OK;
  const HostPlan& hp = pl->hp;
  const int nleaf = (int)hp.pk.leaves.size();
  pl->d64.F[0] = const_cast<double*>(b);
  pl->d64.U[0] = u;
  std::vector<Stage<double>>& st = pl->stages;
  st.clear();
  int prev = -1;
  int per_cycle = -1;
  for (int c = 0; c < mgwr_plan::kMaxPipeCycles; ++c) {
    prev = append_cycle_stages(pl, 0, prev, st);
    // defect of the full system after the cycle: its norm is the stopping test
    Stage<double> nd{};
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
    pl->norm_chunks = nd.nchunks;
    nd.norm_out = pl->norms + (size_t)c * nd.nchunks;
    st.push_back(nd);
    prev = (int)st.size() - 1;
    if (per_cycle < 0) per_cycle = (int)st.size();
  }
  int task = 0;
  for (size_t i = 0; i < st.size(); ++i) {
    st[i].task0 = task;
    task += st[i].nchunks;
    st[i].cnt_off = (int)i * nleaf;
  }
  pl->stages_per_cycle = per_cycle;
  pl->cycle_flops = pl->cycle_bytes = 0.0;
  for (int i = 0; i < per_cycle; ++i) {
    const Stage<double>& x = st[i];
    if (x.kind == STG_SMOOTH || x.kind == STG_RESID) {
      pl->cycle_flops += 2.0 * hp.stored * x.m.ncols;
      pl->cycle_bytes += 3.0 * hp.p.M * x.m.ncols * sizeof(double);
    } else {
      const double Nf = hp.p.dim == 1 ? x.nf : (double)x.nf * x.nf;
      const double Nc = hp.p.dim == 1 ? x.nc : (double)x.nc * x.nc;
      pl->cycle_bytes += (x.kind == STG_RESTRICT ? (Nf + 2 * Nc) : (Nc + 2 * Nf)) * hp.p.M * sizeof(double);
    }
  }
  pl->tasks_per_cycle = st[per_cycle].task0;
  if ((size_t)st.size() * sizeof(Stage<double>) > pl->off.counters - pl->off.stages)
    return fail(MGWR_ERR_STATE, "internal error: stage table larger than its workspace region");
  HIP_TRY(hipMemcpyAsync(pl->stages_dev, st.data(), st.size() * sizeof(Stage<double>), hipMemcpyHostToDevice,
                         pl->stream));
  pl->stages_f = b;
  pl->stages_u = u;
  return MGWR_OK;
}

// Runs `K` cycles in one launch; per-cycle residual norms land in res[0..K).
int run_pipelined(mgwr_plan* pl, const double* b, double* u, int K, double* res) {
  int rc;
  if ((rc = upload_stages(pl, b, u))) return rc;
  const int nleaf = (int)pl->hp.pk.leaves.size();
  const int S = pl->stages_per_cycle * K;
  HIP_TRY(launch_fill_int(pl->counters, (long long)S * nleaf, 0, pl->stream));
  HIP_TRY(launch_fill_int(pl->flags_dev, 2, 0, pl->stream));
  PipeArgs<double> pa;
  pa.stages = pl->stages_dev;
  pa.nstages = S;
  pa.ntasks = pl->tasks_per_cycle * K;
  pa.counters = pl->counters;
  pa.ticket = pl->flags_dev;
  pa.abortf = pl->flags_dev + 1;
  size_t lds = march_lds_bytes<double>(base_args<double>(pl, pl->d64, 0));
  {
    Timed tm(pl, MGWR_K_PIPE64, pl->cycle_flops * K, pl->cycle_bytes * K);
    HIP_TRY(launch_pipeline<double>(pa, lds, pl->stream));
  }
  std::vector<double> nh((size_t)K * pl->norm_chunks);
  int flags[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(nh.data(), pl->norms, nh.size() * sizeof(double), hipMemcpyDeviceToHost, pl->stream));
  HIP_TRY(hipMemcpyAsync(flags, pl->flags_dev, sizeof(flags), hipMemcpyDeviceToHost, pl->stream));
  HIP_TRY(hipStreamSynchronize(pl->stream));
  if (!pl->pending.empty()) drain_timing(pl);
  if (flags[1]) return fail(MGWR_ERR_HIP, "pipelined cycles stalled (a progress wait exceeded its bound)");
  for (int c = 0; c < K; ++c) {
    double m = 0.0;
    bool bad = false;
    for (int j = 0; j < pl->norm_chunks; ++j) {
      double v = nh[(size_t)c * pl->norm_chunks + j];
      if (v != v) bad = true;
      else m = std::max(m, v);
    }
    res[c] = bad ? std::nan("") : m;
  }
  return MGWR_OK;
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
}

int mgwr_plan_create(const mgwr_params* p, const double* t_host, mgwr_plan** out) {
  if (!p || !out) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
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
  *out = pl;
  return MGWR_OK;
}

int mgwr_plan_workspace_bytes(const mgwr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  *bytes = plan->off.total;
  return MGWR_OK;
}

int mgwr_plan_bind(mgwr_plan* pl, void* ws, size_t bytes, void* stream) {
  if (!pl || !ws) return fail(MGWR_ERR_INVALID_ARG, "null argument");
  if (bytes < pl->off.total) return fail(MGWR_ERR_STATE, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return fail(MGWR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  HIP_TRY(hipGetDevice(&pl->device));
  pl->stream = (hipStream_t)stream;
  pl->ws = (unsigned char*)ws;
  pl->ws_bytes = bytes;
  const HostPlan& hp = pl->hp;
  const PackedPlan& pk = hp.pk;
  const auto& o = pl->off;
  unsigned char* w = pl->ws;
  pl->leaves = (LeafDesc*)(w + o.leaves);
  pl->dn_list = (int*)(w + o.dn_list);
  pl->ff_row = (int*)(w + o.ff_row);
  pl->zu_row = (int*)(w + o.zu_row);
  pl->a1 = (double*)(w + o.a1);
  pl->part = (double*)(w + o.part);
  pl->scal = (double*)(w + o.scal);
  pl->B0 = (double*)(w + o.B0);
  pl->stages_dev = (Stage<double>*)(w + o.stages);
  pl->counters = (int*)(w + o.counters);
  pl->flags_dev = (int*)(w + o.flags);
  pl->norms = (double*)(w + o.norms);
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
  put(o.dense64, pk.dense.data(), pk.dense.size() * sizeof(double));
  put(o.dinv64, pk.dinv.data(), pk.dinv.size() * sizeof(double));
  put(o.ffA64, pk.ffA.data(), pk.ffA.size() * sizeof(double));
  put(o.zuB64, pk.zuB.data(), pk.zuB.size() * sizeof(double));
  HIP_TRY(hipMemcpyAsync(w, img.data(), img.size(), hipMemcpyHostToDevice, pl->stream));
  if (pl->mixed) {
    pl->d32.dense = (float*)(w + o.dense32);
    pl->d32.dinv = (float*)(w + o.dinv32);
    pl->d32.ffA = (float*)(w + o.ffA32);
    pl->d32.zuB = (float*)(w + o.zuB32);
    pl->d32.U.assign(L, nullptr); pl->d32.F.assign(L, nullptr); pl->d32.R.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
      pl->d32.U[l] = (float*)(w + o.U32[l]);
      pl->d32.F[l] = (float*)(w + o.F32[l]);
      if (l + 1 < L) pl->d32.R[l] = (float*)(w + o.R32[l]);
    }
    // float copies are rounded on the device from the float64 image
    HIP_TRY(launch_cast<double, float>(pl->d64.dense, pl->d32.dense, (long long)pk.dense.size(), pl->stream));
    HIP_TRY(launch_cast<double, float>(pl->d64.dinv, pl->d32.dinv, (long long)pk.dinv.size(), pl->stream));
    HIP_TRY(launch_cast<double, float>(pl->d64.ffA, pl->d32.ffA, (long long)pk.ffA.size(), pl->stream));
    HIP_TRY(launch_cast<double, float>(pl->d64.zuB, pl->d32.zuB, (long long)pk.zuB.size(), pl->stream));
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
  HIP_TRY(set_pipeline_lds_limit<double>(cap));
  HIP_TRY(set_pipeline_lds_limit<float>(cap));
  HIP_TRY(hipStreamSynchronize(pl->stream));
  pl->bound = true;
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
  if ((rc = defect<double>(pl, pl->d64, 0, b, const_cast<double*>(u), dst))) return rc;
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
  const HostPlan& hp = pl->hp;
  const int M = hp.p.M;
  const long long MN = (long long)M * hp.levels[0].N;
  mgwr_stats s{};
  const double* b = f;
  if (g) {
    HIP_TRY(launch_rhs0(f, g, pl->a1, pl->B0, M, hp.levels[0].N, pl->stream));
    b = pl->B0;
  }
  if (!(flags & MGWR_GUESS_IN_U)) HIP_TRY(launch_fill<double>(u, MN, 0.0, pl->stream));
  if ((rc = norm_inf<double>(pl, b, MN, &s.bnorm))) return rc;
  if (!std::isfinite(s.bnorm)) {
    if (st) *st = s;
    return fail(MGWR_ERR_NONFINITE, "right-hand side is not finite");
  }
  if (flags & MGWR_GUESS_IN_U) {
    if ((rc = defect<double>(pl, pl->d64, 0, b, u, pl->d64.R[0]))) return rc;
    if ((rc = norm_inf<double>(pl, pl->d64.R[0], MN, &s.res0))) return rc;
  } else {
    s.res0 = s.bnorm;
  }
  s.res = s.res0;
  const double target = tol * s.bnorm;
  int status = MGWR_ERR_NOT_CONVERGED;
  if (!std::isfinite(s.res0)) status = MGWR_ERR_NONFINITE;
  else if (s.res0 <= target) status = MGWR_OK;

  if (status == MGWR_ERR_NOT_CONVERGED && !pl->mixed && hp.p.schedule == MGWR_SCHED_PIPELINED) {
    int K = pl->khint > 0 ? pl->khint : 8;
    int converged_at = -1;
    while (s.cycles < hp.p.max_cycles) {
      K = std::max(1, std::min({K, mgwr_plan::kMaxPipeCycles, hp.p.max_cycles - s.cycles}));
      double res[mgwr_plan::kMaxPipeCycles];
      if ((rc = run_pipelined(pl, b, u, K, res))) return rc;
      for (int c = 0; c < K; ++c) {
        if (s.cycles + c < 64) s.history[s.cycles + c] = res[c];
        if (converged_at < 0 && res[c] <= target) converged_at = s.cycles + c + 1;
      }
      const double first = s.cycles == 0 ? s.res0 : s.res;
      s.cycles += K;
      s.res = res[K - 1];
      if (!std::isfinite(s.res)) { status = MGWR_ERR_NONFINITE; break; }
      if (s.res <= target) { status = MGWR_OK; break; }
      // extrapolate the remaining cycles from the observed contraction
      double rate = std::pow(std::max(s.res / first, 1e-300), 1.0 / K);
      K = (rate < 0.99 && rate > 0) ? (int)std::ceil(std::log(target / s.res) / std::log(rate)) : K;
    }
    if (converged_at > 0) pl->khint = converged_at;
  } else if (status == MGWR_ERR_NOT_CONVERGED && !pl->mixed) {
    pl->d64.F[0] = const_cast<double*>(b);
    pl->d64.U[0] = u;
    while (s.cycles < hp.p.max_cycles) {
      if ((rc = cycle<double>(pl, pl->d64, 0))) return rc;
      s.cycles++;
      if ((rc = defect<double>(pl, pl->d64, 0, b, u, pl->d64.R[0]))) return rc;
      if ((rc = norm_inf<double>(pl, pl->d64.R[0], MN, &s.res))) return rc;
      if (s.cycles <= 64) s.history[s.cycles - 1] = s.res;
      if (!std::isfinite(s.res)) { status = MGWR_ERR_NONFINITE; break; }
      if (s.res <= target) { status = MGWR_OK; break; }
    }
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
      if ((rc = defect<double>(pl, pl->d64, 0, b, u, pl->d64.R[0]))) return rc;
      if ((rc = norm_inf<double>(pl, pl->d64.R[0], MN, &s.res))) return rc;
      if (s.refinements <= 64) s.history[s.refinements - 1] = s.res;
      if (!std::isfinite(s.res)) { status = MGWR_ERR_NONFINITE; break; }
      if (s.res <= target) { status = MGWR_OK; break; }
      HIP_TRY(launch_cast<double, float>(pl->d64.R[0], pl->d32.F[0], MN, pl->stream));
    }
  }
  s.avg_factor = (s.cycles > 0 && s.res0 > 0) ? std::pow(s.res / s.res0, 1.0 / s.cycles) : 0.0;
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
  a.ld = ncols; a.ncols = ncols; a.cstride = 1; a.coff = 0; a.dim = 0; a.n = 0; a.inv_h2 = 0.0;
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
  a.ld = ncols; a.ncols = ncols; a.cstride = 1; a.coff = 0; a.dim = 0; a.n = 0; a.inv_h2 = 0.0;
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

int mgwr_plan_destroy(mgwr_plan* pl) {
  if (!pl) return MGWR_OK;
  if (pl->bound && !pl->pending.empty()) {
    hipStreamSynchronize(pl->stream);
    drain_timing(pl);
  }
  for (hipEvent_t e : pl->event_pool) hipEventDestroy(e);
  delete pl;
  return MGWR_OK;
}

const char* mgwr_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
