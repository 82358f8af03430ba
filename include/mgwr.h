/*
 * mgwr.h -- C ABI of libmgwr: multigrid waveform relaxation (MGWR) with an
 * H-matrix representation of the L1 time discretisation, for the
 * time-fractional heat equation on graded time meshes, on AMD gfx950.
 *
 * Method (Hu, Rodrigo, Gaspar, arXiv 1706.07632):
 *   Section 2  -- model problem, Caputo derivative, L1 scheme on the graded
 *                 mesh t_m = T (m/M)^r, matrix R (lower triangular).
 *   Section 3  -- H-matrix representation R~ of R: admissibility
 *                 (Definition 3.1), rank-k Taylor factors A, B, recursive 2x2
 *                 block construction.
 *   Section 4  -- Algorithm 2 (discrete WRMG: zebra-in-time red-black line
 *                 relaxation, coarsening in space only), Algorithm 3 (H-matrix
 *                 matrix-vector product), Algorithm 4 (H-matrix forward
 *                 substitution).
 *
 * The discrete system solved (interior points q, levels m = 1..M):
 *   sum_j R~_{m,j} u_{q,j} + (A_h u_{.,m})_q = f_{q,m} + a_{m,1} g_q
 * with A_h the 3-point (1D) / 5-point (2D) negative Laplacian over h^2 and
 * homogeneous Dirichlet values.
 *
 * Conventions
 *  - Pointers named *_dev are device pointers of the GPU the plan is bound
 *    to (e.g. torch.Tensor.data_ptr() of a ROCm tensor); every other pointer
 *    is host memory.
 *  - Space-time arrays are [M][N] row-major, float64: row m-1 holds time level
 *    t_m, N = n^dim interior points, in 2D the flat index is q = iy*n + ix.
 *  - The library never allocates device memory.  The caller provides one
 *    workspace (mgwr_plan_workspace_bytes) at bind time and owns all arrays.
 *  - All entry points return an mgwr status; on failure mgwr_last_error()
 *    returns a thread-local message.  Nothing throws across the ABI.
 *  - A plan is bound to one device and one stream; it is not thread-safe.
 *    Calls are asynchronous on that stream unless stated otherwise.
 */
#ifndef MGWR_H
#define MGWR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MGWR_OK = 0,
  MGWR_ERR_INVALID_ARG = 1,   /* parameter validation failed; no device work done */
  MGWR_ERR_STATE = 2,         /* plan not bound, or workspace too small */
  MGWR_ERR_HIP = 3,           /* a HIP runtime call failed */
  MGWR_ERR_NOT_CONVERGED = 4, /* max_cycles reached; u and stats still written */
  MGWR_ERR_NONFINITE = 5,     /* a residual norm was NaN/Inf; u and stats still written */
  MGWR_ERR_MODEL = 6          /* learned weights missing or corrupt (mgwr_model_load) */
};

typedef enum {
  MGWR_FP64 = 0,        /* every cycle in float64 */
  MGWR_MIXED_FP32 = 1,  /* float64 outer residual and correction, float32 inner V-cycles */
  MGWR_MIXED_BF16 = 2   /* as MGWR_MIXED_FP32, with the low-rank (Taylor) factors of the inner cycles
                           stored in bfloat16 (round to nearest even from their float32 values) and
                           widened to float32 for the products; dense leaves, shifted inverses, the
                           iterates and every accumulation stay float32, the outer steps float64 */
} mgwr_precision;

/* Flags of mgwr_solve. */
enum {
  MGWR_GUESS_IN_U = 1u,  /* u_dev holds the initial iterate (otherwise the zero grid function) */
  MGWR_WARM_START = 2u,  /* initial iterate predicted by the plan's network (mgwr_plan_set_warm_start
                            or mgwr_model_load).  Judged by the true float64 residual: the prediction's
                            defect is always evaluated (stats.warm_res0) and a prediction whose defect
                            is not finite is dropped at once; after the first outer step from it (the
                            first pipelined launch, or the first cycle / refinement of a staged solve)
                            its residual is compared with the residual the zero iterate reaches in the
                            same number of cycles, ||b||_inf rho0^c with rho0 the plan's average
                            factor of its last solve from zero (rho0 = 1 before there is one).  Above
                            twice that (and above the tolerance): the prediction is dropped, the solve
                            restarts from the zero iterate and the cycles already spent stay counted */
  MGWR_WARM_RES0 = 4u    /* kept for compatibility: the prediction's residual is always evaluated */
};

typedef struct {
  int dim;          /* 1 or 2 */
  int n;            /* interior points per side; n = 2^L - 1 with L >= 1; N = n^dim */
  double length;    /* spatial domain (0, length)^dim */
  int M;            /* number of time steps, >= 1 */
  double T;         /* final time (used only when no explicit mesh is given) */
  double alpha;     /* fractional order, 0 < alpha < 1 */
  double r;         /* grading exponent >= 1 (used only when no explicit mesh is given) */
  int k;            /* Taylor terms per admissible block (rank), 1 <= k <= 32 */
  int leaf;         /* cluster leaf size, 1 <= leaf <= 16 (16 by default) */
  int nu1, nu2;     /* pre/post smoothing steps of one cycle (Algorithm 2) */
  int gamma;        /* cycles on each coarser level: 1 = V-cycle, 2 = W-cycle */
  int max_cycles;   /* cap on cycles (plain) or inner cycles in total (mixed) */
  int precision;    /* mgwr_precision */
  int inner_cycles; /* mixed precision: inner V-cycles per outer refinement step (1..16) */
  int schedule;     /* MGWR_SCHED_AUTO (default), MGWR_SCHED_STAGED or MGWR_SCHED_PIPELINED */
  double eta;       /* admissibility parameter, > 0 (default 1): a block whose row and column
                       supports I_t, I_s satisfy d < a and diam(I_t) <= eta dist(I_s, I_t) is kept
                       in low-rank form.  eta = 1 is Definition 3.1; other values are the more
                       general conditions the remark after it allows.  The Taylor error of a block
                       decays like (eta / (eta + 2))^k (proof of Theorem 3.1 with the contraction
                       ratio of the condition), so larger eta compresses more at a given k */
  int cluster;      /* cluster tree: MGWR_CLUSTER_INDEX (default) or MGWR_CLUSTER_GEOMETRIC */
} mgwr_params;

/* Cluster trees of the time indices 1..M (Section 3 leaves the split rule open).
 * INDEX: a cluster of s > leaf indices splits into s/2 (rounded down) and the rest.
 * GEOMETRIC: a cluster splits where its time interval [t_lo+1, t_hi] is halved
 * (the first index past the midpoint starts the second child, each child keeping
 * at least one index): on a graded mesh the early clusters then hold many short
 * steps and the late ones few long steps, so blocks of similar time extent meet. */
enum { MGWR_CLUSTER_INDEX = 0, MGWR_CLUSTER_GEOMETRIC = 1 };

/* Cycle schedules (float64 solver).  Every operator of a cycle is causal in
 * time, so the pipelined schedule runs several whole cycles in one launch,
 * each stage (a smoothing half-sweep, a defect, a grid transfer) starting
 * time leaf i as soon as the stage before it has finished leaf i.  The staged
 * schedule launches one kernel per stage and checks the residual after every
 * cycle.  Both compute the same iterates up to the order of float64 rounding. */
enum { MGWR_SCHED_AUTO = 0, MGWR_SCHED_STAGED = 1, MGWR_SCHED_PIPELINED = 2 };
/* AUTO pipelines when the finest level has few 16-column chains (the staged
 * launches then leave most of the GPU idle) and stages otherwise. */

/* Fill *p with defaults: leaf 16, V(1,1), gamma 1, max_cycles 50, FP64, length 1, T 1,
 * automatic schedule, eta 1, index-bisection clusters. */
void mgwr_params_default(mgwr_params* p);

typedef struct {
  int cycles;        /* V-cycles run (all precisions) */
  int refinements;   /* outer float64 residual evaluations in mixed precision */
  double res0;       /* ||b - A u_initial||_inf */
  double bnorm;      /* ||b||_inf, b = f + a_{.,1} g */
  double res;        /* final ||b - A u||_inf (float64; a staged 2D solve in split storage takes it
                        from the last half-sweep's changes, see mgwr_plan_set_layout) */
  double avg_factor; /* (res/res0)^(1/cycles) */
  double history[64]; /* ||b - A u||_inf after each of the first 64 outer steps (cycles or
                         refinements); 0 where a pipelined launch with a learned cycle count
                         evaluated the norm only after its last cycle */
  int used_warm_start; /* 1 if the network's prediction was the initial iterate of the returned solution */
  double warm_res0;    /* ||b - A u_predicted||_inf (every warm start; NaN without one) */
  double setup_ms;     /* host set-up of the plan: mgwr_plan_create plus the last mgwr_plan_bind */
  double solve_ms;     /* wall time of this solve (it returns with all its device work finished) */
} mgwr_stats;

typedef struct mgwr_plan mgwr_plan;

/* Host-only setup (no device work).  Builds the time mesh (t_host[0..M] if
 * given, else t_m = T (m/M)^r), the L1 weights, the cluster tree, the block
 * tree of Definition 3.1, the Taylor factors of Section 3 and every level's
 * shifted diagonal blocks, all in float64, and packs them for the device.
 * t_host must be strictly increasing with t_host[0] = 0.
 * Errors: MGWR_ERR_INVALID_ARG (n not 2^L-1, alpha outside (0,1), M < 1,
 * k or leaf out of range, non-monotone mesh). */
int mgwr_plan_create(const mgwr_params* p, const double* t_host, mgwr_plan** out);

/* Device bytes the caller must provide at bind time. */
int mgwr_plan_workspace_bytes(const mgwr_plan* plan, size_t* bytes);

/* Bind to the current device: copies the packed H-matrix (one host-to-device
 * copy on `stream`) into workspace_dev, which must stay valid and unused by
 * the caller until the plan is destroyed or re-bound.  `stream` is a
 * hipStream_t (NULL = default stream).  workspace_dev must be 256-byte
 * aligned.  Synchronises the stream before returning. */
int mgwr_plan_bind(mgwr_plan* plan, void* workspace_dev, size_t bytes, void* stream);

/* Solve the discrete system (Algorithm 2 cycles until
 * ||b - A u||_inf <= tol ||b||_inf, b = f + a_{.,1} g).
 *   f_dev [M][N]  source at t_1..t_M
 *   g_dev [N]     initial value u(x, 0); NULL means zero
 *   u_dev [M][N]  output; read as the initial iterate iff flags & MGWR_GUESS_IN_U
 * Returns MGWR_OK, MGWR_ERR_NOT_CONVERGED or MGWR_ERR_NONFINITE (u and stats
 * written in all three cases).  Synchronises the stream once per cycle to
 * read the residual norm. */
int mgwr_solve(mgwr_plan* plan, const double* f_dev, const double* g_dev, double tol,
               double* u_dev, unsigned flags, mgwr_stats* stats);

/* out_dev = b - A u with b = f + a_{.,1} g (g_dev may be NULL): the float64
 * defect of the full system (the defect step of Algorithm 2, with Algorithm 3
 * for R~).  If norm_host is not NULL the stream is synchronised and
 * ||out||_inf is stored there.  out_dev may be NULL when only the norm is
 * wanted. */
int mgwr_residual(mgwr_plan* plan, const double* f_dev, const double* g_dev, const double* u_dev,
                  double* out_dev, double* norm_host);

/* out_dev = A_{h,tau} u_dev in float64: the space-time operator of the
 * discrete system (Section 2 for R, Section 3 for its representation R~,
 * Algorithm 3 for the product), (A u)_{q,m} = sum_j R~_{m,j} u_{q,j} +
 * (A_h u_{.,m})_q, both arrays [M][N] row-major on the plan's device.
 * u_dev and out_dev must not overlap.  Asynchronous on the plan's stream.
 * Errors: MGWR_ERR_INVALID_ARG (null array), MGWR_ERR_STATE (plan not bound). */
int mgwr_apply_A(mgwr_plan* plan, const double* u_dev, double* out_dev);

/* Algorithm 3 on its own: y_dev = R~ x_dev for `ncols` independent columns,
 * both [M][ncols] row-major. */
int mgwr_hmatvec(mgwr_plan* plan, const double* x_dev, double* y_dev, int ncols);

/* Algorithm 4 on its own: solve (R~ + c_level I) x = b for `ncols` columns,
 * [M][ncols] row-major, where c_level = 2 dim / h_level^2 is the diagonal of
 * the spatial stencil on multigrid level `level` (0 = finest). */
int mgwr_htrsm(mgwr_plan* plan, int level, const double* b_dev, double* x_dev, int ncols);

/* Live kernel timing.  When enabled, every launch of the classes below is
 * bracketed by a pair of hipEvents on the plan's stream; durations, launch
 * counts and the algorithmic flops and HBM bytes of those launches accumulate
 * until read.  Algorithmic counts per launch: time-marching kernels 2 S flops
 * per column (S = stored entries of R~, dense leaves counted full) and 3 M
 * words per column (f, the other colour or u, and the written line);
 * restriction M (N_f + 2 N_c) words, N_f / 2 when it reads the first-colour
 * defect only; prolongation M (N_c + 2 N_f) words, N_c + N_f when it corrects
 * the second colour only (a first-colour half-sweep follows).  In 1D with
 * nu1, nu2 >= 1 both transfers are fused into the marches and have no
 * launches of their own. */
enum {
  MGWR_K_SMOOTH64 = 0,  /* zebra line relaxation, float64 */
  MGWR_K_DEFECT64 = 1,  /* defect b - A u, float64 */
  MGWR_K_SMOOTH32 = 2,  /* zebra line relaxation, float32 (mixed inner cycles) */
  MGWR_K_DEFECT32 = 3,  /* defect, float32 (mixed inner cycles) */
  MGWR_K_RESTRICT = 4,  /* full-weighting restriction (either precision) */
  MGWR_K_PROLONG = 5,   /* interpolation and correction (either precision) */
  MGWR_K_PIPE64 = 6,    /* one launch of K time-pipelined float64 cycles (all stages) */
  MGWR_K_COARSE = 7,    /* staged schedule: one pipelined launch of a cycle's coarse levels (either precision) */
  MGWR_K_SIDE = 8,      /* a batch's staged instances solved side by side: one entry per batch solve, the
                           wall time of that whole phase and the algorithmic work of all its cycles */
  MGWR_K_CLASSES = 9
};
typedef struct {
  long long launches[MGWR_K_CLASSES];
  double ms[MGWR_K_CLASSES];      /* summed event-measured durations */
  double flops[MGWR_K_CLASSES];   /* summed algorithmic flops */
  double bytes[MGWR_K_CLASSES];   /* summed algorithmic HBM bytes */
} mgwr_timing;
/* enable != 0 turns timing on and clears the counters; 0 turns it off. */
int mgwr_timing_enable(mgwr_plan* plan, int enable);
/* Synchronises the plan's stream and returns the counters. */
int mgwr_timing_get(mgwr_plan* plan, mgwr_timing* out);

/* Batched solves: several bound plans (different n, M, alpha, k, dim allowed,
 * same device) solved together.  Their time-pipelined cycles are merged into
 * one launch with the stages of the instances interleaved, so the instances
 * advance concurrently; every instance keeps its own cycle count and
 * stopping test.  The batch owns a small workspace of its own (stage table,
 * progress counters, norms); each plan keeps using its own workspace. */
typedef struct mgwr_batch mgwr_batch;
/* plans[0..count) must stay alive and bound while the batch is used. */
int mgwr_batch_create(int count, mgwr_plan* const* plans, mgwr_batch** out);
int mgwr_batch_workspace_bytes(const mgwr_batch* batch, size_t* bytes);
/* workspace_dev: 256-byte aligned device memory; stream: hipStream_t or NULL. */
int mgwr_batch_bind(mgwr_batch* batch, void* workspace_dev, size_t bytes, void* stream);
/* f_dev[i], g_dev[i] (g_dev or g_dev[i] may be NULL), u_dev[i]: the arrays of
 * mgwr_solve for instance i; stats may be NULL or hold `count` entries.
 * Instances with the pipelined schedule run first, in one merged launch on
 * the batch's stream.  Instances with the staged schedule are then solved
 * side by side by up to 8 host threads, each on a HIP stream the batch owns
 * (default priority).  Each plan's own stream is synchronised before its
 * arrays are touched, and all work is complete when the call returns.  They
 * run one by one instead when two entries share a plan.  With
 * MGWR_WARM_START the predictions of plans sharing a network take turns on
 * it (its buffers and stream) while the cycles run side by side.  With at
 * least 8 staged instances each starts its coarse pipelined launch one level
 * below the single-solve rule (mgwr_plan_tuned reports the single-solve
 * choice).  The worker streams overlap only on hardware queues of their own:
 * HIP gives a process 4 unless GPU_MAX_HW_QUEUES (read when HIP starts) asks
 * for more; 16 suits the 8 workers.  Returns MGWR_OK when every instance
 * converged, else the first non-OK status in entry order. */
int mgwr_batch_solve(mgwr_batch* batch, const double* const* f_dev, const double* const* g_dev, double tol,
                     double* const* u_dev, unsigned flags, mgwr_stats* stats);
/* Timing of the batch's work: event-timed merged launches (class
 * MGWR_K_PIPE64) and the side-by-side phase of its staged instances (class
 * MGWR_K_SIDE, host wall clock; per-launch timing of the plans involved is
 * suspended while worker threads solve them, so that no plan's events are
 * recorded from another thread); synchronises.
 * out (nullable) receives the counters; enable 1 clears them and turns timing
 * on, 0 turns it off, -1 leaves it unchanged. */
int mgwr_batch_timing(mgwr_batch* batch, int enable, mgwr_timing* out);
int mgwr_batch_destroy(mgwr_batch* batch);
/* Graph replay of the batched launch (off by default).  When on, a launch
 * whose stage table, counters and grid equal the previous one's (the same
 * plans and arrays solved again with the learned cycle counts) is replayed
 * from a captured HIP graph (fill kernels + pipeline kernel, no memset
 * nodes) instead of being re-uploaded and re-launched; any change recaptures. */
int mgwr_batch_set_graph(mgwr_batch* batch, int enable);
/* Number of graph replays so far (host). */
int mgwr_batch_graph_replays(const mgwr_batch* batch, long long* replays);

/* Per-XCD work queues of the time-pipelined launches (process-wide, off by
 * default: the static split loses the global ticket's load balance, and the
 * launches measured slower although they fetch less).  Workgroups are dispatched to the chip's 8 XCDs round-robin
 * (workgroup b on XCD b mod 8, each XCD with its own L2); with the queues a
 * launch's work items are dealt to the XCDs so that each round of the merged
 * instances' stages is cut into 8 contiguous blocks, one per XCD: an
 * instance's chains stay on the same XCDs in every stage, and its H-matrix
 * rows are read from their L2 instead of once per XCD per stage.  Each
 * queue lists its work items in stage order and holds exactly as many as its
 * XCD runs workgroups, which keeps the launch free of deadlock as with one
 * global ticket; the dispatch order is checked on each device (a probe
 * launch at the first binding) and the queues are used only where it holds.
 * Results are the same either way.  *previous (nullable) receives the old
 * setting. */
int mgwr_set_xcd_queues(int enable, int* previous);
/* Whether this plan's pipelined launches use the queues (enabled and the
 * device's dispatch confirmed); the plan must be bound. */
int mgwr_xcd_queues_in_use(const mgwr_plan* plan, int* in_use);

/* Autotuner of the schedule and of the staged schedule's knobs: solves f
 * twice with each candidate (the second solve of each runs with the cycle
 * count the first one learned) and keeps the fastest.  Candidates: whole
 * cycles time-pipelined in one launch; staged launches per operator with the
 * shallow or the deep operand prefetch in the marches (see
 * mgwr_plan_set_staging) and the coarse pipelined launch starting at the
 * level the rule picks or one level either side; in 2D the best of these is
 * then timed once more in the other storage (mgwr_plan_set_layout).  The
 * choice holds for this plan and for every MGWR_SCHED_AUTO plan of the same
 * (dim, n, M, precision,
 * inner cycles, k) in this process; the schedule is returned in *chosen
 * (MGWR_SCHED_STAGED or MGWR_SCHED_PIPELINED, nullable).  u receives the
 * solution.  A batch runs its pipelined instances in one merged launch and
 * its staged ones side by side on worker streams. */
int mgwr_plan_autotune(mgwr_plan* plan, const double* f_dev, const double* g_dev, double tol, double* u_dev,
                       int* chosen);

/* Knobs of the staged schedule (host only; Section 4's cycle is unchanged,
 * only how its operators are launched).  prefetch: operand prefetch of the
 * marches launched on their own, 0 = by mesh length (deep from 128 time
 * leaves), 1 = shallow (2 update tiles, 3 far-field chunks per wave), 2 =
 * deep (6 and 5).  coarse_level: the level from which each cycle's remaining
 * levels run as one pipelined launch, -1 = by rule (first level with at most
 * 64 chains of 16 columns), 0 = none, 1 .. levels-1.  (0, -1) restores the
 * rules.  MGWR_ERR_INVALID_ARG for values out of range. */
int mgwr_plan_set_staging(mgwr_plan* plan, int prefetch, int coarse_level);

/* What a solve of this plan uses now: schedule (MGWR_SCHED_STAGED or
 * MGWR_SCHED_PIPELINED), march prefetch (0 by mesh length, 1 shallow, 2
 * deep) and coarse level (0 none) of the staged schedule.  Host only;
 * every pointer nullable. */
int mgwr_plan_tuned(const mgwr_plan* plan, int* schedule, int* prefetch, int* coarse_level);

/* Storage of the space-time arrays of a 2D plan inside its solves (host
 * only).  The caller's f, g, u are always in the natural order of the array
 * layout above.  The pipelined schedule computes the same iterates in either
 * storage, bit for bit.  The staged schedule in SPLIT storage forms the
 * defects of its cycles (and the norm of its float64 stopping test) from the
 * changes of the last second-colour half-sweep: after it the defect is zero
 * on that colour and, at a first-colour point, 1/h^2 times the sum of those
 * changes over its neighbours, which saves the H-matrix product of a defect
 * (Algorithm 3) per level and cycle; its iterates equal NATURAL's up to
 * rounding.  (Pipelined cycles, 1D and 2D in either storage, restrict the
 * same way; the coarse launch of the staged schedule keeps its defect
 * stages.)  These zebra
 * defects carry the rounding of the line solves, so solves with a tolerance
 * below 1e-10 use the defect of Algorithm 3 throughout.
 * MGWR_LAYOUT_SPLIT: every time row holds the first colour's points (the
 * even flat indices q, in order) and then the second colour's (the odd
 * ones), at every level, so a half-sweep of the red-black relaxation reads
 * and writes whole contiguous lines and the grid transfers touch one colour
 * block at a time; b = f + a_1 g is formed in it, a given initial iterate is
 * moved in at the start and the result moved back at the end (two passes
 * over u each).  MGWR_LAYOUT_NATURAL: natural order throughout.
 * MGWR_LAYOUT_AUTO (the default): the autotuner's choice for the shape, else
 * SPLIT.  1D plans always use the natural order.  MGWR_ERR_INVALID_ARG for
 * other values. */
enum { MGWR_LAYOUT_AUTO = -1, MGWR_LAYOUT_NATURAL = 0, MGWR_LAYOUT_SPLIT = 1 };
int mgwr_plan_set_layout(mgwr_plan* plan, int layout);

/* Learned initial guess.  Not part of the paper's method, which starts its
 * iteration from a given iterate: this network only proposes that iterate,
 * and the multigrid iteration's own float64 residual judges the proposal.
 *
 * A stack of 3x3 convolutions (zero padding, tanh after all layers but the
 * last) applied band by band to a spatial pyramid.  Input x [B][S+E][H][W]
 * float32 with S = nsignal signal channels and E = channels[0] - 1 - S extra
 * channels; a 1D grid is an image of height 1, a 2D grid has H = W; W must be
 * 2^p - 1 >= 3.  Levels n_0 = W, n_{l+1} = (n_l - 1)/2 down to 3 points; the
 * signal is split into bands band_l = c_l - P c_{l+1} (c_0 = signal,
 * c_{l+1} = full-weighting restriction of c_l, P 4-point (cubic) interpolation
 * with odd reflection at the zero boundary,
 * band_last = c_last); the convolution stack maps [band_l, the extra channels
 * sampled at the level's points, log2(1/h_l)/10] (channels[0] channels) to
 * out_l (channels[L] channels), and the output is
 * y = sum_l P^l (4 h_l^2 out_l), h_l = 2^l h with h the fine-grid spacing.
 * Inference (mgwr_net_forward and the solver's prediction) runs the
 * convolutions on the bfloat16 matrix cores: bfloat16 weights and each
 * convolution's input rounded to bfloat16 (nearest even), float32
 * accumulation, float32 bias and tanh.  Training (mgwr_net_gradient) runs
 * float32 kernels on bfloat16 weights with float32 activations, and the
 * gradient is that of this float32 forward pass; master weights, gradients
 * and Adam moments are float32.  Parameter layout: for each layer, weights
 * [c_out][c_in][3][3] then biases [c_out].  All arrays are device pointers on the stream given to
 * mgwr_net_bind; calls are asynchronous unless stated. */
typedef struct mgwr_net mgwr_net;
/* layers in [1, 16]; channels[0..layers] in [1, 1024]; nsignal in [1, channels[0] - 1]. */
int mgwr_net_create(int layers, const int* channels, int nsignal, mgwr_net** out);
int mgwr_net_param_count(const mgwr_net* net, size_t* count);
/* Device bytes for activations and optimiser state when batch*H*W <= max_bhw. */
int mgwr_net_workspace_bytes(const mgwr_net* net, long long max_bhw, size_t* bytes);
/* params_dev: caller-owned float32 master weights (mgwr_net_param_count
 * entries); workspace 256-byte aligned; resets the Adam moments and rounds
 * the bfloat16 copies (synchronises). */
int mgwr_net_bind(mgwr_net* net, float* params_dev, long long max_bhw, void* workspace_dev, size_t bytes,
                  void* stream);
/* Re-round the bfloat16 copies after the caller changed params_dev. */
int mgwr_net_sync_weights(mgwr_net* net);
/* y [B][channels[L]][H][W] = network(x); h > 0 the fine-grid spacing.  The
 * grid shape is checked (MGWR_ERR_INVALID_ARG). */
int mgwr_net_forward(mgwr_net* net, const float* x_dev, int batch, int H, int W, double h, float* y_dev);
/* Loss L = (1/B) sum_b ||y_b - t_b||^2 / ||t_b||^2 and its gradient with
 * respect to every parameter (kept in the net; copied to grad_dev if not
 * NULL); loss_host (nullable) synchronises. */
int mgwr_net_gradient(mgwr_net* net, const float* x_dev, const float* target_dev, int batch, int H, int W,
                      double h, float* grad_dev, double* loss_host);
/* Leave out every level with spacing h_l < h_min (its convolution stack is not
 * run and out_l counts as zero): bands finer than the grids a network was
 * trained on.  0 (the default) keeps all levels.  Gradients follow the same
 * rule. */
int mgwr_net_set_finest(mgwr_net* net, double h_min);
/* Adam update of params_dev with the last gradient (step counts from 1);
 * refreshes the bfloat16 copies. */
int mgwr_net_adam_step(mgwr_net* net, float lr, float beta1, float beta2, float eps, int step);
int mgwr_net_destroy(mgwr_net* net);

/* Attach a bound network to a plan for MGWR_WARM_START solves.  Its input is
 * b = f + a_{.,1} g at the `nslices` time rows rows_host[0..nslices)
 * (increasing, in [0, M)) divided by ||b||_inf, then the constant channels
 * alpha and r/10 (nsignal = nslices, channels[0] = nslices + 3); its output
 * (channels[L] = nslices) times ||b||_inf is the solution at those rows,
 * placed at t_{rows[s]+1} and interpolated piecewise linearly in the variable
 * t^alpha (the solution's behaviour near t = 0, Section 2) from the initial
 * value g (zero if NULL) at t_0, constant after the last row.  Needs
 * n = 2^p - 1 and a network bound with max_bhw >= N on the plan's device;
 * the network must outlive the attachment.  net NULL detaches. */
int mgwr_plan_set_warm_start(mgwr_plan* plan, mgwr_net* net, int nslices, const int* rows_host);

/* Learned weights as one self-describing host blob (little endian):
 *   char magic[8] = "MGWRNET1"; int32 version = 1; int32 layers L;
 *   int32 channels[L + 1]; int32 nsignal; int32 nslices; int32 rows[nslices];
 *   double h_min; int64 nparam; float32 params[nparam] (the layout of
 *   mgwr_net_param_count); uint64 checksum = 64-bit FNV-1a of every byte before it.
 * mgwr_model_describe checks a blob and reports its shape; mgwr_model_load
 * checks it against `net` (same layers, channels and nsignal), copies the
 * weights into the net's master array (synchronises the net's stream),
 * refreshes the bfloat16 copies, applies h_min (mgwr_net_set_finest) and
 * attaches the net to the plan with the blob's slice rows
 * (mgwr_plan_set_warm_start).  A missing blob (NULL or 0 bytes), a wrong
 * magic, version or size, a checksum mismatch, non-finite weights, shape
 * fields out of range, or a shape that differs from net's return
 * MGWR_ERR_MODEL and change nothing; the plan then keeps its previous
 * network, if any (solves with MGWR_WARM_START and no network fail with
 * MGWR_ERR_STATE). */
typedef struct {
  int layers;
  int channels[17];
  int nsignal, nslices;
  int rows[64];
  double h_min;
  long long nparam;
} mgwr_model_info;
int mgwr_model_describe(const void* blob_host, size_t bytes, mgwr_model_info* info);
int mgwr_model_load(mgwr_plan* plan, mgwr_net* net, const void* blob_host, size_t bytes);

/* Plan facts for tests and reports (host, no device work). */
typedef struct {
  int M, nleaf, nclusters, ndense, nrk, nzclusters, nslots, window, levels, k;
  long long stored_entries;  /* dense entries + k (|rows| + |cols|) over low-rank blocks */
  double shift0;             /* c_0 = 2 dim / h^2 */
  int layout;                /* storage the next solve uses: MGWR_LAYOUT_NATURAL or MGWR_LAYOUT_SPLIT */
  int nf64leaves;            /* leaves solved in float64 inside float32 cycles (steps within the leaf
                                differ by more than 8x: the near-origin leaves of graded meshes) */
} mgwr_plan_info;
int mgwr_plan_get_info(const mgwr_plan* plan, mgwr_plan_info* info);

/* Host copy of the mesh t[0..M] and of the initial-value weights a_{m,1}
 * (m = 1..M) used by the plan. */
int mgwr_plan_get_mesh(const mgwr_plan* plan, double* t_host, double* a1_host);

/* Expand R~ to a dense M x M row-major host array from the packed blocks the
 * device receives (tests compare it with an independent construction). */
int mgwr_plan_export_dense(const mgwr_plan* plan, double* Rt_host);

/* Bound on the polls one work item of a pipelined launch (the pipelined
 * schedule, a batch holding the plan, the coarse levels of staged cycles)
 * makes while waiting for the progress of the stage it consumes.  When a wait
 * exceeds it, the launch sets an abort flag, every waiting work item gives up,
 * and the solve returns MGWR_ERR_HIP ("... stalled"); the arrays then hold no
 * meaningful result.  The default, 4194304 polls, is seconds (a failed poll
 * sleeps about 128 cycles); smaller values make a stalled launch fail sooner.
 * 0: give up at the first wait whose producer has not finished already (used
 * to exercise this path).  A batch uses the smallest bound of its plans. */
int mgwr_plan_set_progress_limit(mgwr_plan* plan, unsigned polls);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): mgwr_solve
 * with the library's own static device array as the plan's workspace, so
 * that neither the library nor the caller allocates.  The caller passes the
 * inputs and outputs as for mgwr_solve (f_dev, g_dev, u_dev on the current
 * device) and the stream (hipStream_t or NULL).  The plan needs no binding of
 * its own; each call copies the plan's packed H-matrix into the array (one
 * host-to-device copy), solves, synchronises `stream`, and then points the
 * plan back at its own workspace if it had one (which keeps working as
 * before).  Limits: mgwr_plan_workspace_bytes(plan) must not exceed
 * MGWR_STATIC_WORKSPACE_BYTES (64 MiB: 1D n = 255, M = 512 needs 7 MiB and
 * 2D n = 63, M = 512 48 MiB; 1D n = 1023, M = 4096 needs 173 MiB), else
 * MGWR_ERR_INVALID_ARG; MGWR_WARM_START is refused (MGWR_ERR_INVALID_ARG).
 * Every call on a device shares that device's one array, which keeps the
 * last call's contents: calls that overlap on one device (other threads or
 * streams) race and must be serialised by the caller.  Each device the
 * library runs on holds its array until the process ends.  Returns what
 * mgwr_solve returns. */
#define MGWR_STATIC_WORKSPACE_BYTES (64ull << 20)
int mgwr_solve_static(mgwr_plan* plan, void* stream, const double* f_dev, const double* g_dev, double tol,
                      double* u_dev, unsigned flags, mgwr_stats* stats);

/* Release host state.  Never frees caller memory.  Safe on NULL. */
int mgwr_plan_destroy(mgwr_plan* plan);

/* Message of the last non-OK return on this thread ("" if none). */
const char* mgwr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MGWR_H */
