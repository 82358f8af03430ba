// Launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "hplan.h"

namespace mgwr {

enum { MODE_SMOOTH = 0, MODE_RESID = 1, MODE_TRSM = 2, MODE_MATVEC = 3 };

// Arguments of the time-marching kernel.  Column p (0 <= p < ncols) of the
// launch is the spatial index q = cstride * p + coff of arrays [M][ld].
template <typename T>
struct MarchArgs {
  // packed H-matrix (device)
  const LeafDesc* leaves;
  int nleaf;
  const int* dn_list;
  const T* dense;
  const T* dinv;      // this level's shifted diagonal inverses [nleaf][256] (SMOOTH/TRSM)
  const double* dinv_hi;  // float64 copies of them, for leaves flagged f64solve in float32 cycles (or null)
  const int* ff_row;
  const T* ffA;
  const int* zu_row;
  const T* zuB;
  // float32 marches only: when set, ffA and zuB point at bfloat16 copies of
  // the far-field chunks and update tiles (2-byte entries, same indexing)
  int lr_bf16;
  // operand prefetch of a march launched on its own: 0 by mesh length, 1
  // shallow, 2 deep (the pipelined kernel always prefetches deep)
  int prefetch;
  int k, nslots, ring;
  // data
  const T* F;         // right-hand side (SMOOTH, RESID, TRSM)
  T* U;               // iterate: written (SMOOTH, TRSM) or read (RESID, MATVEC)
  T* Out;             // defect (RESID) or product (MATVEC)
  long long ld;
  // columns: storage index cstride * p + coff (natural layout), or coff + p
  // in the colour-split layout of 2D grids (split = 1: the n0 = (N + 1) / 2
  // even flat indices first, then the odd ones; neighbours are mapped)
  int ncols, cstride, coff;
  int split;
  long long n0;
  // stencil: dim 0 (none), 1 or 2; n points per side; 1/h^2
  int dim, n;
  T inv_h2;
  // Grid transfers fused into the march in 1D (null pointers: not fused).
  // Columns are q = 2p + 1, the coarse points p < nc.
  //  RESID: the first-colour full weighting of the defect is the injection
  //         Inj[m][p] = r[m][q] / 2, and the coarse iterate starts at Inj0[m][p] = 0.
  //  SMOOTH: the neighbours q -/+ 1 are read with the coarse correction Ec
  //         interpolated onto them (linear interpolation), which adds
  //         (Ec[m][p-1] + 2 Ec[m][p] + Ec[m][p+1]) / 2 to their sum.
  T* Inj;
  T* Inj0;
  const T* Ec;
  int nc;
  // RESID (float64) of a mixed-precision refinement step: the defect goes to
  // Out32 rounded to float32 (the next inner right-hand side) instead of
  // Out, and the marches launched on their own write each chain's max |r|
  // to norm_out[chunk] (null: neither).  A march launched on its own with
  // neither Out nor Out32 stores no defect, only its norms (stopping tests).
  float* Out32;
  double* norm_out;
  // SMOOTH launched on its own: when set, the change of every solved entry
  // (new value minus the iterate it replaces) goes to Dout at the same
  // index.  After a second-colour half-sweep the defect is zero on that
  // colour and, at a first-colour point, 1/h^2 times the sum of those
  // changes at its neighbours (each first-colour line was solved exactly
  // against the old values), which the zebra transfers below use.
  T* Dout;
};

// One stage of the time-pipelined kernel.  Stage kinds:
enum {
  STG_SMOOTH = 0, STG_RESID = 1, STG_RESTRICT = 2, STG_PROLONG = 3,          // float64
  STG_SMOOTH32 = 4, STG_RESID32 = 5, STG_RESTRICT32 = 6, STG_PROLONG32 = 7,  // float32 (inner cycles)
  STG_CAST = 8,     // float32 right-hand side := float64 defect, float32 iterate := 0 (leaf rows)
  STG_CORRECT = 9   // float64 iterate += float32 correction (leaf rows)
};

struct Stage {
  int kind;
  int prev;          // producer stage (index into the stage array) or -1
  int nchunks;       // work items of this stage
  int round;         // stages of one round (the same position in several instances' lists) are independent
  int task0;         // first work item (tickets are taken in stage order)
  int cnt_off;       // this stage's per-leaf counters start at counters + cnt_off
  int nleaf;
  const LeafDesc* leaves;
  MarchArgs<double> m;   // STG_SMOOTH / STG_RESID
  MarchArgs<float> mf;   // STG_SMOOTH32 / STG_RESID32
  double* norm_out;      // STG_RESID: per-work-item max |r| (or null)
  // STG_RESTRICT*: src = fine defect, dst = coarse right-hand side, zero = coarse iterate
  // STG_PROLONG*:  src = coarse correction, dst = fine iterate (updated)
  // STG_CAST: src = float64 defect, dst = float32 right-hand side, zero = float32 iterate
  // STG_CORRECT: src = float32 correction, dst = float64 iterate (updated)
  const void* src;
  void* dst;
  void* zero;
  int dim, nf, nc;
  int red_only;          // STG_RESTRICT*: the defect is held on the first colour only (see launch_restrict)
  int black_only;        // STG_PROLONG*: correct the second-colour points only (see launch_prolong)
  int split;             // STG_RESTRICT* / STG_PROLONG*: 2D grids in colour-split storage (see MarchArgs)
  // STG_RESTRICT* with zebra set: src holds the changes d of the
  // second-colour half-sweep before it (MarchArgs::Dout), and the stage
  // restricts the first-colour defect formed from them (zscale = 1/h^2 times
  // the sum of d over a point's neighbours): 1D zscale / 2 * (d[2p] +
  // d[2p + 2]); 2D the full weighting of that defect (centre and corners)
  int zebra;
  double zscale;
  long long npoints;     // STG_CAST / STG_CORRECT: points per time row
};

// Workgroup b of a launch runs on XCD b mod kXcdQueues (round-robin
// dispatch, checked on the device before per-XCD queues are used).
constexpr int kXcdQueues = 8;

struct PipeArgs {
  const Stage* stages = nullptr;
  int nstages = 0;
  int ntasks = 0;
  int* counters = nullptr;
  int* ticket = nullptr;
  int* abortf = nullptr;
  unsigned spin_limit = 0;   // polls of a progress wait before the launch gives up
  // Per-XCD work queues (xq null: one global ticket).  Workgroup b takes the
  // next task of queue b mod kXcdQueues: xq[xq_off[x] + t], t < xq_len[x].
  // Every queue lists its tasks in increasing order (stage order) and holds
  // exactly as many tasks as workgroups run on its XCD, so a workgroup waits
  // only for tasks of earlier stages, each already taken by a workgroup that
  // is running (the argument of the global ticket, per XCD).
  const int* xq = nullptr;
  int xq_off[kXcdQueues] = {};
  int xq_len[kXcdQueues] = {};
  int* xq_ticket = nullptr;
};

// One workgroup per block writes the hardware XCD id (XCC_ID) of the XCD it
// runs on to out[blockIdx.x].
hipError_t launch_xcc_probe(int* out, int blocks, hipStream_t s);

// Default bound on the polls of one progress wait (each poll sleeps about
// 128 cycles when it fails): seconds, far beyond any producer's lag.
constexpr unsigned kDefaultSpinLimit = 1u << 22;

constexpr int kStencilCols = 64;   // columns per work item of a stencil stage (leaf rows <= 16 = 4 x 4)

template <typename T> size_t march_lds_bytes(const MarchArgs<T>& a);
hipError_t launch_pipeline(const PipeArgs& pa, size_t lds, hipStream_t s);
hipError_t set_pipeline_lds_limit(size_t bytes);
hipError_t launch_fill_int(int* x, long long count, int v, hipStream_t s);
template <typename T> hipError_t launch_march(int mode, const MarchArgs<T>& a, hipStream_t s);
template <typename T> hipError_t set_march_lds_limit(size_t bytes);
// red_only: the fine defect is read at first-colour points only (the coarse
// points and, in 2D, the diagonal neighbours); the other colour's defect is
// zero after its line solves and its entries are not read.
template <typename T> hipError_t launch_restrict(const T* rf, T* fc, int dim, int nf, int M, bool red_only,
                                                 bool split, hipStream_t s);
// 2D colour-split grids, right after a second-colour half-sweep that wrote
// the changes d of its entries (MarchArgs::Dout): the first-colour defect is
// r(p) = inv_h2 * (sum of d over the neighbours of p) and the second
// colour's is zero.  launch_restrict_zebra forms the full-weighting
// restriction of that defect from d (same result as launch_restrict with
// red_only on the defect, up to rounding); launch_zebra_norm writes the
// partial maxima of |r| over the first colour to part[0 .. *nparts) (NaN if
// any is NaN; *nparts in: capacity, out: the number written), to be reduced
// by launch_maxabs_parts.
template <typename T> hipError_t launch_restrict_zebra(const T* d, T* fc, int nf, int M, T inv_h2, hipStream_t s);
hipError_t launch_zebra_norm(const double* d, int nf, int M, double inv_h2, double* part, int* nparts,
                             hipStream_t s);
// black_only: only the second-colour fine points are corrected.  A
// first-colour half-sweep that follows reads the iterate only there (its own
// lines are solved afresh), so the other corrections would be overwritten
// unread.
template <typename T> hipError_t launch_prolong(const T* ec, T* uf, int dim, int nf, int M, bool black_only,
                                                bool split, hipStream_t s);
// Colour-split storage of 2D grids (see MarchArgs): b = f + a_1 g written in
// it (gq may be null), and whole [M][N] arrays moved into or out of it.
hipError_t launch_rhs0_split(const double* f, const double* gq, const double* a1, double* b, long long M,
                             long long N, hipStream_t s);
hipError_t launch_relayout(const double* src, double* dst, long long M, long long N, bool to_split, hipStream_t s);
hipError_t launch_rhs0(const double* f, const double* gq, const double* a1, double* b, long long M, long long N,
                       hipStream_t s);
template <typename T> hipError_t launch_fill(T* x, long long count, T v, hipStream_t s);
template <typename S, typename D> hipError_t launch_cast(const S* x, D* y, long long count, hipStream_t s);
// y[i] = bfloat16 bits of (float)x[i], rounded to nearest even (finite x)
hipError_t launch_cast_bf16(const double* x, unsigned short* y, long long count, hipStream_t s);
hipError_t launch_add_correction(double* u, const float* e, long long count, hipStream_t s);
template <typename T>
hipError_t launch_maxabs(const T* x, long long count, double* part, int nparts, double* out, hipStream_t s);
// max over nparts partial maxima (NaN if any is NaN) into out[0]
hipError_t launch_maxabs_parts(const double* part, int nparts, double* out, hipStream_t s);

}  // namespace mgwr
