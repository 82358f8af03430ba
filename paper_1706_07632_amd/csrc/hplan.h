// Host-side construction of the H-matrix plan (float64) and its packed
// device image.  No device code here.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mgwr.h"

namespace mgwr {

// Per-leaf program of the time-marching kernels.  All offsets index the
// packed arrays of PackedPlan.  Mirrored bit-for-bit on the device.
// A leaf whose time steps differ by more than this factor is solved in
// float64 inside float32 cycles (the near-origin leaves of graded meshes).
constexpr double kF64LeafStepRatio = 8.0;

// Mixed precision: at most this many float32 cycles per refinement step (one
// pipelined launch holds at least one whole step).
constexpr int kMaxInnerCycles = 16;

struct LeafDesc {
  int lo, sz;            // first time row (0-based) and number of rows (<= 16)
  int dn_begin, dn_end;  // dense off-diagonal blocks (j < i): pairs in dn_list
  int diag_off;          // unshifted diagonal block (negated) in `dense`, in units of 256 values
  int ff_begin, ff_nchunk;  // far-field: ff_row[4*ff_begin ...], ffA chunk index ff_begin ...
  int zu_begin, zu_ntile;   // column-side updates: zu_row[16*zu_begin ...], zuB tile zu_begin ...
  int f64solve;          // float32 cycles solve this leaf in float64 (steps within it differ by more than 8x)
};

// One multigrid level (space only; the time operator is shared).
struct Level {
  int n;         // interior points per side
  int N;         // n^dim
  double h;      // mesh width
  double shift;  // 2 dim / h^2: diagonal of the stencil, shifts the diagonal leaves
};

struct PackedPlan {
  std::vector<LeafDesc> leaves;
  std::vector<int> dn_list;     // pairs (j, block index into dense)
  std::vector<double> dense;    // [nblocks][4][64] negated blocks, MFMA A-operand order
  std::vector<double> dinv;     // [levels][nleaf][4][64] (D_ii + c_l I)^{-1}, MFMA A-operand order
  std::vector<int> ff_row;      // [nchunks*4] Z row (slot*k + nu) or -1
  std::vector<double> ffA;      // [nchunks][64] negated A values, MFMA A-operand order
  std::vector<int> zu_row;      // [ntiles*16] Z row | (first << 30), or -1
  std::vector<double> zuB;      // [ntiles][4][64] B^T values, MFMA A-operand order
  std::vector<double> a1;       // [M] initial-value weights a_{m,1}
};

struct Cluster {
  int lo, hi;         // 0-based [lo, hi)
  int child[2];       // -1 if leaf
  int leaf_index;     // >= 0 for leaves
  int first_leaf, last_leaf;
  double tc;          // midpoint of [t_{lo+1}, t_hi]
};

struct HostPlan {
  mgwr_params p;
  std::vector<double> t, dt;     // t[0..M], dt[1..M] (dt[0] unused)
  std::vector<Cluster> clusters; // clusters[0] is the root
  std::vector<int> leaf_cluster; // leaf index -> cluster id
  std::vector<std::pair<int, int>> dense_blocks;  // (leaf i, leaf j), j <= i
  std::vector<std::pair<int, int>> rk_blocks;     // (row cluster, col cluster)
  std::vector<int> zslot;        // cluster -> LDS slot (-1 if no low-rank block in its row)
  int nslots = 0, window = 0, nzclusters = 0;
  long long stored = 0;
  std::vector<Level> levels;
  PackedPlan pk;
  // host metadata for export: cluster id of each ff row / zu row (-1 padding)
  std::vector<int> ff_cluster, zu_cluster;
};

// Builds everything; returns an empty string on success, else the error.
std::string build_host_plan(const mgwr_params& p, const double* t_host, HostPlan& out);

// Dense expansion of R~ from the packed arrays (row-major M x M).
void export_dense(const HostPlan& hp, double* Rt);

}  // namespace mgwr
