// Host construction of the H-matrix plan in float64 (Sections 2 and 3 of
// arXiv 1706.07632) and its packing for the gfx950 time-marching kernels.
//
//  * mesh t_m = T (m/M)^r (Section 2) or a caller-supplied mesh;
//  * L1 weights a_{m,j} = [(t_m - t_{j-1})^{1-a} - (t_m - t_j)^{1-a}] / (G(2-a) dt_j),
//    R_{m,m} = a_{m,m}, R_{m,j} = a_{m,j} - a_{m,j+1} (Section 2, entries of R);
//    differences of powers use x^p expm1(p log1p(d/x)) to avoid cancellation
//    near the origin of a graded mesh;
//  * cluster tree by index bisection (or, on request, by halving the time
//    interval of a cluster) down to `leaf` indices; block tree by the
//    recursive 2x2 split of Section 3 with Definition 3.1 on the supports
//    I_t = [t_{m1}, t_{m2}] of the Dirac tests and I_s = [t_{j1-1}, t_{j2+1}] of
//    the hats, diam(I_t) <= eta dist(I_s, I_t) (eta = 1: Definition 3.1; the
//    remark after it allows other conditions);
//  * Taylor factors about the midpoint t_c of I_t (Section 3):
//    A_{m,nu} = (t_m - t_c)^nu / G(1-a),
//    B_{j,nu} = c_nu/(1-a-nu) [(mu_{j-1}-mu_j)/dt_j - (mu_j-mu_{j+1})/dt_{j+1}],
//    mu_i = (t_c - t_i)^{1-a-nu}, c_nu = prod_{l<=nu} (1-a-l) / nu!.
//
// Device formulation of the low-rank part.  A depends only on the row
// cluster, so the low-rank contribution to the rows of a cluster theta is
// A_theta Z_theta with Z_theta = sum over admissible (theta, sigma) of
// B_{theta sigma}^T x_sigma: this is the same sum as Algorithm 3's A(B^T x)
// taken block by block, grouped by row cluster.  Every admissible sigma lies
// strictly before theta, so Z_theta is complete before theta's first row is
// needed; the kernels accumulate it while marching in time.
#include "hplan.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <sstream>

namespace mgwr {

namespace {

// (x + d)^p - x^p for x >= 0, d > 0.
double pow_diff(double x, double d, double p) {
  if (x > 0.0) return std::pow(x, p) * std::expm1(p * std::log1p(d / x));
  return std::pow(d, p);
}

// Power-of-two exponent e with 2^e close to the half-width of the row
// cluster's interval I_t.  The factors are stored as A_{m,nu} 2^{-e nu} and
// B_{j,nu} 2^{e nu}: the product is unchanged (scaling by powers of two is
// exact) while both factors stay O(1) and in float32 range even where the
// graded mesh puts I_t at t ~ 1e-20.
int cluster_scale_exp(const std::vector<double>& t, const Cluster& c) {
  double half = 0.5 * (t[c.hi] - t[c.lo + 1]);
  if (!(half > 0.0)) return 0;
  return std::ilogb(half);
}

// MFMA 16x16x4 A-operand order: value for (row, kidx) lives at [kidx/4][lane],
// lane = row + 16 * (kidx % 4).
inline size_t a_index(int row, int kidx) { return (size_t)(kidx / 4) * 64 + row + 16 * (kidx % 4); }

}  // namespace

std::string build_host_plan(const mgwr_params& p, const double* t_host, HostPlan& hp) {
  std::ostringstream err;
  if (p.dim != 1 && p.dim != 2) return "dim must be 1 or 2";
  if (p.n < 1 || ((p.n + 1) & p.n) != 0) return "n must be 2^L - 1 (L >= 1)";
  if (!(p.alpha > 0.0 && p.alpha < 1.0)) return "alpha must lie in (0, 1)";
  if (p.M < 1) return "M must be >= 1";
  if (p.k < 1 || p.k > 32) return "k must lie in [1, 32]";
  if (p.leaf < 1 || p.leaf > 16) return "leaf must lie in [1, 16]";
  if (!(p.length > 0.0)) return "length must be > 0";
  if (p.nu1 < 0 || p.nu2 < 0 || p.nu1 + p.nu2 < 1) return "nu1, nu2 >= 0 with nu1 + nu2 >= 1";
  if (p.gamma < 1 || p.gamma > 2) return "gamma must be 1 (V) or 2 (W)";
  if (p.max_cycles < 1) return "max_cycles must be >= 1";
  if (p.precision != MGWR_FP64 && p.precision != MGWR_MIXED_FP32 && p.precision != MGWR_MIXED_BF16)
    return "unknown precision";
  if (p.precision != MGWR_FP64 && (p.inner_cycles < 1 || p.inner_cycles > kMaxInnerCycles))
    return "inner_cycles must be between 1 and " + std::to_string(kMaxInnerCycles);
  if (p.schedule != MGWR_SCHED_AUTO && p.schedule != MGWR_SCHED_PIPELINED && p.schedule != MGWR_SCHED_STAGED)
    return "unknown schedule";
  if ((long long)p.M * (long long)std::pow((double)p.n, p.dim) > (1ll << 40)) return "problem too large";
  if (!(p.eta > 0.0) || !std::isfinite(p.eta)) return "eta must be a finite number > 0";
  if (p.cluster != MGWR_CLUSTER_INDEX && p.cluster != MGWR_CLUSTER_GEOMETRIC) return "unknown cluster rule";

  hp.p = p;
  const int M = p.M;
  const double alpha = p.alpha;
  const int k = p.k;

  // ---- mesh -------------------------------------------------------------
  hp.t.assign(M + 1, 0.0);
  if (t_host) {
    if (t_host[0] != 0.0) return "explicit mesh must start at t_0 = 0";
    for (int m = 0; m <= M; ++m) hp.t[m] = t_host[m];
    for (int m = 1; m <= M; ++m)
      if (!(hp.t[m] > hp.t[m - 1]) || !std::isfinite(hp.t[m])) return "explicit mesh must be strictly increasing";
  } else {
    if (!(p.T > 0.0) || !(p.r >= 1.0)) return "T > 0 and r >= 1 required";
    for (int m = 1; m <= M; ++m) hp.t[m] = p.T * std::pow((double)m / (double)M, p.r);
    hp.t[M] = p.T;
  }
  const std::vector<double>& t = hp.t;
  hp.dt.assign(M + 1, 0.0);
  for (int m = 1; m <= M; ++m) hp.dt[m] = t[m] - t[m - 1];
  const std::vector<double>& dt = hp.dt;

  const double g2 = std::tgamma(2.0 - alpha);
  auto aw = [&](int m, int j) -> double {  // a_{m,j}, 1 <= j <= m
    return pow_diff(t[m] - t[j], dt[j], 1.0 - alpha) / (g2 * dt[j]);
  };
  auto Rent = [&](int m, int j) -> double {  // R_{m,j}, 1-based
    if (j > m) return 0.0;
    if (j == m) return aw(m, m);
    return aw(m, j) - aw(m, j + 1);
  };
  hp.pk.a1.resize(M);
  for (int m = 1; m <= M; ++m) hp.pk.a1[m - 1] = aw(m, 1);

  // ---- cluster tree -----------------------------------------------------
  hp.clusters.clear();
  hp.leaf_cluster.clear();
  std::function<int(int, int)> make = [&](int lo, int hi) -> int {
    int id = (int)hp.clusters.size();
    hp.clusters.push_back(Cluster{lo, hi, {-1, -1}, -1, 0, 0, 0.5 * (t[lo + 1] + t[hi])});
    if (hi - lo > p.leaf) {
      int mid = lo + (hi - lo) / 2;
      if (p.cluster == MGWR_CLUSTER_GEOMETRIC) {
        // the levels t_{lo+1} .. t_hi at or before the midpoint of their time
        // interval form the first child (at least one level in each child)
        const double tm = 0.5 * (t[lo + 1] + t[hi]);
        int c = 0;
        while (lo + 1 + c <= hi && t[lo + 1 + c] <= tm) ++c;
        mid = std::min(std::max(lo + c, lo + 1), hi - 1);
      }
      int a = make(lo, mid);
      int b = make(mid, hi);
      hp.clusters[id].child[0] = a;
      hp.clusters[id].child[1] = b;
      hp.clusters[id].first_leaf = hp.clusters[a].first_leaf;
      hp.clusters[id].last_leaf = hp.clusters[b].last_leaf;
    } else {
      int li = (int)hp.leaf_cluster.size();
      hp.leaf_cluster.push_back(id);
      hp.clusters[id].leaf_index = li;
      hp.clusters[id].first_leaf = hp.clusters[id].last_leaf = li;
    }
    return id;
  };
  make(0, M);
  const int nleaf = (int)hp.leaf_cluster.size();
  auto is_leaf = [&](int c) { return hp.clusters[c].child[0] < 0; };

  // ---- block tree (Definition 3.1, recursive 2x2 split) ------------------
  auto admissible = [&](int rc, int cc) {
    const Cluster& R = hp.clusters[rc];
    const Cluster& C = hp.clusters[cc];
    int m1 = R.lo + 1, m2 = R.hi, j2 = C.hi;
    if (j2 + 1 > M) return false;
    double a = t[m1], d = t[j2 + 1];
    return d < a && (t[m2] - t[m1]) <= p.eta * (a - d);
  };
  hp.dense_blocks.clear();
  hp.rk_blocks.clear();
  std::function<void(int, int)> rec = [&](int rc, int cc) {
    if (hp.clusters[cc].lo >= hp.clusters[rc].hi) return;  // zero block above the diagonal
    if (admissible(rc, cc)) { hp.rk_blocks.push_back({rc, cc}); return; }
    bool rl = is_leaf(rc), cl = is_leaf(cc);
    if (rl && cl) {
      hp.dense_blocks.push_back({hp.clusters[rc].leaf_index, hp.clusters[cc].leaf_index});
      return;
    }
    int rs[2] = {rc, -1}, cs[2] = {cc, -1};
    if (!rl) { rs[0] = hp.clusters[rc].child[0]; rs[1] = hp.clusters[rc].child[1]; }
    if (!cl) { cs[0] = hp.clusters[cc].child[0]; cs[1] = hp.clusters[cc].child[1]; }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        if (rs[a] >= 0 && cs[b] >= 0) rec(rs[a], cs[b]);
  };
  rec(0, 0);

  // stored entries (dense + k(|rows| + |cols|))
  hp.stored = 0;
  for (auto& b : hp.dense_blocks) {
    const Cluster& R = hp.clusters[hp.leaf_cluster[b.first]];
    const Cluster& C = hp.clusters[hp.leaf_cluster[b.second]];
    hp.stored += (long long)(R.hi - R.lo) * (C.hi - C.lo);
  }
  for (auto& b : hp.rk_blocks)
    hp.stored += (long long)k * ((hp.clusters[b.first].hi - hp.clusters[b.first].lo) +
                                 (hp.clusters[b.second].hi - hp.clusters[b.second].lo));

  // ---- Z accumulators: live interval per row cluster, slot allocation ------
  const int ncl = (int)hp.clusters.size();
  std::vector<int> first_upd(ncl, -1);
  for (auto& b : hp.rk_blocks) {
    int f = hp.clusters[b.second].first_leaf;
    if (first_upd[b.first] < 0 || f < first_upd[b.first]) first_upd[b.first] = f;
  }
  // Interval in half steps: updates of leaf p happen at 2p+1 (after its solve),
  // reads of leaf p at 2p.  Live [2*first+1, 2*last_leaf].
  std::vector<int> order;
  for (int c = 0; c < ncl; ++c)
    if (first_upd[c] >= 0) order.push_back(c);
  hp.nzclusters = (int)order.size();
  std::sort(order.begin(), order.end(), [&](int a, int b) { return first_upd[a] < first_upd[b]; });
  hp.zslot.assign(ncl, -1);
  {
    // min-heap of (end, slot) of occupied slots; free list of slots
    std::priority_queue<std::pair<int, int>, std::vector<std::pair<int, int>>, std::greater<>> busy;
    std::vector<int> freel;
    int nslots = 0;
    for (int c : order) {
      int start = 2 * first_upd[c] + 1;
      while (!busy.empty() && busy.top().first < start) {
        freel.push_back(busy.top().second);
        busy.pop();
      }
      int s;
      if (!freel.empty()) { s = freel.back(); freel.pop_back(); }
      else s = nslots++;
      hp.zslot[c] = s;
      busy.push({2 * hp.clusters[c].last_leaf, s});
    }
    hp.nslots = nslots;
  }

  // ---- per-leaf programs ----------------------------------------------------
  PackedPlan& pk = hp.pk;
  pk.leaves.assign(nleaf, LeafDesc{});
  pk.dn_list.clear();
  pk.dense.clear();
  pk.ff_row.clear();
  pk.ffA.clear();
  pk.zu_row.clear();
  pk.zuB.clear();
  hp.ff_cluster.clear();
  hp.zu_cluster.clear();

  // dense blocks grouped by row leaf
  std::vector<std::vector<int>> dense_by_row(nleaf);
  for (auto& b : hp.dense_blocks) dense_by_row[b.first].push_back(b.second);
  hp.window = 0;
  auto add_dense_block = [&](int i, int j) -> int {
    const Cluster& Ri = hp.clusters[hp.leaf_cluster[i]];
    const Cluster& Cj = hp.clusters[hp.leaf_cluster[j]];
    int idx = (int)(pk.dense.size() / 256);
    pk.dense.resize(pk.dense.size() + 256, 0.0);
    double* blk = pk.dense.data() + (size_t)idx * 256;
    for (int r = 0; r < Ri.hi - Ri.lo; ++r)
      for (int c = 0; c < Cj.hi - Cj.lo; ++c) blk[a_index(r, c)] = -Rent(Ri.lo + r + 1, Cj.lo + c + 1);
    return idx;
  };

  // row clusters with Z that contain each leaf (ancestors or self)
  std::vector<std::vector<int>> zanc(nleaf);
  for (int c = 0; c < ncl; ++c)
    if (hp.zslot[c] >= 0)
      for (int l = hp.clusters[c].first_leaf; l <= hp.clusters[c].last_leaf; ++l) zanc[l].push_back(c);
  // low-rank blocks whose column cluster contains each leaf
  std::vector<std::vector<int>> zcol(nleaf);
  for (int b = 0; b < (int)hp.rk_blocks.size(); ++b) {
    const Cluster& C = hp.clusters[hp.rk_blocks[b].second];
    for (int l = C.first_leaf; l <= C.last_leaf; ++l) zcol[l].push_back(b);
  }

  const double ginv = 1.0 / std::tgamma(1.0 - alpha);
  std::vector<double> cnu(k);
  cnu[0] = 1.0;
  for (int nu = 1; nu < k; ++nu) cnu[nu] = cnu[nu - 1] * (1.0 - alpha - nu) / nu;

  int nchunks = 0, ntiles = 0;
  for (int i = 0; i < nleaf; ++i) {
    const Cluster& L = hp.clusters[hp.leaf_cluster[i]];
    LeafDesc& d = pk.leaves[i];
    d.lo = L.lo;
    d.sz = L.hi - L.lo;
    {
      // near the origin of a graded mesh the steps inside one leaf span
      // orders of magnitude; float32 inner cycles solve such leaves in float64
      double dmin = 1e300, dmax = 0.0;
      for (int r = 0; r < d.sz; ++r) {
        dmin = std::min(dmin, dt[d.lo + r + 1]);
        dmax = std::max(dmax, dt[d.lo + r + 1]);
      }
      d.f64solve = dmax > kF64LeafStepRatio * dmin ? 1 : 0;
    }
    // dense off-diagonal blocks, then the unshifted diagonal
    d.dn_begin = (int)pk.dn_list.size() / 2;
    std::sort(dense_by_row[i].begin(), dense_by_row[i].end());
    for (int j : dense_by_row[i]) {
      if (j == i) continue;
      hp.window = std::max(hp.window, i - j);
      int idx = add_dense_block(i, j);
      pk.dn_list.push_back(j);
      pk.dn_list.push_back(idx);
    }
    d.dn_end = (int)pk.dn_list.size() / 2;
    d.diag_off = add_dense_block(i, i);

    // far-field: stacked K rows (cluster, nu) over row clusters containing i
    d.ff_begin = nchunks;
    int K = (int)zanc[i].size() * k;
    int nch = (K + 3) / 4;
    d.ff_nchunk = nch;
    size_t base = pk.ffA.size();
    pk.ffA.resize(base + (size_t)nch * 64, 0.0);
    pk.ff_row.resize((size_t)(nchunks + nch) * 4, -1);
    hp.ff_cluster.resize((size_t)(nchunks + nch) * 4, -1);
    for (int a = 0; a < (int)zanc[i].size(); ++a) {
      int c = zanc[i][a];
      double tc = hp.clusters[c].tc;
      int ex = cluster_scale_exp(t, hp.clusters[c]);
      for (int nu = 0; nu < k; ++nu) {
        int kr = a * k + nu;
        pk.ff_row[(size_t)nchunks * 4 + kr] = hp.zslot[c] * k + nu;
        hp.ff_cluster[(size_t)nchunks * 4 + kr] = c;
        for (int r = 0; r < d.sz; ++r) {
          double dtm = t[d.lo + r + 1] - tc;
          pk.ffA[base + a_index(r, kr)] = -std::pow(std::ldexp(dtm, -ex), nu) * ginv;
        }
      }
    }
    nchunks += nch;

    // column-side updates: output rows (cluster theta, nu) for blocks (theta, sigma ni i)
    d.zu_begin = ntiles;
    int O = (int)zcol[i].size() * k;
    int nt = (O + 15) / 16;
    d.zu_ntile = nt;
    size_t zb = pk.zuB.size();
    pk.zuB.resize(zb + (size_t)nt * 256, 0.0);
    pk.zu_row.resize((size_t)(ntiles + nt) * 16, -1);
    hp.zu_cluster.resize((size_t)(ntiles + nt) * 16, -1);
    for (int bi = 0; bi < (int)zcol[i].size(); ++bi) {
      int theta = hp.rk_blocks[zcol[i][bi]].first;
      double tc = hp.clusters[theta].tc;
      int ex = cluster_scale_exp(t, hp.clusters[theta]);
      bool first = (first_upd[theta] == i);
      for (int nu = 0; nu < k; ++nu) {
        int o = bi * k + nu;
        int tile = o / 16, orow = o % 16;
        pk.zu_row[(size_t)(ntiles + tile) * 16 + orow] = (hp.zslot[theta] * k + nu) | (first ? (1 << 30) : 0);
        hp.zu_cluster[(size_t)(ntiles + tile) * 16 + orow] = theta;
        double q = 1.0 - alpha - nu;
        double* tb = pk.zuB.data() + zb + (size_t)tile * 256;
        // B_{j,nu} 2^{e nu} = c_nu/q s^{1-alpha} [pd(x_j/s, dt_j/s)/dt_j - pd(x_{j+1}/s, dt_{j+1}/s)/dt_{j+1}],
        // s = 2^e, x_i = t_c - t_i, pd(x, d) = (x + d)^q - x^q: every power has a base >= 1
        const double sfac = cnu[nu] / q * std::pow(2.0, ex * (1.0 - alpha));
        for (int r = 0; r < d.sz; ++r) {
          int j = d.lo + r + 1;  // 1-based column index
          double left = pow_diff(std::ldexp(tc - t[j], -ex), std::ldexp(dt[j], -ex), q) / dt[j];
          double right = pow_diff(std::ldexp(tc - t[j + 1], -ex), std::ldexp(dt[j + 1], -ex), q) / dt[j + 1];
          tb[a_index(orow, r)] = sfac * (left - right);
        }
      }
    }
    ntiles += nt;
  }

  // ---- levels and shifted diagonal inverses --------------------------------
  hp.levels.clear();
  for (int n = p.n; n >= 1; n = (n - 1) / 2) {
    Level lv;
    lv.n = n;
    lv.N = p.dim == 1 ? n : n * n;
    lv.h = p.length / (n + 1);
    lv.shift = 2.0 * p.dim / (lv.h * lv.h);
    hp.levels.push_back(lv);
    if (n == 1) break;
  }
  const int nlev = (int)hp.levels.size();
  pk.dinv.assign((size_t)nlev * nleaf * 256, 0.0);
  for (int l = 0; l < nlev; ++l) {
    double c = hp.levels[l].shift;
    for (int i = 0; i < nleaf; ++i) {
      const LeafDesc& d = pk.leaves[i];
      int s = d.sz;
      std::vector<double> D((size_t)s * s, 0.0), X((size_t)s * s, 0.0);
      for (int r = 0; r < s; ++r)
        for (int cc = 0; cc <= r; ++cc) D[r * s + cc] = Rent(d.lo + r + 1, d.lo + cc + 1) + (r == cc ? c : 0.0);
      // X = D^{-1} by forward substitution on the unit vectors (column by column)
      for (int e = 0; e < s; ++e) {
        for (int r = 0; r < s; ++r) {
          double acc = (r == e) ? 1.0 : 0.0;
          for (int cc = e; cc < r; ++cc) acc -= D[r * s + cc] * X[cc * s + e];
          X[r * s + e] = (r < e) ? 0.0 : acc / D[r * s + r];
        }
      }
      double* blk = pk.dinv.data() + ((size_t)l * nleaf + i) * 256;
      for (int r = 0; r < s; ++r)
        for (int cc = 0; cc < s; ++cc) blk[a_index(r, cc)] = X[r * s + cc];
    }
  }

  // ---- consistency: clusters sharing a slot have disjoint live intervals ----
  {
    std::vector<std::vector<std::pair<int, int>>> by_slot(hp.nslots);
    for (int c = 0; c < ncl; ++c)
      if (hp.zslot[c] >= 0) by_slot[hp.zslot[c]].push_back({2 * first_upd[c] + 1, 2 * hp.clusters[c].last_leaf});
    for (auto& v : by_slot) {
      std::sort(v.begin(), v.end());
      for (size_t a = 1; a < v.size(); ++a)
        if (v[a].first <= v[a - 1].second) return "internal error: overlapping accumulator slots";
    }
  }
  return "";
}

void export_dense(const HostPlan& hp, double* Rt) {
  const int M = hp.p.M;
  const int nleaf = (int)hp.pk.leaves.size();
  std::fill(Rt, Rt + (size_t)M * M, 0.0);
  const PackedPlan& pk = hp.pk;
  auto put_block = [&](int i, int j, int idx) {
    const LeafDesc& di = pk.leaves[i];
    const LeafDesc& dj = pk.leaves[j];
    const double* blk = pk.dense.data() + (size_t)idx * 256;
    for (int r = 0; r < di.sz; ++r)
      for (int c = 0; c < dj.sz; ++c) Rt[(size_t)(di.lo + r) * M + dj.lo + c] = -blk[a_index(r, c)];
  };
  for (int i = 0; i < nleaf; ++i) {
    const LeafDesc& d = pk.leaves[i];
    for (int e = d.dn_begin; e < d.dn_end; ++e) put_block(i, pk.dn_list[2 * e], pk.dn_list[2 * e + 1]);
    put_block(i, i, d.diag_off);
  }
  // low-rank part: update row (theta, nu) of column leaf j times far-field
  // row (theta, nu) of every row leaf i inside theta
  const int k = hp.p.k;
  std::vector<std::vector<std::pair<int, int>>> ffpos(nleaf);  // per leaf: (theta, ff row base)
  for (int i = 0; i < nleaf; ++i) {
    const LeafDesc& di = pk.leaves[i];
    for (int fr = 0; fr < di.ff_nchunk * 4; fr += 1) {
      int theta = hp.ff_cluster[(size_t)di.ff_begin * 4 + fr];
      if (theta >= 0 && pk.ff_row[(size_t)di.ff_begin * 4 + fr] % k == 0) ffpos[i].push_back({theta, fr});
    }
  }
  for (int j = 0; j < nleaf; ++j) {
    const LeafDesc& dj = pk.leaves[j];
    for (int zr = 0; zr < dj.zu_ntile * 16; ++zr) {
      int theta = hp.zu_cluster[(size_t)dj.zu_begin * 16 + zr];
      if (theta < 0) continue;
      int nu = (pk.zu_row[(size_t)dj.zu_begin * 16 + zr] & ((1 << 30) - 1)) % k;
      const double* tb = pk.zuB.data() + (size_t)(dj.zu_begin + zr / 16) * 256;
      const Cluster& th = hp.clusters[theta];
      for (int i = th.first_leaf; i <= th.last_leaf; ++i) {
        const LeafDesc& di = pk.leaves[i];
        int fr = -1;
        for (auto& pr : ffpos[i])
          if (pr.first == theta) fr = pr.second + nu;
        if (fr < 0) continue;
        for (int r = 0; r < di.sz; ++r) {
          double av = -pk.ffA[(size_t)(di.ff_begin + fr / 4) * 64 + r + 16 * (fr % 4)];
          for (int c = 0; c < dj.sz; ++c) Rt[(size_t)(di.lo + r) * M + dj.lo + c] += av * tb[a_index(zr % 16, c)];
        }
      }
    }
  }
}

}  // namespace mgwr
