// CPU emulation of the time-marching kernel's arithmetic on the packed plan
// (test only).  Emulates the 64-lane MFMA 16x16x4 operand layout used by the
// kernel, runs H-matvec and H-forward-substitution over random columns, and
// compares with dense products / dense forward substitution of the plan's own
// dense expansion.  Prints "matvec_err trsm_err" (relative max errors).
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <random>
#include <vector>

#include "hplan.h"

using namespace mgwr;

// Output row held by lane group g in element r of the f64 16x16x4 instruction.
static inline int drow(int g, int r) { return g + 4 * r; }

// D[drow][c] += sum_kk A[drow][kk] B[kk][c], A[row][kk] = a[row + 16 kk], B[kk][c] = b[c + 16 kk]
static void mfma(const double* a, const double* b, double acc[64][4]) {
  for (int l = 0; l < 64; ++l) {
    int g = l >> 4, c = l & 15;
    for (int r = 0; r < 4; ++r) {
      int row = drow(g, r);
      double s = 0;
      for (int kk = 0; kk < 4; ++kk) s += a[row + 16 * kk] * b[c + 16 * kk];
      acc[l][r] += s;
    }
  }
}

int main(int argc, char** argv) {
  if (argc < 7) {
    std::fprintf(stderr, "usage: M alpha r k leaf ncols [eta [cluster]]\n");
    return 2;
  }
  mgwr_params p{};
  p.length = 1.0; p.T = 1.0; p.nu1 = 1; p.nu2 = 1; p.gamma = 1; p.max_cycles = 1;
  p.precision = MGWR_FP64; p.inner_cycles = 1;
  p.dim = 1;
  p.n = 7;
  p.M = std::atoi(argv[1]);
  p.alpha = std::atof(argv[2]);
  p.r = std::atof(argv[3]);
  p.k = std::atoi(argv[4]);
  p.leaf = std::atoi(argv[5]);
  int ncols = std::atoi(argv[6]);
  p.eta = argc > 7 ? std::atof(argv[7]) : 1.0;
  p.cluster = argc > 8 ? std::atoi(argv[8]) : MGWR_CLUSTER_INDEX;
  HostPlan hp;
  std::string e = build_host_plan(p, nullptr, hp);
  if (!e.empty()) {
    std::fprintf(stderr, "%s\n", e.c_str());
    return 1;
  }
  const int M = p.M, k = p.k;
  const PackedPlan& pk = hp.pk;
  const int nleaf = (int)pk.leaves.size();
  std::vector<double> Rt((size_t)M * M);
  export_dense(hp, Rt.data());
  const double shift = hp.levels[0].shift;

  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  std::vector<double> X((size_t)M * ncols), Y((size_t)M * ncols), B((size_t)M * ncols), S((size_t)M * ncols);
  for (auto& v : X) v = nd(rng);
  for (auto& v : B) v = nd(rng);

  // Schedule of the kernel: per leaf s, phase 1 = solve (or output) of leaf s
  // from the partial right-hand sides plus the column-side updates of leaf s-1;
  // phase 2 = partial right-hand sides of leaf s+1 split over NW waves.
  const int NW = 4;
  const int R = std::max(hp.window + 2, 3);
  for (int mode = 0; mode < 2; ++mode) {  // 0: matvec, 1: trsm
    for (int c0 = 0; c0 < ncols; c0 += 16) {
      std::vector<double> ring((size_t)R * 256, 0.0), Z((size_t)hp.nslots * k * 16, 0.0);
      std::vector<double> part((size_t)NW * 256, 0.0);  // [w][row][col]
      std::vector<double> bop(64);
      auto load_x = [&](int li) {  // known iterate of leaf li into the ring (matvec)
        const LeafDesc& d = pk.leaves[li];
        double* cur = ring.data() + (li % R) * 256;
        for (int row = 0; row < 16; ++row)
          for (int c = 0; c < 16; ++c) {
            bool ok = c0 + c < ncols && row < d.sz;
            cur[row * 16 + c] = ok ? X[(size_t)(d.lo + row) * ncols + c0 + c] : 0.0;
          }
      };
      auto partial = [&](int li) {
        const LeafDesc& d = pk.leaves[li];
        int ndoff = d.dn_end - d.dn_begin;
        int nd = ndoff + (mode == 0 ? 1 : 0);
        for (int w = 0; w < NW; ++w) {
          double acc[64][4] = {};
          if (w == 0 && mode == 1)
            for (int l = 0; l < 64; ++l)
              for (int r = 0; r < 4; ++r) {
                int row = drow(l >> 4, r), col = c0 + (l & 15);
                acc[l][r] = (col < ncols && row < d.sz) ? B[(size_t)(d.lo + row) * ncols + col] : 0.0;
              }
          for (int e = w; e < nd; e += NW) {
            int j;
            const double* D;
            if (e < ndoff) { j = pk.dn_list[2 * (d.dn_begin + e)]; D = pk.dense.data() + (size_t)pk.dn_list[2 * (d.dn_begin + e) + 1] * 256; }
            else { j = li; D = pk.dense.data() + (size_t)d.diag_off * 256; }
            const double* xj = ring.data() + (j % R) * 256;
            for (int kc = 0; kc < 4; ++kc) {
              for (int l = 0; l < 64; ++l) bop[l] = xj[(4 * kc + (l >> 4)) * 16 + (l & 15)];
              mfma(D + kc * 64, bop.data(), acc);
            }
          }
          for (int ch = w; ch < d.ff_nchunk; ch += NW) {
            for (int l = 0; l < 64; ++l) {
              int zr = pk.ff_row[(size_t)(d.ff_begin + ch) * 4 + (l >> 4)];
              bop[l] = zr >= 0 ? Z[(size_t)zr * 16 + (l & 15)] : 0.0;
            }
            mfma(pk.ffA.data() + (size_t)(d.ff_begin + ch) * 64, bop.data(), acc);
          }
          for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) part[(size_t)w * 256 + drow(l >> 4, r) * 16 + (l & 15)] = acc[l][r];
        }
      };
      auto zupdate = [&](int li) {
        const LeafDesc& d = pk.leaves[li];
        const double* xs = ring.data() + (li % R) * 256;
        for (int tt = 0; tt < d.zu_ntile; ++tt) {
          double z[64][4];
          int zr[64][4];
          for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
              zr[l][r] = pk.zu_row[(size_t)(d.zu_begin + tt) * 16 + drow(l >> 4, r)];
              int v = zr[l][r];
              z[l][r] = (v >= 0 && !(v & (1 << 30))) ? Z[(size_t)(v & ((1 << 30) - 1)) * 16 + (l & 15)] : 0.0;
            }
          const double* Bt = pk.zuB.data() + (size_t)(d.zu_begin + tt) * 256;
          for (int kc = 0; kc < 4; ++kc) {
            for (int l = 0; l < 64; ++l) bop[l] = xs[(4 * kc + (l >> 4)) * 16 + (l & 15)];
            mfma(Bt + kc * 64, bop.data(), z);
          }
          for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r)
              if (zr[l][r] >= 0) Z[(size_t)(zr[l][r] & ((1 << 30) - 1)) * 16 + (l & 15)] = z[l][r];
        }
      };
      if (mode == 0) load_x(0);
      partial(0);
      for (int i = 0; i < nleaf; ++i) {
        const LeafDesc& d = pk.leaves[i];
        double* cur = ring.data() + (i % R) * 256;
        // phase 1: the helpers' updates of leaf i-1 read the ring before wave 0 writes slot i
        if (i >= 1) zupdate(i - 1);
        double acc[64][4];
        for (int l = 0; l < 64; ++l)
          for (int r = 0; r < 4; ++r) {
            double v = 0;
            for (int w = 0; w < NW; ++w) v += part[(size_t)w * 256 + drow(l >> 4, r) * 16 + (l & 15)];
            acc[l][r] = v;
          }
        if (mode == 1) {
          double x[64][4] = {};
          const double* Di = pk.dinv.data() + (size_t)i * 256;
          for (int kc = 0; kc < 4; ++kc) {
            // f64 layout: element kc of lane (g, c) is row g + 4 kc = B row of chunk kc
            for (int l = 0; l < 64; ++l) bop[l] = acc[l][kc];
            mfma(Di + kc * 64, bop.data(), x);
          }
          for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
              int g = l >> 4, c = l & 15, row = drow(g, r), col = c0 + c;
              bool ok = col < ncols && row < d.sz;
              if (ok) S[(size_t)(d.lo + row) * ncols + col] = x[l][r];
              cur[row * 16 + c] = ok ? x[l][r] : 0.0;
            }
        } else {
          for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) {
              int g = l >> 4, c = l & 15, row = drow(g, r), col = c0 + c;
              if (col < ncols && row < d.sz) Y[(size_t)(d.lo + row) * ncols + col] = -acc[l][r];
            }
          if (i + 1 < nleaf) load_x(i + 1);
        }
        // phase 2
        if (i + 1 < nleaf) partial(i + 1);
      }
    }
  }
  // references from the dense expansion
  double emv = 0, nmv = 0, ets = 0, nts = 0;
  for (int m = 0; m < M; ++m)
    for (int c = 0; c < ncols; ++c) {
      double s = 0;
      for (int j = 0; j <= m; ++j) s += Rt[(size_t)m * M + j] * X[(size_t)j * ncols + c];
      emv = std::fmax(emv, std::fabs(s - Y[(size_t)m * ncols + c]));
      nmv = std::fmax(nmv, std::fabs(s));
    }
  std::vector<double> Xs((size_t)M * ncols);
  for (int c = 0; c < ncols; ++c)
    for (int m = 0; m < M; ++m) {
      double s = B[(size_t)m * ncols + c];
      for (int j = 0; j < m; ++j) s -= Rt[(size_t)m * M + j] * Xs[(size_t)j * ncols + c];
      Xs[(size_t)m * ncols + c] = s / (Rt[(size_t)m * M + m] + shift);
    }
  for (size_t q = 0; q < Xs.size(); ++q) {
    ets = std::fmax(ets, std::fabs(Xs[q] - S[q]));
    nts = std::fmax(nts, std::fabs(Xs[q]));
  }
  std::printf("%.3e %.3e %d %d\n", emv / nmv, ets / nts, hp.nslots, hp.window);
  return 0;
}
