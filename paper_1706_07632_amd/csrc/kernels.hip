// gfx950 kernels of the MGWR path.
//
// march_kernel: a workgroup owns 16 spatial columns and marches through the
// time leaves of the H-matrix in order (Algorithm 4 for the
// smoother, Algorithm 3 for the defect).  Per leaf i it
//   1. forms the right-hand side of the leaf rows (stencil of the other colour
//      for the zebra line relaxation of Algorithm 2, or the defect's f - A_h u),
//   2. subtracts the dense near-diagonal blocks D_ij x_j (j < i, x_j kept in an
//      LDS ring of recent leaves),
//   3. subtracts the low-rank far field A_theta Z_theta of every row cluster
//      theta containing leaf i (Z in LDS, stacked along the MFMA K dimension),
//   4. solves with the pre-inverted shifted diagonal leaf (D_ii + c I)^{-1}
//      (smoother) or subtracts D_ii x_i (defect / product),
//   5. accumulates Z_theta += B_{theta sigma}^T x_i for every admissible block
//      whose column cluster sigma contains leaf i (16-row tiles over (theta, nu)).
// All contractions are v_mfma_*_16x16x4 with the 16 columns as the N dimension.
//
// MFMA 16x16x4 operand layout used throughout (lane l, g = l/16, c = l%16):
//   A (16 x 4):  lane l holds A[c][g]
//   B (4 x 16):  lane l holds B[g][c]
//   C/D (16x16): lane l, element r holds D[drow(g, r)][c] with
//                drow = 4g + r for the f32 instruction and g + 4r for the f64
//                instruction (measured on gfx950).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hplan.h"
#include "kernels.h"

namespace mgwr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct V4;
template <> struct V4<double> { typedef d4 type; };
template <> struct V4<float> { typedef f4 type; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int drow(int g, int r);
template <> __device__ __forceinline__ int drow<double>(int g, int r) { return g + 4 * r; }
template <> __device__ __forceinline__ int drow<float>(int g, int r) { return 4 * g + r; }

// Every pointer the kernels receive inside a struct is a global-memory
// pointer; saying so turns flat accesses (which also count against the LDS
// wait counter, so that an LDS barrier would drain them) into global ones.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ const GLOBAL_AS T* gp(const T* p) { return (const GLOBAL_AS T*)p; }
template <typename T> __device__ __forceinline__ GLOBAL_AS T* gp(T* p) { return (GLOBAL_AS T*)p; }
template <typename T> __device__ __forceinline__ T ld(const T* p) { return *gp(p); }
// Word holding entry i of a low-rank factor array.  In float32 marches of a
// plan that keeps those factors in bfloat16 (`bf16` = 1) the array holds
// 2-byte entries, two to a word, and the word holding entry i is read (two
// lanes share it); the lane's half is picked and widened where the value is
// used, so that nothing waits for the load here.  Otherwise the entry itself.
template <typename T>
__device__ __forceinline__ T ld_lr(const T* p, int bf16, long long i) {
  if constexpr (sizeof(T) == 4) return ld(p + (i >> bf16));
  else return ld(p + i);
}
// Read-only tables indexed uniformly across a wave (leaf descriptors, the
// dense-block list, stage arguments) are read through the constant address
// space, i.e. scalar loads with their own cache and shorter latency.
#define CONST_AS __attribute__((address_space(4)))
template <typename T> __device__ __forceinline__ T ldc(const T* p) { return *(const CONST_AS T*)p; }
// a struct, word by word (its copy constructor cannot read another address
// space); `uniform`: the address is the same in every lane (scalar loads)
template <typename T, bool uniform = false> __device__ __forceinline__ T ld_struct(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized struct");
  T out;
  unsigned int* dst = reinterpret_cast<unsigned int*>(&out);
  if constexpr (uniform) {
    const CONST_AS unsigned int* src = (const CONST_AS unsigned int*)p;
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
  } else {
    const GLOBAL_AS unsigned int* src = (const GLOBAL_AS unsigned int*)p;
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
  }
  return out;
}

// Loads and stores of the space-time arrays.  Inside the pipelined cycle
// kernel a stage reads rows another workgroup (possibly on another XCD) has
// just written, so those accesses are device-coherent (relaxed agent-scope
// atomics: sc1 loads/stores, no cache flushes); the hand-off order is
// established by the per-leaf progress counters below.
template <bool PIPE, typename T>
__device__ __forceinline__ T gld(const T* p) {
  if constexpr (!PIPE) {
    return *gp(p);
  } else if constexpr (sizeof(T) == 8) {
    unsigned long long v = __hip_atomic_load((const GLOBAL_AS unsigned long long*)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(T, v);
  } else {
    unsigned int v = __hip_atomic_load((const GLOBAL_AS unsigned int*)p, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(T, v);
  }
}
template <bool PIPE, typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  if constexpr (!PIPE) {
    *gp(p) = v;
  } else if constexpr (sizeof(T) == 8) {
    __hip_atomic_store((GLOBAL_AS unsigned long long*)p, __builtin_bit_cast(unsigned long long, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store((GLOBAL_AS unsigned int*)p, __builtin_bit_cast(unsigned int, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Colour-split storage of a 2D grid (see MarchArgs): storage index of flat
// index q, and back; n0 = (N + 1) / 2 even flat indices come first.
__device__ __forceinline__ long long split_index(long long q, long long n0) { return (q & 1) ? n0 + (q >> 1) : (q >> 1); }
__device__ __forceinline__ long long natural_index(long long s, long long n0) { return s < n0 ? 2 * s : 2 * (s - n0) + 1; }

// Progress hand-off between pipeline stages.  done[i] counts the work items of
// a stage that have finished (and made visible) their rows of leaf i.
struct PipeCtx {
  const int* wait;   // producer's per-leaf counters, or null
  int need;          // producer's number of work items
  int* done;         // this stage's per-leaf counters
  int* abortf;       // set when a wait exceeds its bound; every waiter then gives up
  double* norm_out;  // defect stages: max |r| of this work item, or null
  unsigned spin_limit = kDefaultSpinLimit;   // polls before a wait gives up
};

// Waits until the producer has finished leaf `leaf` (of nleaf).  `ready` is
// held by the calling wave: the last leaf known finished.  A wait that must
// read reads the counters of up to kReadAhead consecutive leaves at once (one
// round trip through the device-coherent level), so a producer running ahead
// is checked once per kReadAhead leaves.  Called by whole waves (uniform);
// returns false if the pipeline was aborted.
// Measured: 2 against 4 leaves is neutral on 1D n = 1023, M = 4096 and 2 %
// faster on 2D n = 255, M = 1024 and on batches of uneven 2D instances (1
// leaf: 3 % faster there, 1 % slower on the long 1D mesh; 8 leaves: 5 %
// slower in 2D).
constexpr int kReadAhead = 2;
__device__ bool wait_leaf(const PipeCtx& pc, int leaf, int nleaf, int& ready) {
  if (!pc.wait || leaf <= ready) return true;
  const int n = min(kReadAhead, nleaf - leaf);
  for (unsigned it = 0;; ++it) {
    int cnt[kReadAhead];
#pragma unroll
    for (int i = 0; i < kReadAhead; ++i)
      cnt[i] = i < n ? __hip_atomic_load(pc.wait + leaf + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    int k = 0;
#pragma unroll
    for (int i = 0; i < kReadAhead; ++i)
      if (k == i && i < n && cnt[i] >= pc.need) k = i + 1;
    k = __builtin_amdgcn_readfirstlane(k);
    if (k > 0) {
      ready = leaf + k - 1;
      return true;
    }
    if (__hip_atomic_load(pc.abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (it >= pc.spin_limit) {
      __hip_atomic_store(pc.abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Called by one wave after its stores of the leaf rows: wait until they are
// complete, then publish.
__device__ __forceinline__ void signal_leaf(const PipeCtx& pc, int leaf, int lane) {
  __builtin_amdgcn_s_waitcnt(0);
  if (lane == 0) __hip_atomic_fetch_add(pc.done + leaf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations, not for its global loads, which stay in flight
// across the barrier (a full __syncthreads drains them, putting their latency
// on the critical path of every leaf).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Waits for all of this wave's vector-memory operations (vmcnt 0; expcnt and
// lgkmcnt left at their maxima).  Placed where everything outstanding was
// issued at least one phase earlier: the compiler then knows those registers
// are ready and does not wait again (waits count in issue order, so a later
// wait for them would also wait for the prefetches issued after them).
__device__ __forceinline__ void vm_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

constexpr int ZFIRST = 1 << 30;
constexpr int ZMASK = (1 << 30) - 1;

// Work split inside a workgroup: NW waves share one chain of 16 columns
// ("wave k" below is the wave holding role k, see kRoleShift).
// Per time leaf s there are two phases separated by workgroup barriers:
//   phase 1: wave 0 sums the partial right-hand sides of leaf s, solves with
//            the pre-inverted shifted diagonal leaf (or forms the defect) and
//            stores the rows (critical path), then applies its (small) share
//            of the column-side updates Z += B^T x_{s-1}; waves 1 .. NW-2
//            apply theirs; the last wave (IO) forms the stencil part of leaf
//            s+1 from inputs loaded one leaf earlier, waits for the producer
//            and issues the loads of leaf s+2.
//   phase 2: waves 0 .. NW-2 build their partial right-hand sides of leaf s+1
//            (dense near-diagonal blocks and the far field, round-robin); the
//            IO wave applies its share of the updates of leaf s and adds its
//            far-field share of leaf s+1.
// The tiles of the next phase are loaded into registers while the current
// phase runs.  Every admissible column cluster ends at least one leaf before
// its row cluster starts, so the far field of leaf s+1 never needs the updates
// of leaf s, and the accumulators updated with leaf s are not those read for
// leaf s+1 (their live intervals overlap, so they hold different slots).
constexpr int NW = 4;
// Wave w of a workgroup holds role (w + kRoleShift) mod NW.  Measured on
// gfx950: with roles by wave index the pipelined launch is 2.5 % slower
// (large1d 16.4 against 16.0 ms; large2d 1.5 %); shifts 1, 2 and 3 measure
// alike, as does swapping only roles 1 and 2, while swaps that keep roles 1
// and 2 in place gain less.  (Placing roles by the HW_ID SIMD of each wave
// so that the update-heavy roles of the two workgroups on a CU never share a
// SIMD gained less than any constant shift.)
constexpr int kRoleShift = 2;
static_assert((NW & (NW - 1)) == 0, "roles rotate with a mask");

template <typename T, int MODE, bool PIPE, bool DEEP = PIPE>
__device__ __forceinline__ void march_body(const MarchArgs<T>& a, int chunk, const PipeCtx& pc,
                                           unsigned char* smem_raw, int* sh_abort) {
  typedef typename V4<T>::type v4;
  // Operands prefetched per wave, deep or shallow.  Measured: the pipelined
  // kernel (time-staggered stages, one leaf of lag) gains from the deep set;
  // a march launched on its own runs faster with the shallow set (frees 50
  // registers) up to 64 time leaves (2D n = 255: 7 % at M = 512 and 1024)
  // and slower from 128 leaves on (4 % at M = 2048), where a leaf row holds
  // more low-rank blocks whose loads the deep set hides.
  constexpr int ZPF = DEEP ? 6 : 2;   // column-update tiles (even: applied in pairs)
  constexpr int DPF = 2;              // dense blocks
  constexpr int FPF = DEEP ? 5 : 3;   // far-field chunks
  T* ring = reinterpret_cast<T*>(smem_raw);   // [R][16][16] x of recent leaves, row-major
  T* part = ring + a.ring * 256;               // [NW + 1][16][16] partial right-hand sides (slot NW:
                                               // the IO wave's, odd leaves)
  T* Z = part + (NW + 1) * 256;                // [nslots*k + 1][16]; the last row takes the writes of unused slots

  const int wave = __builtin_amdgcn_readfirstlane(((threadIdx.x >> 6) + kRoleShift) & (NW - 1));   // role
  // In the pipelined kernel the IO wave (producer wait, loads of the leaf
  // after next) issues ahead of the other workgroup's waves on its SIMD:
  // measured 1.3 % faster on 1D n = 1023, M = 4096, neutral in 2D; for
  // marches launched on their own it was 2 % slower on 2D n = 255.
  if (PIPE && wave == NW - 1) __builtin_amdgcn_s_setprio(1);
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int c = lane & 15;
  const int p = chunk * 16 + c;
  const bool colok = p < a.ncols;
  // The column's natural flat index q (grid position) and its storage index
  // qs.  Colour-split storage (2D): the even flat indices (first colour)
  // come first, qs = q / 2, then the odd ones, qs = n0 + (q - 1) / 2; column
  // p is storage index coff + p, so a half-sweep's lines are contiguous.
  long long q, qs;
  if (a.split) {
    qs = colok ? (long long)a.coff + p : 0;
    q = qs < a.n0 ? 2 * qs : 2 * (qs - a.n0) + 1;
  } else {
    q = colok ? (long long)a.cstride * p + a.coff : 0;
    qs = q;
  }

  long long nb[4] = {0, 0, 0, 0};
  bool nbok[4] = {false, false, false, false};
  // 1D smoothing with the coarse correction fused: slots 2 and 3 hold the
  // coarse values p - 1 and p + 1 (weight 1/2), pf_c the value p (weight 1)
  const bool fuse_ec = MODE == MODE_SMOOTH && a.Ec != nullptr;
  if (a.dim == 1) {
    nb[0] = q - 1; nbok[0] = colok && q >= 1;
    nb[1] = q + 1; nbok[1] = colok && q + 1 < a.n;
    if (fuse_ec) {
      nb[2] = p - 1; nbok[2] = colok && p >= 1 && p - 1 < a.nc;
      nb[3] = p + 1; nbok[3] = colok && p + 1 < a.nc;
    }
  } else if (a.dim == 2) {
    long long ix = q % a.n, iy = q / a.n;
    nb[0] = q - 1;   nbok[0] = colok && ix >= 1;
    nb[1] = q + 1;   nbok[1] = colok && ix + 1 < a.n;
    nb[2] = q - a.n; nbok[2] = colok && iy >= 1;
    nb[3] = q + a.n; nbok[3] = colok && iy + 1 < a.n;
    if (a.split) {
#pragma unroll
      for (int e = 0; e < 4; ++e) nb[e] = (nb[e] & 1) ? a.n0 + (nb[e] >> 1) : (nb[e] >> 1);
    }
  }
  const T diagc = (T)(2 * a.dim);
  // Low-rank factor operands as ld_lr() loaded them, made values of T.  Every
  // factor entry a lane reads has the lane's parity (offsets are whole chunks
  // of 64 plus the lane), so with bfloat16 factors an even lane's entry is the
  // low half of its word and an odd lane's the high half; a bfloat16 value
  // widens to float32 as the upper half of the word, the lower half zero.
  const unsigned lr_shr = (sizeof(T) == 4 && a.lr_bf16) ? (unsigned)(lane & 1) * 16u : 0u;
  const unsigned lr_shl = (sizeof(T) == 4 && a.lr_bf16) ? 16u : 0u;
  auto lr = [&](T v) -> T {
    if constexpr (sizeof(T) == 4) return __uint_as_float((__float_as_uint(v) >> lr_shr) << lr_shl);
    else return v;
  };
  constexpr bool kSolve = (MODE == MODE_SMOOTH || MODE == MODE_TRSM);
  constexpr bool kKnownX = (MODE == MODE_RESID || MODE == MODE_MATVEC);
  // Work split: wave 0 sums, solves (or forms the defect) and stores the
  // leaf's rows straight from its registers, signalling them one leaf later
  // (by then they are complete without a wait of their own).  The last wave
  // (kIO) loads the stencil inputs one leaf ahead: the inputs of leaf s + 2
  // are in flight while leaf s + 1 is solved, so no global-memory round trip
  // lies on the path from one solve to the next.
  constexpr int kIO = NW - 1;
  // waves sharing the dense blocks and the far-field products of phase 2 (the
  // IO wave only takes far-field chunks left over by them)
  constexpr int NPW = NW - 1;
  const bool pworker = wave < NPW;
  // Prefetch slots.  Far-field chunk of slot k2: workers take chunks
  // wave + k2 NPW (the first FPF NPW), the IO wave the next FPF; chunks
  // beyond FPF NW go round-robin to the workers, loaded when used.  Update
  // tile of slot k2: waves 1 .. NW-1 take tiles (wave - 1) + k2 (NW - 1)
  // (waves 1 .. NW-2 in phase 1 of the next leaf, the IO wave in phase 2 of
  // the leaf itself), wave 0 (which solves first) the next ZPF; tiles beyond
  // ZPF NW go round-robin to waves 1 .. NW-1, loaded when used.
  const int ffbase = pworker ? wave : FPF * NPW;
  const int ffstride = pworker ? NPW : 1;
  const int zbase = wave == 0 ? ZPF * (NW - 1) : wave - 1;
  const int zstride = wave == 0 ? 1 : NW - 1;
  const int nleaf = a.nleaf;
  int ready = -1;   // IO wave: last producer leaf known finished

  // ---- registers holding prefetched operands -------------------------------
  constexpr int NB = 4;                 // stencil neighbours loaded per row (2 used in 1D)
  T pf_f[4], pf_n[4][NB], pf_u[4];      // IO wave: raw stencil inputs of a later leaf's rows
  T pf_c[4];                            // fused coarse correction at the column's own coarse point
  T dpf[DPF][4];                        // dense tiles of the next phase 2
  int djj[DPF];
  T fpf[FPF];                           // far-field chunks of the next phase 2
  int fzr[FPF];
  T zpf[ZPF][4];                        // column-update tiles of this wave's next Z update
  int zpr[ZPF][4];
  T di[4];                              // wave 0: diagonal inverse of the next solve

  // dense items of leaf d: the off-diagonal blocks, then (known x) the diagonal
  auto n_dense = [&](const LeafDesc& d) { return d.dn_end - d.dn_begin + (kKnownX ? 1 : 0); };
  auto dense_item = [&](const LeafDesc& d, int li, int e, int& j) -> const T* {
    if (e < d.dn_end - d.dn_begin) {
      j = ldc(a.dn_list + 2 * (d.dn_begin + e));
      return a.dense + (long long)ldc(a.dn_list + 2 * (d.dn_begin + e) + 1) * 256;
    }
    j = li;
    return a.dense + (long long)d.diag_off * 256;
  };

  // IO wave: stencil inputs of leaf li (in the pipeline, after the producer finished it)
  auto prefetch_inputs = [&](int li) -> bool {
    if constexpr (PIPE) {
      if (!wait_leaf(pc, li, nleaf, ready)) return false;
    }
    const LeafDesc d = ld_struct<LeafDesc, true>(a.leaves + li);
    // every load is issued before any of them is used, so that they are in
    // flight together; they are consumed at the end of the next phase 2
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = drow<T>(g, r);
      const bool ok = colok && row < d.sz;
      const long long off = (long long)(d.lo + (ok ? row : 0)) * a.ld;
      pf_f[r] = (MODE != MODE_MATVEC && ok) ? gld<PIPE>(a.F + off + qs) : (T)0;
      const T* ecrow = fuse_ec ? a.Ec + (long long)(d.lo + (ok ? row : 0)) * a.nc : nullptr;
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const T* src = (fuse_ec && e >= 2) ? ecrow + nb[e] : a.U + off + nb[e];
        pf_n[r][e] = ((MODE == MODE_SMOOTH || MODE == MODE_RESID || MODE == MODE_MATVEC) && nbok[e] && ok)
                         ? gld<PIPE>(src) : (T)0;
      }
      pf_c[r] = (fuse_ec && ok && p < a.nc) ? gld<PIPE>(ecrow + p) : (T)0;
      pf_u[r] = (kKnownX && ok) ? gld<PIPE>(a.U + off + qs) : (T)0;
    }
    return true;
  };

  // Leaf descriptors read by the prefetches, kept (uniform, in scalar
  // registers) for the phase that uses the tiles: no second scalar load there.
  LeafDesc dt{}, dz{};
  // all waves: H-matrix tiles of their share of leaf li's phase 2
  auto prefetch_tiles = [&](int li) {
    const LeafDesc d = ld_struct<LeafDesc, true>(a.leaves + li);
    dt = d;
    const int nd = pworker ? n_dense(d) : 0;
#pragma unroll
    for (int k2 = 0; k2 < DPF; ++k2) {
      const int e = wave + k2 * NPW;
      if (e < nd) {
        const T* D = dense_item(d, li, e, djj[k2]);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) dpf[k2][kc] = ld(D + kc * 64 + lane);
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < FPF; ++k2) {
      const int ch = ffbase + k2 * ffstride;
      if (ch < d.ff_nchunk) {
        fpf[k2] = ld_lr(a.ffA, a.lr_bf16, (long long)(d.ff_begin + ch) * 64 + lane);
        fzr[k2] = ld(a.ff_row + (d.ff_begin + ch) * 4 + g);
      }
    }
  };

  auto prefetch_zu = [&](int li) {  // update tiles of leaf li in this wave's slots
    const LeafDesc d = ld_struct<LeafDesc, true>(a.leaves + li);
    dz = d;
#pragma unroll
    for (int k2 = 0; k2 < ZPF; ++k2) {
      const int tt = zbase + k2 * zstride;
      if (tt < d.zu_ntile) {
        const long long bt0 = (long long)(d.zu_begin + tt) * 256;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) zpf[k2][kc] = ld_lr(a.zuB, a.lr_bf16, bt0 + kc * 64 + lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) zpr[k2][r] = ld(a.zu_row + (d.zu_begin + tt) * 16 + drow<T>(g, r));
      }
    }
  };

  auto prefetch_dinv = [&](int li) {
    if constexpr (kSolve) {
      const T* Di = a.dinv + (long long)li * 256;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) di[kc] = ld(Di + kc * 64 + lane);
    }
  };
  // wave 0, SMOOTH with Dout: the iterate entries the solve of leaf li
  // replaces, in the row order of its result
  T uold[4] = {0, 0, 0, 0};
  auto prefetch_uold = [&](int li) {
    if constexpr (MODE == MODE_SMOOTH) {
      if (a.Dout) {
        const LeafDesc d = ld_struct<LeafDesc, true>(a.leaves + li);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int row = drow<T>(g, r);
          if constexpr (sizeof(T) == 4) {
            if (d.f64solve && a.dinv_hi) row = drow<double>(g, r);
          }
          const bool ok = colok && row < d.sz;
          uold[r] = ok ? gld<PIPE>(a.U + (long long)(d.lo + row) * a.ld + qs) : (T)0;
        }
      }
    }
  };

  // Partial right-hand side of leaf li from this wave's share, to pw.  The
  // IO wave writes its stencil part in phase 1 (stencil) and adds its
  // far-field share in phase 2 (products, accumulating into pw).
  // (products: after prefetch_tiles(li), whose descriptor it uses)
  auto partial = [&](int li, T* pw, bool products, bool stencil) {
    const LeafDesc& d = dt;
    v4 acc = {0, 0, 0, 0};
    const int nd = (pworker && products) ? n_dense(d) : 0;
    const int nff = products ? d.ff_nchunk : 0;
    if (!stencil && !pworker) {   // IO wave, products: nothing unless it holds far-field chunks
      if (ffbase >= nff) return;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = pw[drow<T>(g, r) * 16 + c];
    }
#pragma unroll
    for (int k2 = 0; k2 < DPF; ++k2) {
      if (wave + k2 * NPW < nd) {
        const T* xj = ring + (djj[k2] % a.ring) * 256;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) acc = mfma(dpf[k2][kc], xj[(4 * kc + g) * 16 + c], acc);
      }
    }
    for (int e = wave + DPF * NPW; e < nd; e += NPW) {   // beyond the prefetched share
      int j;
      const T* D = dense_item(d, li, e, j);
      T t[4];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) t[kc] = ld(D + kc * 64 + lane);
      const T* xj = ring + (j % a.ring) * 256;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) acc = mfma(t[kc], xj[(4 * kc + g) * 16 + c], acc);
    }
#pragma unroll
    for (int k2 = 0; k2 < FPF; ++k2) {
      if (ffbase + k2 * ffstride < nff) {
        const T zv = Z[max(fzr[k2], 0) * 16 + c];   // read unconditionally, selected below
        const T bv = fzr[k2] >= 0 ? zv : (T)0;
        acc = mfma(lr(fpf[k2]), bv, acc);
      }
    }
    for (int ch0 = FPF * NW + wave; pworker && ch0 < nff; ch0 += FPF * NPW) {
      T av[FPF], bv[FPF];
#pragma unroll
      for (int b = 0; b < FPF; ++b) {
        const int ch = min(ch0 + b * NPW, nff - 1);
        av[b] = ld_lr(a.ffA, a.lr_bf16, (long long)(d.ff_begin + ch) * 64 + lane);
        const int zr = ld(a.ff_row + (d.ff_begin + ch) * 4 + g);
        const T zv = Z[max(zr, 0) * 16 + c];
        bv[b] = (zr >= 0 && ch0 + b * NPW < nff) ? zv : (T)0;
      }
#pragma unroll
      for (int b = 0; b < FPF; ++b)
        if (ch0 + b * NPW < nff) acc = mfma(lr(av[b]), bv[b], acc);
    }
    if (stencil) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T sn = pf_n[r][0] + pf_n[r][1];
        if constexpr (MODE == MODE_SMOOTH) {
          sn += (fuse_ec ? (T)0.5 : (T)1) * (pf_n[r][2] + pf_n[r][3]) + pf_c[r];
        } else {
          sn += pf_n[r][2] + pf_n[r][3];
        }
        T v;
        if constexpr (MODE == MODE_SMOOTH) v = pf_f[r] + a.inv_h2 * sn;
        else if constexpr (MODE == MODE_RESID) v = pf_f[r] - a.inv_h2 * (diagc * pf_u[r] - sn);
        else if constexpr (MODE == MODE_TRSM) v = pf_f[r];
        else v = a.dim > 0 ? -a.inv_h2 * (diagc * pf_u[r] - sn) : (T)0;   // MATVEC: the stencil part of A u
        acc[r] += v;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) pw[drow<T>(g, r) * 16 + c] = acc[r];
  };
  auto ioslot = [&](int li) { return part + ((li & 1) ? NW : kIO) * 256; };

  // phase 1: Z += B^T x for the update tiles of leaf li owned by this wave
  // (after prefetch_zu(li), whose descriptor it uses)
  auto zupdate = [&](int li) {
    const LeafDesc& d = dz;
    if (zbase >= d.zu_ntile) return;
    const T* xs = ring + (li % a.ring) * 256;
    T xb[4];   // the x operand, read once (the Z stores below may not move it)
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) xb[kc] = xs[(4 * kc + g) * 16 + c];
    // Branch-free accumulator access: the rows of unused tile rows (zr < 0)
    // read row 0, which is selected away, and write the sink row after the
    // accumulators, so the reads of a tile issue together instead of one
    // divergent branch each (measured 1.7 % on 2D n = 255, M = 1024).
    const int sink = a.nslots * a.k;
    auto zrow = [&](int zr) { return zr >= 0 ? (zr & ZMASK) : 0; };
    auto zdst = [&](int zr) { return zr >= 0 ? (zr & ZMASK) : sink; };
    auto apply = [&](const T* bt, const int* zr) {
      v4 z;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T zv = Z[zrow(zr[r]) * 16 + c];
        z[r] = (zr[r] >= 0 && !(zr[r] & ZFIRST)) ? zv : (T)0;
      }
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) z = mfma(lr(bt[kc]), xb[kc], z);
#pragma unroll
      for (int r = 0; r < 4; ++r) Z[zdst(zr[r]) * 16 + c] = z[r];
    };
    // two tiles at a time: independent accumulation chains on the MFMA pipe
    auto apply2 = [&](const T* b0, const int* r0, const T* b1, const int* r1) {
      v4 z0, z1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T v0 = Z[zrow(r0[r]) * 16 + c];
        const T v1 = Z[zrow(r1[r]) * 16 + c];
        z0[r] = (r0[r] >= 0 && !(r0[r] & ZFIRST)) ? v0 : (T)0;
        z1[r] = (r1[r] >= 0 && !(r1[r] & ZFIRST)) ? v1 : (T)0;
      }
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        z0 = mfma(lr(b0[kc]), xb[kc], z0);
        z1 = mfma(lr(b1[kc]), xb[kc], z1);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Z[zdst(r0[r]) * 16 + c] = z0[r];
        Z[zdst(r1[r]) * 16 + c] = z1[r];
      }
    };
    static_assert(ZPF % 2 == 0, "tiles go in pairs");
#pragma unroll
    for (int k2 = 0; k2 < ZPF; k2 += 2) {
      if (zbase + (k2 + 1) * zstride < d.zu_ntile) apply2(zpf[k2], zpr[k2], zpf[k2 + 1], zpr[k2 + 1]);
      else if (zbase + k2 * zstride < d.zu_ntile) apply(zpf[k2], zpr[k2]);
    }
    for (int tt = ZPF * NW + (wave - 1); wave != 0 && tt < d.zu_ntile; tt += NW - 1) {
      T bt[4];
      int zr[4];
      const long long bt0 = (long long)(d.zu_begin + tt) * 256;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) bt[kc] = ld_lr(a.zuB, a.lr_bf16, bt0 + kc * 64 + lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) zr[r] = ld(a.zu_row + (d.zu_begin + tt) * 16 + drow<T>(g, r));
      apply(bt, zr);
    }
  };

  if (nleaf <= 0) return;
  T nmax = (T)0;
  bool nbad = false;

  // The IO wave and the other waves run separate loops with the same
  // sequence of barriers, so that the registers each role carries from one
  // leaf to the next are allocated side by side rather than added up.
  if (wave == kIO) {
    // ---- IO wave ---------------------------------------------------------------
    // phase 1 of leaf s: stencil part of leaf s + 1 from the inputs loaded one
    // leaf ago, the wait for the producer and the loads of leaf s + 2;
    // phase 2: its share of the updates of leaf s (no partial sum of leaf
    // s + 1 reads those accumulators) and of the far field of leaf s + 1.
    prefetch_tiles(0);
    if (!prefetch_inputs(0)) *sh_abort = 1;
    if constexpr (kKnownX) {
#pragma unroll
      for (int r = 0; r < 4; ++r) ring[drow<T>(g, r) * 16 + c] = pf_u[r];
    }
    prefetch_zu(0);
    __syncthreads();
    if (*sh_abort) return;
    partial(0, ioslot(0), false, true);
    partial(0, ioslot(0), true, false);
    if (nleaf > 1 && !prefetch_inputs(1)) *sh_abort = 1;
    __syncthreads();
    if (*sh_abort) return;
    for (int s = 0; s < nleaf; ++s) {
      vm_drain();
      if (s + 1 < nleaf) {
        if constexpr (kKnownX) {
          T* nxt = ring + ((s + 1) % a.ring) * 256;
#pragma unroll
          for (int r = 0; r < 4; ++r) nxt[drow<T>(g, r) * 16 + c] = pf_u[r];
        }
        partial(s + 1, ioslot(s + 1), false, true);
        if (s + 2 < nleaf && !prefetch_inputs(s + 2)) *sh_abort = 1;
        prefetch_tiles(s + 1);
      }
      lds_barrier();
      if constexpr (PIPE) {
        if (*sh_abort) return;
      }
      if (s + 1 < nleaf) {
        if (s + 2 < nleaf) zupdate(s);
        partial(s + 1, ioslot(s + 1), true, false);
        prefetch_zu(s + 1);
      }
      lds_barrier();
      if constexpr (PIPE) {
        if (*sh_abort) return;
      }
    }
    return;
  }

  // ---- wave 0 and the workers ---------------------------------------------------
  prefetch_tiles(0);
  if (wave == 0) prefetch_dinv(0);
  __syncthreads();
  if (*sh_abort) return;
  // (after the barrier: in the pipelined kernel the IO wave has then waited
  // for the producer's first leaf, before which these entries may still be
  // written by an earlier stage)
  if (wave == 0) prefetch_uold(0);
  partial(0, part + wave * 256, true, false);
  __syncthreads();
  if (*sh_abort) return;

  for (int s = 0; s < nleaf; ++s) {
    const LeafDesc d = ld_struct<LeafDesc, true>(a.leaves + s);
    // ---- phase 1 --------------------------------------------------------------
    vm_drain();
    if (wave == 0) {
      if constexpr (PIPE) {
        if (s >= 1) signal_leaf(pc, s - 1, lane);   // its rows went out in the last phase 1
      }
      // The sum of the partial right-hand sides.  A solve takes it as the B
      // operand of its products: element kc of lane (g, c) sums row
      // 4 kc + g (the float64 result layout, drow<double>), so no float32
      // solve moves it between lanes; a defect keeps the result layout.
      v4 acc;
      const T* io = ioslot(s);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = kSolve ? drow<double>(g, r) : drow<T>(g, r);
        T v = io[row * 16 + c];
#pragma unroll
        for (int w = 0; w < NPW; ++w) v += part[w * 256 + row * 16 + c];
        acc[r] = v;
      }
      T* cur = ring + (s % a.ring) * 256;
      if constexpr (kSolve) {
        v4 x = {0, 0, 0, 0};
        if (sizeof(T) == 8 || !(d.f64solve && a.dinv_hi)) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) x = mfma(di[kc], acc[kc], x);
        }
        if constexpr (sizeof(T) == 4) {
          if (d.f64solve && a.dinv_hi) {
            // near-origin leaf of a graded mesh: float64 inverse and product,
            // rounded to float32 once (f64 result rows are g + 4r)
            d4 xh = {0, 0, 0, 0};
            const double* Dh = a.dinv_hi + (long long)s * 256;
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) xh = mfma(ld(Dh + kc * 64 + lane), (double)acc[kc], xh);
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = (T)xh[r];
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // float32 rows follow drow<float> except after a float64 leaf solve (drow<double>)
          int row = drow<T>(g, r);
          if constexpr (sizeof(T) == 4) {
            if (d.f64solve && a.dinv_hi) row = drow<double>(g, r);
          }
          const bool ok = colok && row < d.sz;
          cur[row * 16 + c] = ok ? x[r] : (T)0;
          if (ok) gst<PIPE>(a.U + (long long)(d.lo + row) * a.ld + qs, x[r]);
          if constexpr (MODE == MODE_SMOOTH) {
            if (ok && a.Dout) gst<PIPE>(a.Dout + (long long)(d.lo + row) * a.ld + qs, x[r] - uold[r]);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = drow<T>(g, r);
          if (colok && row < d.sz) {
            const T v = (MODE == MODE_MATVEC) ? -acc[r] : acc[r];
            if (MODE == MODE_RESID && a.Inj) {   // fused 1D restriction (first-colour defect)
              if (p < a.nc) {
                gst<PIPE>(a.Inj + (long long)(d.lo + row) * a.nc + p, (T)0.5 * v);
                gst<PIPE>(a.Inj0 + (long long)(d.lo + row) * a.nc + p, (T)0);
              }
            } else if (sizeof(T) == 8 && MODE == MODE_RESID && a.Out32) {
              // the float64 defect of a refinement step, rounded once: the
              // next float32 right-hand side
              gst<PIPE>(a.Out32 + (long long)(d.lo + row) * a.ld + qs, (float)v);
            } else if (PIPE || a.Out) {   // (a stopping-test defect keeps only its norm)
              gst<PIPE>(a.Out + (long long)(d.lo + row) * a.ld + qs, v);
            }
            if (PIPE || a.norm_out) {
              if (!(v == v) || __builtin_isinf(v)) nbad = true;
              else nmax = v > nmax ? v : (-v > nmax ? -v : nmax);
            }
          }
        }
      }
    }
    if (s + 1 < nleaf) prefetch_tiles(s + 1);
    if (s >= 1 && s + 1 < nleaf) zupdate(s - 1);
    lds_barrier();
    if constexpr (PIPE) {
      if (*sh_abort) return;
    }
    // ---- phase 2 --------------------------------------------------------------
    vm_drain();
    if (s + 1 < nleaf) {
      if (wave == 0) {
        prefetch_dinv(s + 1);
        prefetch_uold(s + 1);
      }
      prefetch_zu(s);
      partial(s + 1, part + wave * 256, true, false);
    }
    lds_barrier();
    if constexpr (PIPE) {
      if (*sh_abort) return;
    }
  }
  if constexpr (PIPE) {
    if (wave == 0) signal_leaf(pc, nleaf - 1, lane);
  }
  if constexpr (MODE == MODE_RESID) {
    double* const nout = PIPE ? pc.norm_out : a.norm_out;
    if (nout && wave == 0) {
      double m = nbad ? __builtin_nan("") : (double)nmax;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off, 64);
        m = (o != o || m != m) ? __builtin_nan("") : (o > m ? o : m);
      }
      if (lane == 0) nout[chunk] = m;
    }
  }
}

// XCDs of the chip (MI355X: 8, 32 compute units each).
constexpr int kXcds = 8;

template <typename T, int MODE, bool DEEP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void march_kernel(MarchArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh_abort;
  if (threadIdx.x == 0) sh_abort = 0;
  __syncthreads();
  PipeCtx pc{};
  // Workgroups go to the XCDs round-robin (b mod kXcds), each XCD with its
  // own L2.  Chains are handed out in contiguous bands per XCD, so the
  // chains holding a 2D line's neighbours in the rows above and below
  // (about one grid row of chains away) run on the same XCD and find those
  // rows in its L2.  The grid is rounded up to whole bands; the surplus
  // workgroups have no chain.
  const int nchunks = (a.ncols + 15) / 16;
  const int band = (nchunks + kXcds - 1) / kXcds;
  const int chunk = (int)(blockIdx.x % kXcds) * band + (int)(blockIdx.x / kXcds);
  if (chunk >= nchunks) return;
  march_body<T, MODE, false, DEEP>(a, chunk, pc, smem_raw, &sh_abort);
}

// Time leaves from which a march launched on its own takes the deep prefetch.
constexpr int kDeepPrefetchLeaves = 128;


// ---------------------------------------------------------------------------
// Time-pipelined cycles.  Every operator of a cycle of Algorithm 2 is causal
// in time (the line solves and the H-matrix product are lower triangular,
// the grid transfers act on one time level), so stage k may process leaf i as
// soon as stage k-1 has finished leaf i.  One launch runs all stages of
// several cycles; work items take tickets in stage order, so every item a
// workgroup waits for already holds a running workgroup.

static hipError_t set_dyn_lds(const void* fn, size_t bytes);

// Stencil stages: a work item covers kStencilCols columns; thread t handles
// column t % kStencilCols and rows t / kStencilCols + 4 j (j = 0..3) of each
// leaf, loading all its rows before storing, so one leaf costs about one
// memory round trip.
constexpr int kStencilRowsPerPass = 256 / kStencilCols;

// Full-weighting restriction of the rows of one leaf, and the zero start of
// the coarse iterate on those rows.
// Z2: 2D zebra restriction (12 taps on the changes d); otherwise the 9-point
// (2D) / 3-point (1D) stencil on the defect, or the 1D zebra form
template <typename T, bool Z2>
__device__ __forceinline__ void restrict_stage(const Stage& st, int chunk, const PipeCtx& pc, int* sh_abort) {
  const T* src = static_cast<const T*>(st.src);
  T* dst = static_cast<T*>(st.dst);
  T* zero = static_cast<T*>(st.zero);
  const int nf = st.nf, nc = st.nc;
  const long long Nc = st.dim == 1 ? nc : (long long)nc * nc;
  const long long Nf = st.dim == 1 ? nf : (long long)nf * nf;
  const long long Q = (long long)chunk * kStencilCols + (threadIdx.x % kStencilCols);   // storage index
  const int r0 = threadIdx.x / kStencilCols;
  const bool ok = Q < Nc;
  const bool split = st.split;
  const long long n0f = (Nf + 1) / 2;
  const long long Qn = split ? natural_index(Q, (Nc + 1) / 2) : Q;   // natural flat index
  const int lane = threadIdx.x & 63;
  // fine-grid offsets of the 9-point (2D) / 3-point (1D) weighted stencil;
  // tap t sits at a fixed index (registers, not private memory).  With a
  // first-colour defect only the first-colour taps are read.  Zebra
  // restrictions (src = the changes d of the second colour) read d at the
  // first-colour points' neighbours instead: in 2D the centre's four
  // neighbours (each counted by the centre and two corners, weight 6/16)
  // and the corners' eight outer neighbours (1/16), times 1/h^2.
  constexpr int NT = Z2 ? 12 : 9;
  const int nw = Z2 ? 12 : (st.dim == 1 ? 3 : 9);
  const bool red_only = st.red_only;
  long long off[NT];
  T wgt[NT];
  bool tap[NT];
  {
    const long long I = st.dim == 1 ? Q : Qn % nc, J = st.dim == 1 ? 0 : Qn / nc;
    const long long fx = 2 * I + 1, fy = 2 * J + 1;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if constexpr (Z2) {
        constexpr int zdy[12] = {-1, 1, 0, 0, -2, -2, 2, 2, -1, 1, -1, 1};
        constexpr int zdx[12] = {0, 0, -1, 1, -1, 1, -1, 1, -2, -2, 2, 2};
        const long long y = fy + zdy[t], x = fx + zdx[t];
        tap[t] = y >= 0 && y < nf && x >= 0 && x < nf;
        off[t] = tap[t] ? y * nf + x : 0;
        if (split) off[t] = split_index(off[t], n0f);
        wgt[t] = (T)((t < 4 ? 6.0 : 1.0) / 16.0 * st.zscale);
        continue;
      }
      if (st.dim == 1) {
        off[t] = fx - 1 + (t < 3 ? t : 0);
        wgt[t] = t == 1 ? (T)0.5 : (T)0.25;
        tap[t] = t < 3 && (!red_only || t == 1);
        if (st.zebra) {   // half the first-colour defect at fx, from the changes at fx -/+ 1
          wgt[t] = (T)(0.5 * st.zscale);
          tap[t] = t == 0 || t == 2;
        }
      } else {
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        off[t] = (fy + dy) * nf + fx + dx;
        if (split) off[t] = split_index(off[t], n0f);
        wgt[t] = (T)((dx == 0 ? 2 : 1) * (dy == 0 ? 2 : 1)) * (T)(1.0 / 16.0);
        tap[t] = !red_only || (dx == 0) == (dy == 0);   // first colour: centre and corners
      }
    }
  }
  int ready = -1;   // wave 0: last producer leaf known finished
  for (int i = 0; i < st.nleaf; ++i) {
    const LeafDesc d = ld_struct<LeafDesc, true>(st.leaves + i);
    if (threadIdx.x < 64) {
      if (!wait_leaf(pc, i, st.nleaf, ready)) *sh_abort = 1;
    }
    __syncthreads();
    if (*sh_abort) return;
    if (ok) {
      // all loads of a group of rows are issued before any is used (4 rows
      // of 3 taps in 1D, 2 rows of 9 taps in 2D)
      T v[4];
      const int rows_per_group = st.dim == 1 ? 4 : 2;
      for (int j0 = 0; j0 < 4; j0 += rows_per_group) {
        T raw[4][NT];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int row = r0 + (j0 + jj) * kStencilRowsPerPass;
          const bool rok = jj < rows_per_group && row < d.sz;
          const T* r = src + (long long)(d.lo + (rok ? row : 0)) * Nf;
#pragma unroll
          for (int t = 0; t < NT; ++t) raw[jj][t] = (rok && t < nw && tap[t]) ? gld<true>(r + off[t]) : (T)0;
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          if (jj < rows_per_group) {
            T acc = (T)0;
#pragma unroll
            for (int t = 0; t < NT; ++t)
              if (t < nw && tap[t]) acc += wgt[t] * raw[jj][t];
            v[j0 + jj] = acc;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = r0 + j * kStencilRowsPerPass;
        if (row < d.sz) {
          const long long m = d.lo + row;
          gst<true>(dst + m * Nc + Q, v[j]);
          gst<true>(zero + m * Nc + Q, (T)0);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x < 64) signal_leaf(pc, i, lane);
  }
}

// Linear / bilinear interpolation of the coarse correction, added to the
// fine iterate on the rows of one leaf.
template <typename T>
__device__ __forceinline__ void prolong_stage(const Stage& st, int chunk, const PipeCtx& pc, int* sh_abort) {
  const T* src = static_cast<const T*>(st.src);
  T* dst = static_cast<T*>(st.dst);
  const int nf = st.nf, nc = st.nc;
  const long long Nc = st.dim == 1 ? nc : (long long)nc * nc;
  const long long Nf = st.dim == 1 ? nf : (long long)nf * nf;
  // second colour only: flat indices of parity par1 (even in 1D, odd in 2D)
  const int par1 = st.dim == 1 ? 0 : 1;
  const long long Nq = st.black_only ? (Nf - par1 + 1) / 2 : Nf;
  const long long qi = (long long)chunk * kStencilCols + (threadIdx.x % kStencilCols);
  const bool split = st.split;
  const long long n0f = (Nf + 1) / 2, n0c = (Nc + 1) / 2;
  // storage index s of the point, natural flat index q
  const long long s = split ? (st.black_only ? n0f + qi : qi) : (st.black_only ? 2 * qi + par1 : qi);
  const long long q = split ? natural_index(s, n0f) : s;
  const int r0 = threadIdx.x / kStencilCols;
  const bool ok = qi < Nq;
  const int lane = threadIdx.x & 63;
  // coarse neighbours: slot t = 2 b + a of (y neighbour b, x neighbour a);
  // an odd fine index has one neighbour (slot 0 of its axis), an even one two,
  // the outer of which may lie on the boundary (cvalid false).  Fixed slots
  // keep the tables in registers.
  long long cidx[4];
  T cw[4];
  bool cvalid[4];
  {
    const long long ix = st.dim == 1 ? q : q % nf, iy = st.dim == 1 ? 1 : q / nf;
    long long cx[2], cy[2];
    T wx[2], wy[2];
    bool vx[2], vy[2];
    const bool oddx = ix & 1, oddy = iy & 1;
    cx[0] = oddx ? (ix - 1) / 2 : ix / 2 - 1;
    cx[1] = ix / 2;
    wx[0] = wx[1] = oddx ? (T)1 : (T)0.5;
    vx[0] = cx[0] >= 0 && cx[0] < nc;
    vx[1] = !oddx && cx[1] < nc;
    cy[0] = oddy ? (iy - 1) / 2 : iy / 2 - 1;
    cy[1] = iy / 2;
    wy[0] = wy[1] = oddy ? (T)1 : (T)0.5;
    vy[0] = cy[0] >= 0 && cy[0] < nc;
    vy[1] = !oddy && cy[1] < nc;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int b = t >> 1, a2 = t & 1;
      cvalid[t] = ok && vx[a2] && vy[b];
      cidx[t] = cvalid[t] ? (st.dim == 1 ? cx[a2] : cy[b] * nc + cx[a2]) : 0;
      if (split && cvalid[t]) cidx[t] = split_index(cidx[t], n0c);
      cw[t] = wx[a2] * wy[b];
    }
  }
  int ready = -1;   // wave 0: last producer leaf known finished
  for (int i = 0; i < st.nleaf; ++i) {
    const LeafDesc d = ld_struct<LeafDesc, true>(st.leaves + i);
    if (threadIdx.x < 64) {
      if (!wait_leaf(pc, i, st.nleaf, ready)) *sh_abort = 1;
    }
    __syncthreads();
    if (*sh_abort) return;
    if (ok) {
      // every load of the leaf's rows is issued before any is used
      T v[4], u0[4], raw[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = r0 + j * kStencilRowsPerPass;
        const bool rok = row < d.sz;
        const long long m = d.lo + (rok ? row : 0);
        const T* e = src + m * Nc;
#pragma unroll
        for (int t = 0; t < 4; ++t) raw[j][t] = (rok && cvalid[t]) ? gld<true>(e + cidx[t]) : (T)0;
        u0[j] = rok ? gld<true>(dst + m * Nf + s) : (T)0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        T acc = (T)0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (cvalid[t]) acc += cw[t] * raw[j][t];
        v[j] = acc;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = r0 + j * kStencilRowsPerPass;
        if (row < d.sz) gst<true>(dst + (long long)(d.lo + row) * Nf + s, u0[j] + v[j]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x < 64) signal_leaf(pc, i, lane);
  }
}

// Precision hand-over of mixed-precision refinement on the rows of one leaf:
// STG_CAST: float32 right-hand side = float64 defect, float32 iterate = 0;
// STG_CORRECT: float64 iterate += float32 correction.
__device__ __forceinline__ void pointwise_stage(const Stage& st, int chunk, const PipeCtx& pc, int* sh_abort) {
  const long long N = st.npoints;
  const long long q = (long long)chunk * kStencilCols + (threadIdx.x % kStencilCols);
  const int r0 = threadIdx.x / kStencilCols;
  const bool ok = q < N;
  const int lane = threadIdx.x & 63;
  int ready = -1;   // wave 0: last producer leaf known finished
  for (int i = 0; i < st.nleaf; ++i) {
    const LeafDesc d = ld_struct<LeafDesc, true>(st.leaves + i);
    if (threadIdx.x < 64) {
      if (!wait_leaf(pc, i, st.nleaf, ready)) *sh_abort = 1;
    }
    __syncthreads();
    if (*sh_abort) return;
    if (ok) {
      if (st.kind == STG_CAST) {
        const double* src = static_cast<const double*>(st.src);
        float* dst = static_cast<float*>(st.dst);
        float* zero = static_cast<float*>(st.zero);
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = r0 + j * kStencilRowsPerPass;
          v[j] = row < d.sz ? gld<true>(src + (long long)(d.lo + row) * N + q) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = r0 + j * kStencilRowsPerPass;
          if (row < d.sz) {
            gst<true>(dst + (long long)(d.lo + row) * N + q, (float)v[j]);
            gst<true>(zero + (long long)(d.lo + row) * N + q, 0.0f);
          }
        }
      } else {
        const float* src = static_cast<const float*>(st.src);
        double* dst = static_cast<double*>(st.dst);
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = r0 + j * kStencilRowsPerPass;
          v[j] = 0.0;
          if (row < d.sz)
            v[j] = gld<true>(dst + (long long)(d.lo + row) * N + q) +
                   (double)gld<true>(src + (long long)(d.lo + row) * N + q);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = r0 + j * kStencilRowsPerPass;
          if (row < d.sz) gst<true>(dst + (long long)(d.lo + row) * N + q, v[j]);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x < 64) signal_leaf(pc, i, lane);
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void pipeline_kernel(PipeArgs pa) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh_task;
  __shared__ int sh_abort;
  if (threadIdx.x == 0) {
    if (pa.xq) {
      const int x = (int)(blockIdx.x % kXcdQueues);
      const int t = atomicAdd(pa.xq_ticket + x, 1);
      sh_task = t < pa.xq_len[x] ? pa.xq[pa.xq_off[x] + t] : pa.ntasks;
    } else {
      sh_task = atomicAdd(pa.ticket, 1);
    }
    sh_abort = 0;
  }
  __syncthreads();
  const int task = sh_task;
  if (task >= pa.ntasks) return;
  int lo = 0, hi = pa.nstages - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pa.stages[mid].task0 <= task) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const Stage* stp = pa.stages + lo;   // global memory; the fields a march stage needs go to registers
  const int kind = ldc(&stp->kind);
  const int prev = ldc(&stp->prev);
  PipeCtx pc;
  pc.wait = prev >= 0 ? pa.counters + ldc(&pa.stages[prev].cnt_off) : nullptr;
  pc.need = prev >= 0 ? ldc(&pa.stages[prev].nchunks) : 0;
  pc.done = pa.counters + ldc(&stp->cnt_off);
  pc.abortf = pa.abortf;
  pc.spin_limit = pa.spin_limit;
  pc.norm_out = ldc(&stp->norm_out);
  const int chunk = task - ldc(&stp->task0);
  if (kind == STG_SMOOTH || kind == STG_RESID) {
    const MarchArgs<double> m = ld_struct<MarchArgs<double>, true>(&stp->m);
    if (kind == STG_SMOOTH) march_body<double, MODE_SMOOTH, true>(m, chunk, pc, smem_raw, &sh_abort);
    else march_body<double, MODE_RESID, true>(m, chunk, pc, smem_raw, &sh_abort);
    return;
  }
  if (kind == STG_SMOOTH32 || kind == STG_RESID32) {
    const MarchArgs<float> m = ld_struct<MarchArgs<float>, true>(&stp->mf);
    if (kind == STG_SMOOTH32) march_body<float, MODE_SMOOTH, true>(m, chunk, pc, smem_raw, &sh_abort);
    else march_body<float, MODE_RESID, true>(m, chunk, pc, smem_raw, &sh_abort);
    return;
  }
  if (threadIdx.x == 0) sh_abort = 0;
  __syncthreads();
  const Stage& st = *stp;
  switch (kind) {
    case STG_RESTRICT:
      if (st.zebra && st.dim == 2) restrict_stage<double, true>(st, chunk, pc, &sh_abort);
      else restrict_stage<double, false>(st, chunk, pc, &sh_abort);
      break;
    case STG_PROLONG: prolong_stage<double>(st, chunk, pc, &sh_abort); break;
    case STG_RESTRICT32:
      if (st.zebra && st.dim == 2) restrict_stage<float, true>(st, chunk, pc, &sh_abort);
      else restrict_stage<float, false>(st, chunk, pc, &sh_abort);
      break;
    case STG_PROLONG32: prolong_stage<float>(st, chunk, pc, &sh_abort); break;
    case STG_CAST:
    case STG_CORRECT: pointwise_stage(st, chunk, pc, &sh_abort); break;
    default: break;
  }
}

hipError_t launch_pipeline(const PipeArgs& pa, size_t lds, hipStream_t s) {
  if (pa.ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(pipeline_kernel, dim3(pa.ntasks), dim3(256), lds, s, pa);
  return hipGetLastError();
}

hipError_t set_pipeline_lds_limit(size_t bytes) { return set_dyn_lds((const void*)pipeline_kernel, bytes); }

// XCC_ID is hardware register 20 (bits 3:0) on gfx940 and later.
__global__ void xcc_probe_kernel(int* __restrict__ out) {
  if (threadIdx.x == 0) out[blockIdx.x] = __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & 15;
}

hipError_t launch_xcc_probe(int* out, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(xcc_probe_kernel, dim3(blocks), dim3(64), 0, s, out);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* __restrict__ x, long long count, int v) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < count;
       idx += (long long)gridDim.x * blockDim.x)
    x[idx] = v;
}

// ---------------------------------------------------------------------------
// Stencil kernels (space only, every time row independently)

// Full-weighting restriction of the defect in space only (Algorithm 2).
// Grid transfers: blockIdx.y walks the time rows, x the points of a row.
template <typename T>
__global__ void restrict_kernel(const T* __restrict__ rf, T* __restrict__ fc, int dim, int nf, int nc, long long M,
                                int red_only, int split) {
  const long long Nc = dim == 1 ? nc : (long long)nc * nc;
  const long long Nf = dim == 1 ? nf : (long long)nf * nf;
  const long long n0f = (Nf + 1) / 2, n0c = (Nc + 1) / 2;
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const T* r = rf + m * Nf;
    for (long long Q = blockIdx.x * (long long)blockDim.x + threadIdx.x; Q < Nc;
         Q += (long long)gridDim.x * blockDim.x) {
      T v;
      if (dim == 1) {
        const long long f = 2 * Q + 1;
        v = red_only ? (T)0.5 * r[f] : (T)0.25 * (r[f - 1] + (T)2 * r[f] + r[f + 1]);
      } else {
        // coarse point (I, J) is the fine point (2I+1, 2J+1); its corners share
        // its colour (the first), the edge midpoints have the other one
        const long long Qn = split ? natural_index(Q, n0c) : Q;
        const long long I = Qn % nc, J = Qn / nc;
        const long long fx = 2 * I + 1, fy = 2 * J + 1;
        auto at = [&](long long y, long long x) -> T {
          const long long qf = y * nf + x;
          return r[split ? split_index(qf, n0f) : qf];
        };
        const T edges = red_only ? (T)0 : (T)2 * (at(fy - 1, fx) + at(fy + 1, fx) + at(fy, fx - 1) + at(fy, fx + 1));
        v = (T)(1.0 / 16.0) *
            ((at(fy - 1, fx - 1) + at(fy - 1, fx + 1) + at(fy + 1, fx - 1) + at(fy + 1, fx + 1)) + edges +
             (T)4 * at(fy, fx));
      }
      fc[m * Nc + Q] = v;
    }
  }
}

// Linear interpolation of the coarse correction, added to the fine iterate.
// black_only: the second-colour points only (a first-colour half-sweep
// follows, which never reads its own lines' old values).
template <typename T>
__global__ void prolong_kernel(const T* __restrict__ ec, T* __restrict__ uf, int dim, int nf, int nc, long long M,
                               int black_only, int split) {
  const long long Nc = dim == 1 ? nc : (long long)nc * nc;
  const long long Nf = dim == 1 ? nf : (long long)nf * nf;
  const long long n0f = (Nf + 1) / 2, n0c = (Nc + 1) / 2;
  // second colour: flat indices of parity par1 (even in 1D, odd in 2D)
  const int par1 = dim == 1 ? 0 : 1;
  const long long Nq = black_only ? (Nf - par1 + 1) / 2 : Nf;
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const T* e = ec + m * Nc;
    T* u = uf + m * Nf;
    for (long long qi = blockIdx.x * (long long)blockDim.x + threadIdx.x; qi < Nq;
         qi += (long long)gridDim.x * blockDim.x) {
      // storage index s of the point, natural flat index q
      long long s, q;
      if (split) {
        s = black_only ? n0f + qi : qi;
        q = natural_index(s, n0f);
      } else {
        q = black_only ? 2 * qi + par1 : qi;
        s = q;
      }
      T v;
      if (dim == 1) {
        if (q & 1) {
          v = e[(q - 1) / 2];
        } else {
          const long long I = q / 2;  // between coarse I-1 and I
          const T lo = I >= 1 ? e[I - 1] : (T)0;
          const T hi = I < nc ? e[I] : (T)0;
          v = (T)0.5 * (lo + hi);
        }
      } else {
        const long long ix = q % nf, iy = q / nf;
        long long cx[2], cy[2];
        T wx[2], wy[2];
        int nx, ny;
        if (ix & 1) { cx[0] = (ix - 1) / 2; wx[0] = (T)1; nx = 1; }
        else { cx[0] = ix / 2 - 1; cx[1] = ix / 2; wx[0] = wx[1] = (T)0.5; nx = 2; }
        if (iy & 1) { cy[0] = (iy - 1) / 2; wy[0] = (T)1; ny = 1; }
        else { cy[0] = iy / 2 - 1; cy[1] = iy / 2; wy[0] = wy[1] = (T)0.5; ny = 2; }
        v = (T)0;
        for (int b = 0; b < ny; ++b) {
          if (cy[b] < 0 || cy[b] >= nc) continue;
          for (int a2 = 0; a2 < nx; ++a2) {
            if (cx[a2] < 0 || cx[a2] >= nc) continue;
            const long long qc = cy[b] * nc + cx[a2];
            v += wx[a2] * wy[b] * e[split ? split_index(qc, n0c) : qc];
          }
        }
      }
      u[s] += v;
    }
  }
}

// The 2D transfers in colour-split storage with 32-bit indices inside a time
// row (the generic kernels above divide 64-bit flat indices per point).
// Second-colour prolongation: the second colour's storage block of a time row
// lists the fine points with x + y odd row by row; fine rows 2P and 2P + 1
// hold nc and nc + 1 of them, nf together, so entry i = P nf + r is
// (x, y) = (2r + 1, 2P) for r < nc and (2(r - nc), 2P + 1) otherwise.  The
// first kind lies between coarse rows P - 1 and P in coarse column r, the
// second between coarse columns r - nc - 1 and r - nc in coarse row P; each
// takes the mean of the (existing) two, as the generic kernel does.
template <typename T>
__global__ __launch_bounds__(256) void prolong2_black_split_kernel(const T* __restrict__ ec, T* __restrict__ uf,
                                                                   int nf, int nc, long long M) {
  const long long Nf = (long long)nf * nf, Nc = (long long)nc * nc;
  const int n0f = (int)((Nf + 1) / 2), n0c = (int)((Nc + 1) / 2);
  const int Nq = (int)(Nf / 2);
  auto sc = [&](int qc) { return (qc & 1) ? n0c + (qc >> 1) : (qc >> 1); };
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const T* e = ec + m * Nc;
    T* u = uf + m * Nf + n0f;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < Nq; i += gridDim.x * 256) {
      const int P = i / nf, r = i - P * nf;
      T lo = (T)0, hi = (T)0;
      if (r < nc) {
        if (P >= 1) lo = e[sc((P - 1) * nc + r)];
        if (P < nc) hi = e[sc(P * nc + r)];
      } else {
        const int x = r - nc;
        if (x >= 1) lo = e[sc(P * nc + x - 1)];
        if (x < nc) hi = e[sc(P * nc + x)];
      }
      u[i] += (T)0.5 * (lo + hi);
    }
  }
}

// Restriction to coarse storage index Q (colour-split on both grids): the
// coarse point (I, J) is the fine point (2I + 1, 2J + 1), of the first colour
// as its corners; the edge midpoints have the second.
template <typename T>
__global__ __launch_bounds__(256) void restrict2_split_kernel(const T* __restrict__ rf, T* __restrict__ fc, int nf,
                                                              int nc, long long M, int red_only) {
  const long long Nf = (long long)nf * nf, Nc = (long long)nc * nc;
  const int n0f = (int)((Nf + 1) / 2), n0c = (int)((Nc + 1) / 2);
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const T* r = rf + m * Nf;
    for (int Q = blockIdx.x * 256 + threadIdx.x; Q < (int)Nc; Q += gridDim.x * 256) {
      const int Qn = Q < n0c ? 2 * Q : 2 * (Q - n0c) + 1;
      const int J = Qn / nc, I = Qn - J * nc;
      const int c0 = (2 * J + 1) * nf + 2 * I + 1;   // natural fine index of the centre (odd + odd: even)
      // first-colour fine points (even natural index q) sit at q / 2, the
      // second colour's (odd q) at n0f + q / 2
      auto f1 = [&](int q) { return r[q >> 1]; };
      auto f2 = [&](int q) { return r[n0f + (q >> 1)]; };
      const T edges = red_only ? (T)0 : (T)2 * (f2(c0 - nf) + f2(c0 + nf) + f2(c0 - 1) + f2(c0 + 1));
      fc[m * Nc + Q] = (T)(1.0 / 16.0) *
                       ((f1(c0 - nf - 1) + f1(c0 - nf + 1) + f1(c0 + nf - 1) + f1(c0 + nf + 1)) + edges +
                        (T)4 * f1(c0));
    }
  }
}

// Zebra transfers (2D, colour-split storage, right after a second-colour
// half-sweep that wrote the changes d of its entries): the first-colour
// defect at grid point (y, x) is inv_h2 times the sum of d over its in-grid
// neighbours, which all have the second colour (point (y, x) is stored at
// n0f + (y nf + x) / 2 in that colour's block).
template <typename T>
__device__ __forceinline__ T zebra_d(const T* __restrict__ d, int y, int x, int nf, int n0f) {
  return (y >= 0 && y < nf && x >= 0 && x < nf) ? d[n0f + ((y * nf + x) >> 1)] : (T)0;
}

// Full weighting of that defect to coarse storage index Q (the second
// colour's defect is zero, so only the centre and the corners count, as in
// the red_only restriction): the centre's four neighbours (edges of the 3x3
// block) and the eight outer neighbours of the corners.
template <typename T>
__global__ __launch_bounds__(256) void restrict2_zebra_kernel(const T* __restrict__ df, T* __restrict__ fc, int nf,
                                                              int nc, long long M, T inv_h2) {
  const long long Nf = (long long)nf * nf, Nc = (long long)nc * nc;
  const int n0f = (int)((Nf + 1) / 2), n0c = (int)((Nc + 1) / 2);
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const T* d = df + m * Nf;
    for (int Q = blockIdx.x * 256 + threadIdx.x; Q < (int)Nc; Q += gridDim.x * 256) {
      const int Qn = Q < n0c ? 2 * Q : 2 * (Q - n0c) + 1;
      const int J = Qn / nc, I = Qn - J * nc;
      const int y = 2 * J + 1, x = 2 * I + 1;   // the centre; corners at y -/+ 1, x -/+ 1
      // edges of the centre (always in the grid)
      const T eN = d[n0f + (((y - 1) * nf + x) >> 1)], eS = d[n0f + (((y + 1) * nf + x) >> 1)];
      const T eW = d[n0f + ((y * nf + x - 1) >> 1)], eE = d[n0f + ((y * nf + x + 1) >> 1)];
      const T rC = inv_h2 * (((eN + eS) + eW) + eE);
      const T rNW = inv_h2 * (((zebra_d(d, y - 2, x - 1, nf, n0f) + eW) + zebra_d(d, y - 1, x - 2, nf, n0f)) + eN);
      const T rNE = inv_h2 * (((zebra_d(d, y - 2, x + 1, nf, n0f) + eE) + eN) + zebra_d(d, y - 1, x + 2, nf, n0f));
      const T rSW = inv_h2 * (((eS + zebra_d(d, y + 2, x - 1, nf, n0f)) + zebra_d(d, y + 1, x - 2, nf, n0f)) + eW);
      const T rSE = inv_h2 * (((eS + zebra_d(d, y + 2, x + 1, nf, n0f)) + eE) + zebra_d(d, y + 1, x + 2, nf, n0f));
      fc[m * Nc + Q] = (T)(1.0 / 16.0) * (((rNW + rNE) + rSW + rSE) + (T)4 * rC);
    }
  }
}

// max |defect| over the first colour: block (bx, by) takes the time rows
// by, by + gridDim.y, ... and in each the first-colour points bx * 256 +
// threadIdx.x + k gridDim.x 256, and writes its maximum to
// part[by * gridDim.x + bx] (NaN propagates).  First-colour point s of a row
// is s = P nf + r: (y, x) = (2P, 2r) for r <= nc, (2P + 1, 2(r - nc) - 1)
// otherwise (nf = 2 nc + 1).
__global__ __launch_bounds__(256) void zebra_norm_kernel(const double* __restrict__ df, int nf, long long M,
                                                         double inv_h2, double* __restrict__ part) {
  const long long Nf = (long long)nf * nf;
  const int n0f = (int)((Nf + 1) / 2), nc = (nf - 1) / 2;
  double mx = 0.0;
  bool bad = false;
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const double* d = df + m * Nf;
    for (int s = blockIdx.x * 256 + threadIdx.x; s < n0f; s += gridDim.x * 256) {
      const int P = s / nf, r = s - P * nf;
      const int y = r <= nc ? 2 * P : 2 * P + 1;
      const int x = r <= nc ? 2 * r : 2 * (r - nc) - 1;
      const double v = inv_h2 * (((zebra_d(d, y - 1, x, nf, n0f) + zebra_d(d, y + 1, x, nf, n0f)) +
                                  zebra_d(d, y, x - 1, nf, n0f)) + zebra_d(d, y, x + 1, nf, n0f));
      if (!(v == v)) bad = true;
      else mx = fmax(mx, fabs(v));
    }
  }
  double w = bad ? __builtin_nan("") : mx;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(w, off, 64);
    w = (o != o || w != w) ? __builtin_nan("") : fmax(o, w);
  }
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int i = 1; i < 4; ++i) t = (sh[i] != sh[i] || t != t) ? __builtin_nan("") : fmax(t, sh[i]);
    part[blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// b = f + a_{.,1} g in colour-split storage (2D): b[m][s] from the natural
// f[m][q(s)], g[q(s)] (g may be null).
__global__ void rhs0_split_kernel(const double* __restrict__ f, const double* __restrict__ gq,
                                  const double* __restrict__ a1, double* __restrict__ b, long long M, long long N) {
  const long long n0 = (N + 1) / 2;
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const double am = gq ? a1[m] : 0.0;
    for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < N;
         s += (long long)gridDim.x * blockDim.x) {
      const long long q = natural_index(s, n0);
      b[m * N + s] = gq ? __fma_rn(am, gq[q], f[m * N + q]) : f[m * N + q];   // rounded as rhs0_kernel
    }
  }
}

// [M][N] rows between natural and colour-split storage (2D); src and dst
// must not overlap.
__global__ void relayout_kernel(const double* __restrict__ src, double* __restrict__ dst, long long M, long long N,
                                int to_split) {
  const long long n0 = (N + 1) / 2;
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    const double* a = src + m * N;
    double* b = dst + m * N;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x)
      b[i] = to_split ? a[natural_index(i, n0)] : a[split_index(i, n0)];
  }
}

__global__ void rhs0_kernel(const double* __restrict__ f, const double* __restrict__ gq, const double* __restrict__ a1,
                            double* __restrict__ b, long long M, long long N) {
  const long long total = M * N;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x)
    b[idx] = __fma_rn(a1[idx / N], gq[idx % N], f[idx]);   // one rounding, as rhs0_split_kernel
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ x, long long count, T v) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < count;
       idx += (long long)gridDim.x * blockDim.x)
    x[idx] = v;
}

template <typename S, typename D>
__global__ void cast_kernel(const S* __restrict__ x, D* __restrict__ y, long long count) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < count;
       idx += (long long)gridDim.x * blockDim.x)
    y[idx] = (D)x[idx];
}

// y = bfloat16 bits of (float)x, rounded to nearest with ties to even (the
// values converted here, low-rank factors, are finite)
__global__ void cast_bf16_kernel(const double* __restrict__ x, unsigned short* __restrict__ y, long long count) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < count;
       idx += (long long)gridDim.x * blockDim.x) {
    unsigned u = __float_as_uint((float)x[idx]);
    u += 0x7FFFu + ((u >> 16) & 1u);
    y[idx] = (unsigned short)(u >> 16);
  }
}

// u += e (float correction into the float64 iterate)
__global__ void add_correction_kernel(double* __restrict__ u, const float* __restrict__ e, long long count) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < count;
       idx += (long long)gridDim.x * blockDim.x)
    u[idx] += (double)e[idx];
}

// max |x| in two passes; non-finite values are counted separately
template <typename T>
__global__ __launch_bounds__(256) void maxabs_partial_kernel(const T* __restrict__ x, long long count,
                                                            double* __restrict__ part) {
  __shared__ double sm[256];
  __shared__ int sbad[256];
  double m = 0.0;
  int bad = 0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < count;
       idx += (long long)gridDim.x * blockDim.x) {
    const double v = (double)x[idx];
    if (!isfinite(v)) bad = 1;
    else m = fmax(m, fabs(v));
  }
  sm[threadIdx.x] = m;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sbad[0] ? __builtin_nan("") : sm[0];
}

__global__ __launch_bounds__(256) void maxabs_final_kernel(const double* __restrict__ part, int nparts,
                                                          double* __restrict__ out) {
  __shared__ double sm[256];
  __shared__ int sbad[256];
  double m = 0.0;
  int bad = 0;
  for (int idx = threadIdx.x; idx < nparts; idx += blockDim.x) {
    const double v = part[idx];
    if (v != v) bad = 1;
    else m = fmax(m, v);
  }
  sm[threadIdx.x] = m;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sbad[0] ? __builtin_nan("") : sm[0];
}

// ---------------------------------------------------------------------------
// launchers

static inline int grid_for(long long total, int block) {
  long long g = (total + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T>
size_t march_lds_bytes(const MarchArgs<T>& a) {
  const size_t zrows = (size_t)a.nslots * a.k + 1;   // accumulators and the sink row
  return ((size_t)a.ring * 256 + (size_t)(NW + 1) * 256 + zrows * 16) * sizeof(T);
}

template <typename T>
hipError_t launch_march(int mode, const MarchArgs<T>& a, hipStream_t s) {
  if (a.ncols <= 0) return hipSuccess;
  const int nchunks = (a.ncols + 15) / 16;
  dim3 grid((unsigned)(((nchunks + kXcds - 1) / kXcds) * kXcds)), block(64 * NW);
  size_t lds = march_lds_bytes(a);
  const bool deep = a.prefetch == 2 || (a.prefetch == 0 && a.nleaf >= kDeepPrefetchLeaves);
  switch (mode * 2 + (deep ? 1 : 0)) {
    case 2 * MODE_SMOOTH: hipLaunchKernelGGL((march_kernel<T, MODE_SMOOTH, false>), grid, block, lds, s, a); break;
    case 2 * MODE_SMOOTH + 1: hipLaunchKernelGGL((march_kernel<T, MODE_SMOOTH, true>), grid, block, lds, s, a); break;
    case 2 * MODE_RESID: hipLaunchKernelGGL((march_kernel<T, MODE_RESID, false>), grid, block, lds, s, a); break;
    case 2 * MODE_RESID + 1: hipLaunchKernelGGL((march_kernel<T, MODE_RESID, true>), grid, block, lds, s, a); break;
    case 2 * MODE_TRSM: hipLaunchKernelGGL((march_kernel<T, MODE_TRSM, false>), grid, block, lds, s, a); break;
    case 2 * MODE_TRSM + 1: hipLaunchKernelGGL((march_kernel<T, MODE_TRSM, true>), grid, block, lds, s, a); break;
    case 2 * MODE_MATVEC: hipLaunchKernelGGL((march_kernel<T, MODE_MATVEC, false>), grid, block, lds, s, a); break;
    case 2 * MODE_MATVEC + 1: hipLaunchKernelGGL((march_kernel<T, MODE_MATVEC, true>), grid, block, lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Raises a kernel's dynamic-LDS ceiling to `bytes` minus its static LDS.
static hipError_t set_dyn_lds(const void* fn, size_t bytes) {
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, fn);
  if (e != hipSuccess) return e;
  size_t stat = attr.sharedSizeBytes;
  if (stat >= bytes) return hipErrorInvalidValue;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bytes - stat));
}

template <typename T, bool DEEP>
static hipError_t set_march_lds_limit_depth(size_t bytes) {
  hipError_t e;
  if ((e = set_dyn_lds((const void*)march_kernel<T, MODE_SMOOTH, DEEP>, bytes)) != hipSuccess) return e;
  if ((e = set_dyn_lds((const void*)march_kernel<T, MODE_RESID, DEEP>, bytes)) != hipSuccess) return e;
  if ((e = set_dyn_lds((const void*)march_kernel<T, MODE_TRSM, DEEP>, bytes)) != hipSuccess) return e;
  return set_dyn_lds((const void*)march_kernel<T, MODE_MATVEC, DEEP>, bytes);
}

template <typename T>
hipError_t set_march_lds_limit(size_t bytes) {
  hipError_t e = set_march_lds_limit_depth<T, false>(bytes);
  return e != hipSuccess ? e : set_march_lds_limit_depth<T, true>(bytes);
}

// Launch shape of the transfer kernels: rows over y (at most 65535), a
// row's points over x (each thread covers several when the row is long).
static dim3 row_grid(long long per_row, long long M) {
  const long long gx = std::min<long long>(std::max<long long>((per_row + 255) / 256, 1), 64);
  const long long gy = std::min<long long>(std::max<long long>(M, 1), 65535);
  return dim3((unsigned)gx, (unsigned)gy);
}

template <typename T>
hipError_t launch_restrict(const T* rf, T* fc, int dim, int nf, int M, bool red_only, bool split, hipStream_t s) {
  int nc = (nf - 1) / 2;
  const long long Nc = dim == 1 ? nc : (long long)nc * nc;
  if (Nc <= 0 || M <= 0) return hipSuccess;
  if (dim == 2 && split && (long long)nf * nf < (1ll << 31)) {
    hipLaunchKernelGGL(restrict2_split_kernel<T>, row_grid(Nc, M), dim3(256), 0, s, rf, fc, nf, nc, (long long)M,
                       red_only ? 1 : 0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(restrict_kernel<T>, row_grid(Nc, M), dim3(256), 0, s, rf, fc, dim, nf, nc, (long long)M,
                     red_only ? 1 : 0, split && dim == 2 ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_zebra(const T* d, T* fc, int nf, int M, T inv_h2, hipStream_t s) {
  const int nc = (nf - 1) / 2;
  const long long Nc = (long long)nc * nc;
  if (Nc <= 0 || M <= 0) return hipSuccess;
  if ((long long)nf * nf >= (1ll << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(restrict2_zebra_kernel<T>, row_grid(Nc, M), dim3(256), 0, s, d, fc, nf, nc, (long long)M,
                     inv_h2);
  return hipGetLastError();
}

hipError_t launch_zebra_norm(const double* d, int nf, int M, double inv_h2, double* part, int* nparts,
                             hipStream_t s) {
  if (M <= 0 || !nparts || *nparts < 1) return hipErrorInvalidValue;
  if ((long long)nf * nf >= (1ll << 31)) return hipErrorInvalidValue;
  // gx blocks along a row (at most what its first colour needs), gy over the
  // rows, gx gy <= *nparts; every block has rows and writes its part
  const long long n0f = ((long long)nf * nf + 1) / 2;
  const int gx = (int)std::max<long long>(1, std::min<long long>(std::min<long long>((n0f + 255) / 256, 16), *nparts));
  const int gy = std::max(1, std::min(M, *nparts / gx));
  hipLaunchKernelGGL(zebra_norm_kernel, dim3(gx, gy), dim3(256), 0, s, d, nf, (long long)M, inv_h2, part);
  *nparts = gx * gy;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const T* ec, T* uf, int dim, int nf, int M, bool black_only, bool split, hipStream_t s) {
  int nc = (nf - 1) / 2;
  const long long Nf = dim == 1 ? nf : (long long)nf * nf;
  const long long Nq = black_only ? (Nf - (dim == 1 ? 0 : 1) + 1) / 2 : Nf;
  if (Nq <= 0 || M <= 0) return hipSuccess;
  if (dim == 2 && split && black_only && Nf < (1ll << 31)) {
    hipLaunchKernelGGL(prolong2_black_split_kernel<T>, row_grid(Nq, M), dim3(256), 0, s, ec, uf, nf, nc,
                       (long long)M);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(prolong_kernel<T>, row_grid(Nq, M), dim3(256), 0, s, ec, uf, dim, nf, nc, (long long)M,
                     black_only ? 1 : 0, split && dim == 2 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rhs0_split(const double* f, const double* gq, const double* a1, double* b, long long M,
                             long long N, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(rhs0_split_kernel, row_grid(N, M), dim3(256), 0, s, f, gq, a1, b, M, N);
  return hipGetLastError();
}

hipError_t launch_relayout(const double* src, double* dst, long long M, long long N, bool to_split, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(relayout_kernel, row_grid(N, M), dim3(256), 0, s, src, dst, M, N, to_split ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rhs0(const double* f, const double* gq, const double* a1, double* b, long long M, long long N,
                       hipStream_t s) {
  hipLaunchKernelGGL(rhs0_kernel, dim3(grid_for(M * N, 256)), dim3(256), 0, s, f, gq, a1, b, M, N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* x, long long count, T v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(count, 256)), dim3(256), 0, s, x, count, v);
  return hipGetLastError();
}

template <typename S, typename D>
hipError_t launch_cast(const S* x, D* y, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((cast_kernel<S, D>), dim3(grid_for(count, 256)), dim3(256), 0, s, x, y, count);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(const double* x, unsigned short* y, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(cast_bf16_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, x, y, count);
  return hipGetLastError();
}

hipError_t launch_add_correction(double* u, const float* e, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_correction_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, u, e, count);
  return hipGetLastError();
}

hipError_t launch_maxabs_parts(const double* part, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(maxabs_final_kernel, dim3(1), dim3(256), 0, s, part, nparts, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_maxabs(const T* x, long long count, double* part, int nparts, double* out, hipStream_t s) {
  int blocks = grid_for(count, 256);
  if (blocks > nparts) blocks = nparts;
  hipLaunchKernelGGL(maxabs_partial_kernel<T>, dim3(blocks), dim3(256), 0, s, x, count, part);
  hipLaunchKernelGGL(maxabs_final_kernel, dim3(1), dim3(256), 0, s, part, blocks, out);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* x, long long count, int v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, x, count, v);
  return hipGetLastError();
}

// explicit instantiations

template size_t march_lds_bytes<double>(const MarchArgs<double>&);
template size_t march_lds_bytes<float>(const MarchArgs<float>&);
template hipError_t launch_march<double>(int, const MarchArgs<double>&, hipStream_t);
template hipError_t launch_march<float>(int, const MarchArgs<float>&, hipStream_t);
template hipError_t set_march_lds_limit<double>(size_t);
template hipError_t set_march_lds_limit<float>(size_t);
template hipError_t launch_restrict<double>(const double*, double*, int, int, int, bool, bool, hipStream_t);
template hipError_t launch_restrict<float>(const float*, float*, int, int, int, bool, bool, hipStream_t);
template hipError_t launch_restrict_zebra<double>(const double*, double*, int, int, double, hipStream_t);
template hipError_t launch_restrict_zebra<float>(const float*, float*, int, int, float, hipStream_t);
template hipError_t launch_prolong<double>(const double*, double*, int, int, int, bool, bool, hipStream_t);
template hipError_t launch_prolong<float>(const float*, float*, int, int, int, bool, bool, hipStream_t);
template hipError_t launch_fill<double>(double*, long long, double, hipStream_t);
template hipError_t launch_fill<float>(float*, long long, float, hipStream_t);
template hipError_t launch_cast<double, float>(const double*, float*, long long, hipStream_t);
template hipError_t launch_cast<float, double>(const float*, double*, long long, hipStream_t);
template hipError_t launch_maxabs<double>(const double*, long long, double*, int, double*, hipStream_t);
template hipError_t launch_maxabs<float>(const float*, long long, double*, int, double*, hipStream_t);

}  // namespace mgwr
