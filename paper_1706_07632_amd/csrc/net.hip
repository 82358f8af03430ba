// Learned initial guess: a convolution network applied band by band to a
// spatial pyramid, with hand-written forward, backward and Adam kernels for
// the gfx950.
//
// Input x [B][S + E][H][W]: S signal channels and E extra channels (H = 1 for
// a 1D grid, else H = W; W = 2^p - 1).  The signal is split into bands over
// the grid hierarchy n_0 = W, n_{l+1} = (n_l - 1) / 2 (down to 3 points):
//   c_0 = signal,  c_{l+1} = R c_l (full weighting),
//   band_l = c_l - P c_{l+1} (P 4-point interpolation),  band_last = c_last,
// so that sum_l P^l band_l = signal.  At every level the same stack of 3x3
// convolutions (zero padding, tanh between layers, none after the last) maps
// [band_l, extra channels sampled at the level's points, log2(1/h_l)/10] to
// out_l, and the output is
//   y = sum_l P^l (4 h_l^2 out_l),   h_l = 2^l h_0,
// the factor h_l^2 carrying the scale of the inverse of a second-order
// operator on the band's grid.  The forward pass and the data gradient use
// bfloat16 copies of the convolution weights (biases stay float32) with
// float32 accumulation; master weights, gradients and Adam moments are
// float32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mgwr.h"
#include "net.h"

namespace mgwr {

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                             // round to nearest even
  return (uint16_t)(u >> 16);
}

constexpr int kCoTile = 8;   // output (forward) or input (data gradient) channels per thread
constexpr int kPx = 2;       // pixels per thread (weights read once from LDS serve both)
constexpr int kCiChunk = 64; // input channels whose weights a block stages in LDS at a time

// Forward convolution.  Grid: x = blocks of 256 x kPx pixels over B*H*W, y =
// groups of kCoTile output channels.  The block's weights (bfloat16 ->
// float32) are staged in LDS per chunk of input channels; every thread
// computes kCoTile channels of kPx pixels (p and p + 256).
// y[b][co][p] = bias[co] + sum_ci sum_k w[co][ci][k] x[b][ci][p + off(k)]
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float* __restrict__ x, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, float* __restrict__ y, int B,
                                                       int cin, int cout, int H, int W, int act) {
  __shared__ float wsh[kCoTile][kCiChunk * 9];
  const int HW = H * W;
  const long long total = (long long)B * HW;
  const int co0 = blockIdx.y * kCoTile;
  long long t[kPx];
  bool tok[kPx];
  int off[kPx][9];
  bool ok[kPx][9];
  const float* xb[kPx];
#pragma unroll
  for (int u = 0; u < kPx; ++u) {
    t[u] = (long long)blockIdx.x * (256 * kPx) + u * 256 + threadIdx.x;
    tok[u] = t[u] < total;
    const long long tt = tok[u] ? t[u] : 0;
    const int b = (int)(tt / HW), p = (int)(tt % HW);
    const int py = p / W, px = p % W;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int yy = py + k / 3 - 1, xx = px + k % 3 - 1;
      ok[u][k] = tok[u] && yy >= 0 && yy < H && xx >= 0 && xx < W;
      off[u][k] = ok[u][k] ? yy * W + xx : 0;
    }
    xb[u] = x + (long long)b * cin * HW;
  }
  float acc[kPx][kCoTile];
#pragma unroll
  for (int j = 0; j < kCoTile; ++j) {
    const float bj = co0 + j < cout ? bias[co0 + j] : 0.0f;
#pragma unroll
    for (int u = 0; u < kPx; ++u) acc[u][j] = bj;
  }
  for (int c0 = 0; c0 < cin; c0 += kCiChunk) {
    const int nc = min(kCiChunk, cin - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < kCoTile * nc * 9; e += 256) {
      const int j = e / (nc * 9), r = e % (nc * 9);
      wsh[j][r] = co0 + j < cout ? bf16_to_f32(w[((long long)(co0 + j) * cin + c0) * 9 + r]) : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int ci = 0; ci < nc; ++ci) {   // unrolled: several channels' loads in flight (small images are latency-bound)
      float xv[kPx][9];
#pragma unroll
      for (int u = 0; u < kPx; ++u)
#pragma unroll
        for (int k = 0; k < 9; ++k) xv[u][k] = ok[u][k] ? xb[u][(long long)(c0 + ci) * HW + off[u][k]] : 0.0f;
#pragma unroll
      for (int j = 0; j < kCoTile; ++j) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const float wv = wsh[j][ci * 9 + k];
#pragma unroll
          for (int u = 0; u < kPx; ++u) acc[u][j] += wv * xv[u][k];
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kPx; ++u) {
    if (!tok[u]) continue;
    const int b = (int)(t[u] / HW), p = (int)(t[u] % HW);
    float* yb = y + (long long)b * cout * HW + p;
#pragma unroll
    for (int j = 0; j < kCoTile; ++j)
      if (co0 + j < cout) yb[(long long)(co0 + j) * HW] = act ? tanhf(acc[u][j]) : acc[u][j];
  }
}

// Data gradient.  Grid: x = blocks of 256 x kPx pixels, y = groups of kCoTile
// input channels; the weights w[co][ci0..ci0+7][.] of a chunk of output
// channels are staged in LDS.
// dx[b][ci][p] = sum_co sum_k w[co][ci][k] dy[b][co][p - off(k)], times
// (1 - a^2) when the layer's input is the tanh output a of the previous layer.
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(const float* __restrict__ dy,
                                                            const uint16_t* __restrict__ w,
                                                            const float* __restrict__ a_prev, float* __restrict__ dx,
                                                            int B, int cin, int cout, int H, int W, int act_prev) {
  __shared__ float wsh[kCiChunk][kCoTile * 9];   // [co - c0][j * 9 + k]
  const int HW = H * W;
  const long long total = (long long)B * HW;
  const int ci0 = blockIdx.y * kCoTile;
  long long t[kPx];
  bool tok[kPx];
  int off[kPx][9];
  bool ok[kPx][9];
  const float* db[kPx];
#pragma unroll
  for (int u = 0; u < kPx; ++u) {
    t[u] = (long long)blockIdx.x * (256 * kPx) + u * 256 + threadIdx.x;
    tok[u] = t[u] < total;
    const long long tt = tok[u] ? t[u] : 0;
    const int b = (int)(tt / HW), p = (int)(tt % HW);
    const int py = p / W, px = p % W;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int yy = py - (k / 3 - 1), xx = px - (k % 3 - 1);
      ok[u][k] = tok[u] && yy >= 0 && yy < H && xx >= 0 && xx < W;
      off[u][k] = ok[u][k] ? yy * W + xx : 0;
    }
    db[u] = dy + (long long)b * cout * HW;
  }
  float acc[kPx][kCoTile];
#pragma unroll
  for (int u = 0; u < kPx; ++u)
#pragma unroll
    for (int j = 0; j < kCoTile; ++j) acc[u][j] = 0.0f;
  for (int c0 = 0; c0 < cout; c0 += kCiChunk) {
    const int nc = min(kCiChunk, cout - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < nc * kCoTile * 9; e += 256) {
      const int co = e / (kCoTile * 9), r = e % (kCoTile * 9), j = r / 9, k = r % 9;
      wsh[co][r] = ci0 + j < cin ? bf16_to_f32(w[((long long)(c0 + co) * cin + ci0 + j) * 9 + k]) : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int co = 0; co < nc; ++co) {
      float dv[kPx][9];
#pragma unroll
      for (int u = 0; u < kPx; ++u)
#pragma unroll
        for (int k = 0; k < 9; ++k) dv[u][k] = ok[u][k] ? db[u][(long long)(c0 + co) * HW + off[u][k]] : 0.0f;
#pragma unroll
      for (int j = 0; j < kCoTile; ++j) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const float wv = wsh[co][j * 9 + k];
#pragma unroll
          for (int u = 0; u < kPx; ++u) acc[u][j] += wv * dv[u][k];
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kPx; ++u) {
    if (!tok[u]) continue;
    const int b = (int)(t[u] / HW), p = (int)(t[u] % HW);
#pragma unroll
    for (int j = 0; j < kCoTile; ++j) {
      if (ci0 + j < cin) {
        const long long idx = ((long long)b * cin + ci0 + j) * HW + p;
        float v = acc[u][j];
        if (act_prev) {
          const float a = a_prev[idx];
          v *= 1.0f - a * a;
        }
        dx[idx] = v;
      }
    }
  }
}

constexpr int kWgCo = 4;  // output channels per block of the weight gradient

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

// Weight gradient, accumulated (+=) into dw and dbias.  One block per
// (group of kWgCo output channels, input channel):
//   dw[co][ci][k] += sum_{b,p} dy[b][co][p] x[b][ci][p + off(k)],
//   dbias[co]     += sum_{b,p} dy[b][co][p]   (blocks with ci == 0).
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const float* __restrict__ dy,
                                                              const float* __restrict__ x, float* __restrict__ dw,
                                                              float* __restrict__ dbias, int B, int cin, int cout,
                                                              int H, int W) {
  constexpr int NV = kWgCo * 10;
  __shared__ float red[4][NV];
  const int ci = blockIdx.x % cin;
  const int co0 = (blockIdx.x / cin) * kWgCo;
  const int HW = H * W;
  const long long total = (long long)B * HW;
  float acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0f;
  for (long long t = threadIdx.x; t < total; t += 256) {
    const int b = (int)(t / HW), p = (int)(t % HW);
    const int py = p / W, px = p % W;
    const float* xc = x + ((long long)b * cin + ci) * HW;
    float xv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int yy = py + k / 3 - 1, xx = px + k % 3 - 1;
      xv[k] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? xc[yy * W + xx] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kWgCo; ++j) {
      const float d = co0 + j < cout ? dy[((long long)b * cout + co0 + j) * HW + p] : 0.0f;
#pragma unroll
      for (int k = 0; k < 9; ++k) acc[j * 10 + k] += d * xv[k];
      acc[j * 10 + 9] += d;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const float s = wave_sum(acc[j]);
    if (lane == 0) red[wv][j] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int j = threadIdx.x / 10, k = threadIdx.x % 10;
    const int co = co0 + j;
    if (co < cout) {
      const float s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
      if (k < 9) dw[((long long)co * cin + ci) * 9 + k] += s;
      else if (ci == 0) dbias[co] += s;
    }
  }
}

// Grid of n points per side onto the next coarser one: coarse point i sits on
// fine point 2i + 1.  Full weighting, (1/4)[1 2 1] per dimension.
// dst [B][C][HWc] from src[b * sbs + c * HWf + ...]
__global__ void pyr_restrict_kernel(const float* __restrict__ src, long long sbs, float* __restrict__ dst, int B,
                                    int C, int nf, int two_d) {
  const int nc = (nf - 1) / 2;
  const int HWc = (two_d ? nc : 1) * nc;
  const int HWf = (two_d ? nf : 1) * nf;
  const long long total = (long long)B * C * HWc;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(idx % HWc);
    const long long bc = idx / HWc;
    const int c = (int)(bc % C), b = (int)(bc / C);
    const int i = q / nc, j = q % nc;
    const float* s = src + b * sbs + (long long)c * HWf;
    const int fj = 2 * j + 1;
    float v;
    if (two_d) {
      const int fi = 2 * i + 1;
      const float* r0 = s + (long long)(fi - 1) * nf;
      const float* r1 = r0 + nf;
      const float* r2 = r1 + nf;
      v = 0.0625f * (r0[fj - 1] + 2.0f * r0[fj] + r0[fj + 1]) + 0.125f * (r1[fj - 1] + 2.0f * r1[fj] + r1[fj + 1]) +
          0.0625f * (r2[fj - 1] + 2.0f * r2[fj] + r2[fj + 1]);
    } else {
      v = 0.25f * (s[fj - 1] + 2.0f * s[fj] + s[fj + 1]);
    }
    dst[idx] = v;
  }
}

// Interpolation P from a coarse grid (nc points per side) to the next finer
// one, per dimension: a fine point on coarse point i takes its value; a fine
// point halfway between coarse i-1 and i takes the 4-point (cubic) value
// (-c_{i-2} + 9 c_{i-1} + 9 c_i - c_{i+1}) / 16, where the coarse values are
// extended by the zero boundary values (c_{-1} = c_{nc} = 0) and their odd
// reflections (c_{-2} = -c_0, c_{nc+1} = -c_{nc-1}), as grid functions with
// homogeneous Dirichlet data are.  Sine modes are reproduced up to the factor
// (9 cos(theta/2) - cos(3 theta/2)) / 8.
__device__ __forceinline__ float p4_ext(const float* __restrict__ r, int nc, int j) {
  if (j >= 0 && j < nc) return r[j];
  if (j == -1 || j == nc) return 0.0f;
  return j < 0 ? -r[0] : -r[nc - 1];
}
__device__ __forceinline__ float p4_row(const float* __restrict__ r, int nc, int fj) {
  if (fj & 1) return r[(fj - 1) >> 1];
  const int i = fj >> 1;
  return (9.0f * (p4_ext(r, nc, i - 1) + p4_ext(r, nc, i)) - (p4_ext(r, nc, i - 2) + p4_ext(r, nc, i + 1))) *
         0.0625f;
}
// row ri of the coarse grid (extended like the values of one row) at fine column fj
__device__ __forceinline__ float p4_rowsel(const float* __restrict__ c, int nc, int ri, int fj) {
  if (ri >= 0 && ri < nc) return p4_row(c + (long long)ri * nc, nc, fj);
  if (ri == -1 || ri == nc) return 0.0f;
  return -p4_row(c + (long long)(ri < 0 ? 0 : nc - 1) * nc, nc, fj);
}
__device__ __forceinline__ float prolong_at(const float* __restrict__ c, int nc, int fi, int fj, int two_d) {
  if (!two_d) return p4_row(c, nc, fj);
  if (fi & 1) return p4_row(c + (long long)((fi - 1) >> 1) * nc, nc, fj);
  const int i = fi >> 1;
  return (9.0f * (p4_rowsel(c, nc, i - 1, fj) + p4_rowsel(c, nc, i, fj)) -
          (p4_rowsel(c, nc, i - 2, fj) + p4_rowsel(c, nc, i + 1, fj))) *
         0.0625f;
}

// Weights of coarse point i in the fine points (1D): P^T collects
// fine 2i+1 (1), 2i and 2i+2 (9/16), 2i-2 and 2i+4 (-1/16), and through the
// odd reflections fine 0 (+1/16 more, i = 0) and fine 2nc (+1/16 more, i = nc-1).
__device__ __forceinline__ int p4_adj_taps(int i, int nc, int* f, float* w) {
  int k = 0;
  const int nf = 2 * nc + 1;
  auto add = [&](int fi, float wi) {
    if (fi >= 0 && fi < nf) { f[k] = fi; w[k] = wi; ++k; }
  };
  add(2 * i - 2, -0.0625f);
  add(2 * i, i == 0 ? 0.625f : 0.5625f);
  add(2 * i + 1, 1.0f);
  add(2 * i + 2, i == nc - 1 ? 0.625f : 0.5625f);
  add(2 * i + 4, -0.0625f);
  return k;
}

// Level input [B][S + E + 1][HW_l]: the band (S channels), the extra channels
// of x sampled at the level's points, the level value.  sig[b * sbs + c * HW_l]
// is this level's signal, sig_next [B][S][HW_{l+1}] the next one (null at the
// coarsest level); x the fine input [B][S + E][HW_0].
__global__ void pyr_input_kernel(const float* __restrict__ sig, long long sbs, const float* __restrict__ sig_next,
                                 const float* __restrict__ x, float* __restrict__ xin, int B, int S, int E, int n,
                                 int n0, int stride, int two_d, float lval) {
  const int HW = (two_d ? n : 1) * n;
  const int HW0 = (two_d ? n0 : 1) * n0;
  const int C0 = S + E + 1;
  const int nc = (n - 1) / 2;
  const int HWc = (two_d ? nc : 1) * nc;
  const long long total = (long long)B * C0 * HW;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(idx % HW);
    const long long bc = idx / HW;
    const int c = (int)(bc % C0), b = (int)(bc / C0);
    const int i = q / n, j = q % n;
    float v;
    if (c < S) {
      v = sig[b * sbs + (long long)c * HW + q];
      if (sig_next) v -= prolong_at(sig_next + ((long long)b * S + c) * HWc, nc, i, j, two_d);
    } else if (c < S + E) {
      const int fi = two_d ? stride * (i + 1) - 1 : 0, fj = stride * (j + 1) - 1;
      v = x[((long long)b * (S + E) + c) * HW0 + (long long)fi * n0 + fj];
    } else {
      v = lval;
    }
    xin[idx] = v;
  }
}

// Y_l = s * out_l + P Y_{l+1}  (Y_next null at the coarsest level, out null
// for a level the network leaves out)
__global__ void pyr_combine_kernel(const float* __restrict__ out, const float* __restrict__ ynext,
                                   float* __restrict__ y, int BC, int n, int two_d, float s) {
  const int HW = (two_d ? n : 1) * n;
  const int nc = (n - 1) / 2;
  const int HWc = (two_d ? nc : 1) * nc;
  const long long total = (long long)BC * HW;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(idx % HW);
    const long long bc = idx / HW;
    float v = out ? s * out[idx] : 0.0f;
    if (ynext) v += prolong_at(ynext + bc * HWc, nc, q / n, q % n, two_d);
    y[idx] = v;
  }
}

// Adjoint of the interpolation, g_c = P^T g_f (taps of p4_adj_taps per dimension).
__global__ void pyr_prolong_adj_kernel(const float* __restrict__ gf, float* __restrict__ gc, int BC, int nf,
                                       int two_d) {
  const int nc = (nf - 1) / 2;
  const int HWc = (two_d ? nc : 1) * nc;
  const int HWf = (two_d ? nf : 1) * nf;
  const long long total = (long long)BC * HWc;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(idx % HWc);
    const long long bc = idx / HWc;
    const int i = q / nc, j = q % nc;
    const float* g = gf + bc * HWf;
    int fj[5], fi[5];
    float wj[5], wi[5];
    const int kj = p4_adj_taps(j, nc, fj, wj);
    float v = 0.0f;
    if (two_d) {
      const int ki = p4_adj_taps(i, nc, fi, wi);
      for (int a = 0; a < ki; ++a) {
        const float* r = g + (long long)fi[a] * nf;
        float rs = 0.0f;
        for (int b = 0; b < kj; ++b) rs += wj[b] * r[fj[b]];
        v += wi[a] * rs;
      }
    } else {
      for (int b = 0; b < kj; ++b) v += wj[b] * g[fj[b]];
    }
    gc[idx] = v;
  }
}

__global__ void scale_kernel(const float* __restrict__ x, float* __restrict__ y, long long n, float s) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = s * x[i];
}

// per-sample ||t_b||^2 and ||y_b - t_b||^2 (one block per sample)
__global__ __launch_bounds__(256) void loss_norms_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                         long long per, double* __restrict__ out) {
  __shared__ double r1[256], r2[256];
  const int b = blockIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (long long i = threadIdx.x; i < per; i += blockDim.x) {
    const double tv = t[b * per + i], d = (double)y[b * per + i] - tv;
    s1 += tv * tv;
    s2 += d * d;
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * b] = r1[0];
    out[2 * b + 1] = r2[0];
  }
}

// dL/dy for L = (1/B) sum_b ||y_b - t_b||^2 / (||t_b||^2 + eps)
__global__ void loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                 const double* __restrict__ norms, float* __restrict__ dy, int B, long long per,
                                 double eps) {
  const long long total = (long long)B * per;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(idx / per);
    dy[idx] = (float)(2.0 * ((double)y[idx] - t[idx]) / ((norms[2 * b] + eps) * B));
  }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, uint16_t* __restrict__ wbf, long long n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    wbf[i] = f32_to_bf16(pi);
  }
}

__global__ void round_bf16_kernel(const float* __restrict__ p, uint16_t* __restrict__ wbf, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    wbf[i] = f32_to_bf16(p[i]);
}

// ---------------------------------------------------------------------------
// Inference convolution on the bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16):
// the 3x3 convolution as nine shifted 1x1 products,
//   y[b][co][p] = bias[co] + sum_k sum_ci wk[k][co][ci] x[b][ci][p + off(k)],
// a GEMM per tap with the output channels as M, the pixels as N and the input
// channels as K.  The weights are re-laid out per tap as wk[k][co][cpad]
// (bfloat16, cpad = cin rounded up to 32, zero padded) so that a lane's 8
// consecutive K entries are one 16-byte load; the activations are read in
// float32 and rounded to bfloat16 (nearest even) as they enter the product;
// accumulation is float32.  Operand layout of the 16x16x32 instruction (lane
// l, c = l % 16, g = l / 16): A lane holds row c, K entries 8g .. 8g+7; B
// lane holds column c, the same K entries; the result element r of lane l is
// row 4g + r, column c.  A block of 4 waves covers 64 pixels (16 per wave)
// and 64 output channels (4 tiles of 16, grid.y over the rest); one launch
// covers every level of the pyramid (the small levels alone would leave the
// chip idle and pay a launch each).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaK = 32;

// Every pyramid level of one layer in one launch: level l owns the blocks
// [blk0[l], blk0[l+1]) and reads/writes its own arena regions.
constexpr int kMaxConvLevels = 32;
struct ConvLevels {
  int n;                                   // levels in the table
  int blk0[kMaxConvLevels + 1];            // first block of each level (blk0[n] = total)
  int H[kMaxConvLevels], W[kMaxConvLevels];
  long long in_off[kMaxConvLevels], out_off[kMaxConvLevels];  // floats from the arena bases
};

__global__ __launch_bounds__(256) void conv_fwd_mfma_kernel(const float* __restrict__ xbase,
                                                            const uint16_t* __restrict__ wk,
                                                            const float* __restrict__ bias, float* __restrict__ ybase,
                                                            int B, int cin, int cpad, int cout, ConvLevels lv,
                                                            int act) {
  int l = 0;
  while (l + 1 < lv.n && (int)blockIdx.x >= lv.blk0[l + 1]) ++l;   // uniform across the block
  const int H = lv.H[l], W = lv.W[l];
  const float* __restrict__ x = xbase + lv.in_off[l];
  float* __restrict__ y = ybase + lv.out_off[l];
  const int HW = H * W;
  const long long total = (long long)B * HW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const long long t = ((long long)(blockIdx.x - lv.blk0[l]) * 4 + wave) * 16 + c;   // this lane's pixel
  const bool tok = t < total;
  const long long tt = tok ? t : 0;
  const int b = (int)(tt / HW), p = (int)(tt % HW);
  const int py = p / W, px = p % W;
  const float* xb = x + (long long)b * cin * HW;
  const int co0 = blockIdx.y * 64;
  f32x4 acc[4];
#pragma unroll
  for (int tl = 0; tl < 4; ++tl) acc[tl] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  // the nine taps' neighbour offsets (-1: outside the grid or past the end)
  long long off[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int yy = py + k / 3 - 1, xx = px + k % 3 - 1;
    off[k] = (tok && yy >= 0 && yy < H && xx >= 0 && xx < W) ? (long long)yy * W + xx : -1;
  }
  for (int k0 = 0; k0 < cpad; k0 += kMfmaK) {
    // all nine taps' activations of this K chunk are loaded before the
    // products, so the loads overlap instead of waiting one tap at a time
    bf16x8 bv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int ci = k0 + 8 * g + j;
        const float v = (off[k] >= 0 && ci < cin) ? xb[(long long)ci * HW + off[k]] : 0.0f;
        bv[k][j] = __builtin_bit_cast(__bf16, f32_to_bf16(v));
      }
    }
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) {
      if (co0 + 16 * tl >= cout) break;   // uniform across the wave
      const int co = co0 + 16 * tl + c;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        bf16x8 av;
        if (co < cout) {
          av = *reinterpret_cast<const bf16x8*>(wk + ((long long)k * cout + co) * cpad + k0 + 8 * g);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) av[j] = __builtin_bit_cast(__bf16, (uint16_t)0);
        }
        acc[tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[k], acc[tl], 0, 0, 0);
      }
    }
  }
  if (!tok) return;
  float* yb = y + (long long)b * cout * HW + p;
#pragma unroll
  for (int tl = 0; tl < 4; ++tl) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = co0 + 16 * tl + 4 * g + r;
      if (co < cout) {
        const float v = acc[tl][r] + bias[co];
        yb[(long long)co * HW] = act ? tanhf(v) : v;
      }
    }
  }
}

// wk[k][co][ci] (ci < cpad, zero beyond cin) = bfloat16 of w[co][ci][k]
__global__ void relayout_mfma_kernel(const float* __restrict__ w, uint16_t* __restrict__ wk, int cin, int cpad,
                                     int cout) {
  const long long n = 9LL * cout * cpad;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(idx / ((long long)cout * cpad));
    const long long rem = idx % ((long long)cout * cpad);
    const int co = (int)(rem / cpad), ci = (int)(rem % cpad);
    wk[idx] = ci < cin ? f32_to_bf16(w[((long long)co * cin + ci) * 9 + k]) : (uint16_t)0;
  }
}

// Input channels of the warm start for one instance: b at the slice rows
// divided by `scale`, then constant channels alpha and r / 10.
// split: b is in the solver's colour-split storage of 2D grids (the even
// flat indices first, then the odd ones); x is in natural order.
__global__ void gather_slices_kernel(const double* __restrict__ b, const int* __restrict__ rows, int nslices,
                                     long long N, double scale, float alpha, float rdiv, float* __restrict__ x,
                                     int split) {
  const long long total = (long long)(nslices + 2) * N;
  const long long n0 = (N + 1) / 2;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(idx / N);
    const long long q = idx % N;
    const long long qs = split ? ((q & 1) ? n0 + (q >> 1) : (q >> 1)) : q;
    float v;
    if (c < nslices) v = (float)(b[(long long)rows[c] * N + qs] / scale);
    else v = c == nslices ? alpha : rdiv;
    x[idx] = v;
  }
}

// Slices a solver prediction may take (the plan's limit).
constexpr int kMaxSlices = 64;

// u[m][q] = interpolation of the predicted slices (times scale), piecewise
// linear in the variable s = t^alpha (tp[m] = t_m^alpha): slice k sits at
// tp[rows[k] + 1].  Before the first slice it runs from the initial value g
// (zero if null) at tp[0]; after the last slice it stays constant.  split: u
// is written in the solver's colour-split storage (y and g are natural).
__global__ void time_interp_kernel(const float* __restrict__ y, const int* __restrict__ rows, int nslices,
                                   const double* __restrict__ t, const double* __restrict__ g, long long M,
                                   long long N, double scale, double* __restrict__ u, int split) {
  // blockIdx.y walks the time rows: the bracketing slices and the weights
  // are the same for the whole row, the columns are plain coalesced streams
  __shared__ int srows[kMaxSlices];
  for (int i = threadIdx.x; i < nslices; i += blockDim.x) srows[i] = rows[i];
  __syncthreads();
  for (long long m = blockIdx.y; m < M; m += gridDim.y) {
    int s = 0;
    while (s < nslices && srows[s] < m) ++s;
    // u[m][q] = wa * ya[q] + wb * yb[q], ya from slice sa (-1: g, or zero)
    int sa, sb;
    double wa, wb;
    if (s == nslices) {
      sa = -2; sb = nslices - 1; wa = 0.0; wb = scale;
    } else if (srows[s] == m) {
      sa = -2; sb = s; wa = 0.0; wb = scale;
    } else {
      const double ta = s == 0 ? t[0] : t[srows[s - 1] + 1];
      const double tb = t[srows[s] + 1];
      const double th = (t[m + 1] - ta) / (tb - ta);
      sa = s - 1; sb = s;
      wa = 1.0 - th; wb = scale * th;
    }
    const float* yb = y + (long long)sb * N;
    const float* ya = sa >= 0 ? y + (long long)sa * N : nullptr;
    const double* ga = sa == -1 ? g : nullptr;
    double* um = u + m * N;
    const long long n0 = (N + 1) / 2;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
      const long long q = split ? (i < n0 ? 2 * i : 2 * (i - n0) + 1) : i;   // storage i holds point q
      double v = wb * (double)yb[q];
      if (ya) v += wa * (scale * (double)ya[q]);
      else if (ga) v += wa * ga[q];
      um[i] = v;
    }
  }
}

static inline int grid_of(long long total) {
  long long g = (total + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

hipError_t launch_gather_slices(const double* b, const int* rows, int nslices, long long N, double scale,
                                float alpha, float rdiv, float* x, bool split, hipStream_t s) {
  hipLaunchKernelGGL(gather_slices_kernel, dim3(grid_of((long long)(nslices + 2) * N)), dim3(256), 0, s, b, rows,
                     nslices, N, scale, alpha, rdiv, x, split ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_time_interp(const float* y, const int* rows, int nslices, const double* t, const double* g,
                              long long M, long long N, double scale, double* u, bool split, hipStream_t s) {
  if (nslices < 1 || nslices > kMaxSlices) return hipErrorInvalidValue;
  // a few blocks per row (each thread streams several columns), rows over y
  const long long gx = std::min<long long>((N + 255) / 256, 16);
  const long long gy = std::min<long long>(M, 65535);
  hipLaunchKernelGGL(time_interp_kernel, dim3((unsigned)std::max<long long>(gx, 1), (unsigned)std::max<long long>(gy, 1)),
                     dim3(256), 0, s, y, rows, nslices, t, g, M, N, scale, u, split ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mgwr

using namespace mgwr;

namespace {
int nfail(int code, const std::string& m) {
  set_last_error(m);
  return code;
}
#define NET_TRY(...)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (__VA_ARGS__);                                                                \
    if (e_ != hipSuccess) return nfail(MGWR_ERR_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Pyramid geometry of one call.
struct Geo {
  int B, H, W, two_d, nlev;
  std::vector<int> n;         // points per side at each level
  std::vector<long long> hw;  // points per level
  std::vector<long long> cum; // sum of hw over the finer levels
};

bool geometry(int B, int H, int W, Geo* g) {
  if (B < 1 || W < 3 || ((W + 1) & W) != 0 || !(H == 1 || H == W)) return false;
  g->B = B;
  g->H = H;
  g->W = W;
  g->two_d = H == W ? 1 : 0;
  g->n.clear();
  g->hw.clear();
  g->cum.clear();
  long long acc = 0;
  for (int n = W; n >= 3; n = (n - 1) / 2) {
    g->n.push_back(n);
    const long long hw = (long long)(g->two_d ? n : 1) * n;
    g->cum.push_back(acc);
    g->hw.push_back(hw);
    acc += hw;
  }
  g->nlev = (int)g->n.size();
  return true;
}
}  // namespace

struct mgwr_net {
  std::vector<int> ch;              // convolution channels c_0..c_L (c_0 = S + E + 1)
  int nsig = 0, nextra = 0;
  std::vector<size_t> woff, boff;   // parameter offsets (floats)
  size_t nparam = 0;
  long long cap = 0;                // bound capacity: batch * H * W of the finest level
  int maxc = 0;
  bool bound = false;
  hipStream_t stream = nullptr;
  float* params = nullptr;          // caller-owned master weights
  uint16_t* wbf = nullptr;
  float *grad = nullptr, *m = nullptr, *v = nullptr;
  float *sig = nullptr, *xin = nullptr, *ybuf = nullptr, *gy = nullptr;  // per-level arenas
  float* xstage = nullptr;          // the solver's input staging [S+E][cap] (a fixed address for graph replay)
  uint16_t* wmf = nullptr;          // per-tap bfloat16 weights of the matrix-core convolution
  std::vector<size_t> mfoff;        // per layer: offset into wmf (entries)
  std::vector<int> cpad;            // per layer: input channels rounded up to 32
  std::mutex mu;                    // one solver prediction at a time (shared buffers and stream)
  std::vector<float*> act;          // act[j]: output of layer j at every level
  float *g0 = nullptr, *g1 = nullptr;  // backprop scratch of one level [cap * maxc]
  double* norms = nullptr;          // per-sample loss norms
  double h_min = 0.0;               // levels with h_l < h_min contribute nothing
  // the solver's inference replayed from a captured graph while its input
  // array, grid and spacing stay the same (the weights are read at replay)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;
  const float* graph_x = nullptr;
  int graph_H = 0, graph_W = 0;
  double graph_h = 0.0;
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  ~mgwr_net() {
    drop_graph();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
  static constexpr int kMaxBatch = 4096;

  // a level takes part when its spacing is not finer than h_min
  bool active(double hl) const { return hl >= h_min * (1.0 - 1e-9); }

  int L() const { return (int)ch.size() - 1; }
  int in_channels() const { return nsig + nextra; }

  long long layout(long long cap_, std::vector<size_t>* offs) const {
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off += (bytes + 255) & ~size_t(255);
      return o;
    };
    const size_t P = (size_t)2 * cap_;  // all levels of a pyramid fit in twice the finest
    std::vector<size_t> o;
    o.push_back(take(nparam * 2));                      // 0 wbf
    o.push_back(take(nparam * 4));                      // 1 grad
    o.push_back(take(nparam * 4));                      // 2 m
    o.push_back(take(nparam * 4));                      // 3 v
    o.push_back(take(P * nsig * 4));                    // 4 sig
    o.push_back(take(P * ch[0] * 4));                   // 5 xin
    o.push_back(take(P * ch.back() * 4));               // 6 ybuf
    o.push_back(take(P * ch.back() * 4));               // 7 gy
    o.push_back(take((size_t)cap_ * maxc * 4));         // 8 g0
    o.push_back(take((size_t)cap_ * maxc * 4));         // 9 g1
    o.push_back(take(kMaxBatch * 2 * sizeof(double)));  // 10 norms
    o.push_back(take((size_t)cap_ * in_channels() * 4)); // 11 xstage
    size_t nmf = 0;
    for (int j = 0; j < L(); ++j) nmf += (size_t)9 * ch[j + 1] * ((ch[j] + 31) / 32 * 32);
    o.push_back(take(nmf * 2));                         // 12 wmf
    for (int j = 0; j < L(); ++j) o.push_back(take(P * ch[j + 1] * 4));  // 13 + j act
    if (offs) *offs = o;
    return (long long)off;
  }
};

namespace {

int check_net(mgwr_net* net, int B, int H, int W, Geo* g) {
  if (!net || !net->bound) return nfail(MGWR_ERR_STATE, "network is not bound");
  if (B > mgwr_net::kMaxBatch) return nfail(MGWR_ERR_INVALID_ARG, "batch exceeds 4096");
  if (!geometry(B, H, W, g))
    return nfail(MGWR_ERR_INVALID_ARG, "grid must have W = 2^p - 1 >= 3 points with H = 1 or H = W");
  if ((long long)B * H * W > net->cap) return nfail(MGWR_ERR_INVALID_ARG, "batch*H*W exceeds the bound capacity");
  return MGWR_OK;
}

int launch_conv_fwd(mgwr_net* net, int j, const float* in, float* out, int B, int H, int W) {
  const int cin = net->ch[j], cout = net->ch[j + 1];
  const long long px = (long long)B * H * W;
  dim3 grid((unsigned)((px + 256 * kPx - 1) / (256 * kPx)), (unsigned)((cout + kCoTile - 1) / kCoTile));
  hipLaunchKernelGGL(conv_fwd_kernel, grid, dim3(256), 0, net->stream, in, net->wbf + net->woff[j],
                     net->params + net->boff[j], out, B, cin, cout, H, W, j + 1 < net->L() ? 1 : 0);
  NET_TRY(hipGetLastError());
  return MGWR_OK;
}

// Layer j of every active level on the matrix cores, one launch; in_base /
// out_base are the arenas (level l at B * channels * cum[l]).
int launch_conv_fwd_mfma(mgwr_net* net, int j, const float* in_base, float* out_base, const Geo& g, double h0) {
  const int B = g.B, cin = net->ch[j], cout = net->ch[j + 1];
  ConvLevels lv{};
  long long blocks = 0;
  for (int l = 0; l < g.nlev; ++l) {
    if (!net->active(std::ldexp(h0, l))) continue;
    if (lv.n == kMaxConvLevels) return nfail(MGWR_ERR_INVALID_ARG, "too many pyramid levels");
    lv.blk0[lv.n] = (int)blocks;
    lv.H[lv.n] = g.two_d ? g.n[l] : 1;
    lv.W[lv.n] = g.n[l];
    lv.in_off[lv.n] = (long long)B * cin * g.cum[l];
    lv.out_off[lv.n] = (long long)B * cout * g.cum[l];
    blocks += ((long long)B * g.hw[l] + 63) / 64;
    if (blocks > 0x7fffffffLL) return nfail(MGWR_ERR_INVALID_ARG, "grid too large");
    ++lv.n;
  }
  if (lv.n == 0) return MGWR_OK;
  lv.blk0[lv.n] = (int)blocks;
  dim3 grid((unsigned)blocks, (unsigned)((cout + 63) / 64));
  hipLaunchKernelGGL(conv_fwd_mfma_kernel, grid, dim3(256), 0, net->stream, in_base, net->wmf + net->mfoff[j],
                     net->params + net->boff[j], out_base, B, cin, net->cpad[j], cout, lv, j + 1 < net->L() ? 1 : 0);
  NET_TRY(hipGetLastError());
  return MGWR_OK;
}

// Per-tap bfloat16 weights of the matrix-core convolution from the master
// weights (after every change of them).
int refresh_mfma_weights(mgwr_net* net) {
  for (int j = 0; j < net->L(); ++j) {
    const long long n = 9LL * net->ch[j + 1] * net->cpad[j];
    hipLaunchKernelGGL(relayout_mfma_kernel, dim3(grid_of(n)), dim3(256), 0, net->stream, net->params + net->woff[j],
                       net->wmf + net->mfoff[j], net->ch[j], net->cpad[j], net->ch[j + 1]);
    NET_TRY(hipGetLastError());
  }
  return MGWR_OK;
}

// Forward pass of the whole pyramid; leaves the activations of every level in
// the arenas and the output in level 0 of ybuf.  mfma: the convolutions run
// on the bfloat16 matrix cores (activations rounded to bfloat16 at their
// input; inference), else the float32 kernels (training: the gradient is that
// of this forward pass).
int net_forward(mgwr_net* net, const float* x, const Geo& g, double h0, bool mfma) {
  const int B = g.B, S = net->nsig, E = net->nextra, C0 = net->ch[0], CL = net->ch.back();
  const long long HW0 = g.hw[0];
  int rc;
  // the signal of level l: x itself at level 0, the sig arena below
  auto sig_at = [&](int l) -> const float* { return l == 0 ? x : net->sig + (size_t)B * S * g.cum[l]; };
  auto sig_bs = [&](int l) -> long long { return l == 0 ? (long long)(S + E) * HW0 : (long long)S * g.hw[l]; };
  for (int l = 0; l + 1 < g.nlev; ++l) {
    float* dst = net->sig + (size_t)B * S * g.cum[l + 1];
    hipLaunchKernelGGL(pyr_restrict_kernel, dim3(grid_of((long long)B * S * g.hw[l + 1])), dim3(256), 0,
                       net->stream, sig_at(l), sig_bs(l), dst, B, S, g.n[l], g.two_d);
    NET_TRY(hipGetLastError());
  }
  for (int l = 0; l < g.nlev; ++l) {
    const int Hl = g.two_d ? g.n[l] : 1, Wl = g.n[l];
    const float* sn = l + 1 < g.nlev ? net->sig + (size_t)B * S * g.cum[l + 1] : nullptr;
    float* xin = net->xin + (size_t)B * C0 * g.cum[l];
    const double hl = std::ldexp(h0, l);
    if (!net->active(hl)) continue;
    hipLaunchKernelGGL(pyr_input_kernel, dim3(grid_of((long long)B * C0 * g.hw[l])), dim3(256), 0, net->stream,
                       sig_at(l), sig_bs(l), sn, x, xin, B, S, E, g.n[l], g.W, 1 << l, g.two_d,
                       (float)(std::log2(1.0 / hl) / 10.0));
    NET_TRY(hipGetLastError());
    if (mfma) continue;   // the matrix-core layers run all levels at once below
    const float* in = xin;
    for (int j = 0; j < net->L(); ++j) {
      float* out = net->act[j] + (size_t)B * net->ch[j + 1] * g.cum[l];
      if ((rc = launch_conv_fwd(net, j, in, out, B, Hl, Wl))) return rc;
      in = out;
    }
  }
  if (mfma) {
    for (int j = 0; j < net->L(); ++j)
      if ((rc = launch_conv_fwd_mfma(net, j, j == 0 ? net->xin : net->act[j - 1], net->act[j], g, h0))) return rc;
  }
  for (int l = g.nlev - 1; l >= 0; --l) {
    const double hl = std::ldexp(h0, l);
    const float* out = net->active(hl) ? net->act[net->L() - 1] + (size_t)B * CL * g.cum[l] : nullptr;
    const float* yn = l + 1 < g.nlev ? net->ybuf + (size_t)B * CL * g.cum[l + 1] : nullptr;
    float* y = net->ybuf + (size_t)B * CL * g.cum[l];
    hipLaunchKernelGGL(pyr_combine_kernel, dim3(grid_of((long long)B * CL * g.hw[l])), dim3(256), 0, net->stream,
                       out, yn, y, B * CL, g.n[l], g.two_d, (float)(4.0 * hl * hl));
    NET_TRY(hipGetLastError());
  }
  return MGWR_OK;
}

bool valid_h(double h) { return std::isfinite(h) && h > 0.0; }

}  // namespace

extern "C" {

int mgwr_net_create(int layers, const int* channels, int nsignal, mgwr_net** out) {
  if (!out || !channels || layers < 1 || layers > 16) return nfail(MGWR_ERR_INVALID_ARG, "bad network shape");
  *out = nullptr;
  for (int l = 0; l <= layers; ++l)
    if (channels[l] < 1 || channels[l] > 1024)
      return nfail(MGWR_ERR_INVALID_ARG, "channel counts must lie in [1, 1024]");
  if (nsignal < 1 || nsignal > channels[0] - 1)
    return nfail(MGWR_ERR_INVALID_ARG, "nsignal must lie in [1, channels[0] - 1]");
  mgwr_net* net = new (std::nothrow) mgwr_net();
  if (!net) return nfail(MGWR_ERR_INVALID_ARG, "out of host memory");
  for (int l = 0; l <= layers; ++l) {
    net->ch.push_back(channels[l]);
    net->maxc = std::max(net->maxc, channels[l]);
  }
  net->nsig = nsignal;
  net->nextra = channels[0] - 1 - nsignal;
  size_t off = 0;
  for (int l = 0; l < layers; ++l) {
    net->woff.push_back(off);
    off += (size_t)channels[l + 1] * channels[l] * 9;
    net->boff.push_back(off);
    off += channels[l + 1];
  }
  net->nparam = off;
  *out = net;
  return MGWR_OK;
}

int mgwr_net_param_count(const mgwr_net* net, size_t* n) {
  if (!net || !n) return nfail(MGWR_ERR_INVALID_ARG, "null argument");
  *n = net->nparam;
  return MGWR_OK;
}

int mgwr_net_workspace_bytes(const mgwr_net* net, long long max_bhw, size_t* bytes) {
  if (!net || !bytes || max_bhw < 1) return nfail(MGWR_ERR_INVALID_ARG, "bad argument");
  *bytes = (size_t)net->layout(max_bhw, nullptr);
  return MGWR_OK;
}

int mgwr_net_bind(mgwr_net* net, float* params_dev, long long max_bhw, void* ws, size_t bytes, void* stream) {
  if (!net || !params_dev || !ws || max_bhw < 1) return nfail(MGWR_ERR_INVALID_ARG, "bad argument");
  if (((uintptr_t)ws & 255) != 0) return nfail(MGWR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  std::vector<size_t> o;
  const long long need = net->layout(max_bhw, &o);
  if ((long long)bytes < need) return nfail(MGWR_ERR_STATE, "workspace too small");
  unsigned char* w = (unsigned char*)ws;
  net->stream = (hipStream_t)stream;
  net->params = params_dev;
  net->wbf = (uint16_t*)(w + o[0]);
  net->grad = (float*)(w + o[1]);
  net->m = (float*)(w + o[2]);
  net->v = (float*)(w + o[3]);
  net->sig = (float*)(w + o[4]);
  net->xin = (float*)(w + o[5]);
  net->ybuf = (float*)(w + o[6]);
  net->gy = (float*)(w + o[7]);
  net->g0 = (float*)(w + o[8]);
  net->g1 = (float*)(w + o[9]);
  net->norms = (double*)(w + o[10]);
  net->xstage = (float*)(w + o[11]);
  net->wmf = (uint16_t*)(w + o[12]);
  net->mfoff.clear();
  net->cpad.clear();
  {
    size_t off = 0;
    for (int j = 0; j < net->L(); ++j) {
      net->cpad.push_back((net->ch[j] + 31) / 32 * 32);
      net->mfoff.push_back(off);
      off += (size_t)9 * net->ch[j + 1] * net->cpad.back();
    }
  }
  net->act.assign(net->L(), nullptr);
  for (int j = 0; j < net->L(); ++j) net->act[j] = (float*)(w + o[13 + j]);
  net->cap = max_bhw;
  NET_TRY(hipMemsetAsync(net->m, 0, net->nparam * 4, net->stream));
  NET_TRY(hipMemsetAsync(net->v, 0, net->nparam * 4, net->stream));
  hipLaunchKernelGGL(round_bf16_kernel, dim3(grid_of((long long)net->nparam)), dim3(256), 0, net->stream,
                     net->params, net->wbf, (long long)net->nparam);
  NET_TRY(hipGetLastError());
  int rc = refresh_mfma_weights(net);
  if (rc) return rc;
  NET_TRY(hipStreamSynchronize(net->stream));
  net->drop_graph();
  net->bound = true;
  return MGWR_OK;
}

int mgwr_net_sync_weights(mgwr_net* net) {
  if (!net || !net->bound) return nfail(MGWR_ERR_STATE, "network is not bound");
  hipLaunchKernelGGL(round_bf16_kernel, dim3(grid_of((long long)net->nparam)), dim3(256), 0, net->stream,
                     net->params, net->wbf, (long long)net->nparam);
  NET_TRY(hipGetLastError());
  return refresh_mfma_weights(net);
}

int mgwr_net_forward(mgwr_net* net, const float* x, int B, int H, int W, double h, float* y) {
  Geo g;
  int rc = check_net(net, B, H, W, &g);
  if (rc) return rc;
  if (!x || !y) return nfail(MGWR_ERR_INVALID_ARG, "null array");
  if (!valid_h(h)) return nfail(MGWR_ERR_INVALID_ARG, "h must be positive");
  if ((rc = net_forward(net, x, g, h, true))) return rc;
  NET_TRY(hipMemcpyAsync(y, net->ybuf, (size_t)B * net->ch.back() * g.hw[0] * 4, hipMemcpyDeviceToDevice,
                         net->stream));
  return MGWR_OK;
}

int mgwr_net_gradient(mgwr_net* net, const float* x, const float* target, int B, int H, int W, double h,
                      float* grad_out, double* loss_host) {
  Geo g;
  int rc = check_net(net, B, H, W, &g);
  if (rc) return rc;
  if (!x || !target) return nfail(MGWR_ERR_INVALID_ARG, "null array");
  if (!valid_h(h)) return nfail(MGWR_ERR_INVALID_ARG, "h must be positive");
  if ((rc = net_forward(net, x, g, h, false))) return rc;
  const int L = net->L(), CL = net->ch.back(), C0 = net->ch[0];
  const long long per = (long long)CL * g.hw[0];
  hipLaunchKernelGGL(loss_norms_kernel, dim3(B), dim3(256), 0, net->stream, net->ybuf, target, per, net->norms);
  NET_TRY(hipGetLastError());
  hipLaunchKernelGGL(loss_grad_kernel, dim3(grid_of(B * per)), dim3(256), 0, net->stream, net->ybuf, target,
                     net->norms, net->gy, B, per, 1e-30);
  NET_TRY(hipGetLastError());
  NET_TRY(hipMemsetAsync(net->grad, 0, net->nparam * 4, net->stream));
  for (int l = 0; l < g.nlev; ++l) {
    const int Hl = g.two_d ? g.n[l] : 1, Wl = g.n[l];
    float* gyl = net->gy + (size_t)B * CL * g.cum[l];
    if (l > 0) {
      const float* gyp = net->gy + (size_t)B * CL * g.cum[l - 1];
      hipLaunchKernelGGL(pyr_prolong_adj_kernel, dim3(grid_of((long long)B * CL * g.hw[l])), dim3(256), 0,
                         net->stream, gyp, gyl, B * CL, g.n[l - 1], g.two_d);
      NET_TRY(hipGetLastError());
    }
    const double hl = std::ldexp(h, l);
    if (!net->active(hl)) continue;
    const long long cnt = (long long)B * CL * g.hw[l];
    hipLaunchKernelGGL(scale_kernel, dim3(grid_of(cnt)), dim3(256), 0, net->stream, gyl, net->g0, cnt,
                       (float)(4.0 * hl * hl));
    NET_TRY(hipGetLastError());
    float* dcur = net->g0;
    float* dnext = net->g1;
    for (int j = L - 1; j >= 0; --j) {
      const int cin = net->ch[j], cout = net->ch[j + 1];
      const float* in = j == 0 ? net->xin + (size_t)B * C0 * g.cum[l] : net->act[j - 1] + (size_t)B * cin * g.cum[l];
      const int nblk = ((cout + kWgCo - 1) / kWgCo) * cin;
      hipLaunchKernelGGL(conv_bwd_weight_kernel, dim3(nblk), dim3(256), 0, net->stream, dcur, in,
                         net->grad + net->woff[j], net->grad + net->boff[j], B, cin, cout, Hl, Wl);
      NET_TRY(hipGetLastError());
      if (j > 0) {
        const long long px = (long long)B * Hl * Wl;
        dim3 grid((unsigned)((px + 256 * kPx - 1) / (256 * kPx)), (unsigned)((cin + kCoTile - 1) / kCoTile));
        hipLaunchKernelGGL(conv_bwd_data_kernel, grid, dim3(256), 0, net->stream, dcur, net->wbf + net->woff[j], in,
                           dnext, B, cin, cout, Hl, Wl, 1);
        NET_TRY(hipGetLastError());
        std::swap(dcur, dnext);
      }
    }
  }
  if (grad_out)
    NET_TRY(hipMemcpyAsync(grad_out, net->grad, net->nparam * 4, hipMemcpyDeviceToDevice, net->stream));
  if (loss_host) {
    std::vector<double> nh((size_t)2 * B);
    NET_TRY(hipMemcpyAsync(nh.data(), net->norms, nh.size() * sizeof(double), hipMemcpyDeviceToHost, net->stream));
    NET_TRY(hipStreamSynchronize(net->stream));
    double lsum = 0.0;
    for (int b = 0; b < B; ++b) lsum += nh[2 * b + 1] / (nh[2 * b] + 1e-30);
    *loss_host = lsum / B;
  }
  return MGWR_OK;
}

int mgwr_net_set_finest(mgwr_net* net, double h_min) {
  if (!net) return nfail(MGWR_ERR_INVALID_ARG, "null network");
  if (!(h_min >= 0.0) || !std::isfinite(h_min)) return nfail(MGWR_ERR_INVALID_ARG, "h_min must be >= 0");
  net->h_min = h_min;
  net->drop_graph();
  return MGWR_OK;
}

int mgwr_net_adam_step(mgwr_net* net, float lr, float beta1, float beta2, float eps, int step) {
  if (!net || !net->bound) return nfail(MGWR_ERR_STATE, "network is not bound");
  if (step < 1) return nfail(MGWR_ERR_INVALID_ARG, "step counts from 1");
  const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_of((long long)net->nparam)), dim3(256), 0, net->stream, net->params,
                     net->grad, net->m, net->v, net->wbf, (long long)net->nparam, lr, beta1, beta2, eps, c1, c2);
  NET_TRY(hipGetLastError());
  return refresh_mfma_weights(net);
}

int mgwr_net_destroy(mgwr_net* net) {
  delete net;
  return MGWR_OK;
}

}  // extern "C"

// internal: forward pass for the solver's warm start
namespace mgwr {
int net_infer(mgwr_net* net, const float* x, int H, int W, double h, const float** y) {
  Geo g;
  int rc = check_net(net, 1, H, W, &g);
  if (rc) return rc;
  if (!valid_h(h)) return nfail(MGWR_ERR_INVALID_ARG, "h must be positive");
  *y = net->ybuf;
  if (net->graph_exec && net->graph_x == x && net->graph_H == H && net->graph_W == W && net->graph_h == h) {
    NET_TRY(hipGraphLaunch(net->graph_exec, net->stream));
    return MGWR_OK;
  }
  // capture the ~60 small launches of one inference once (on a private
  // stream: the caller's may be the legacy stream), then replay
  net->drop_graph();
  if (!net->capture_stream) NET_TRY(hipStreamCreateWithFlags(&net->capture_stream, hipStreamNonBlocking));
  hipStream_t keep = net->stream;
  net->stream = net->capture_stream;
  NET_TRY(hipStreamBeginCapture(net->capture_stream, hipStreamCaptureModeRelaxed));
  rc = net_forward(net, x, g, h, true);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(net->capture_stream, &gr);
  net->stream = keep;
  if (rc || e != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc ? rc : nfail(MGWR_ERR_HIP, "capturing the inference failed");
  }
  net->graph = gr;
  NET_TRY(hipGraphInstantiate(&net->graph_exec, gr, nullptr, nullptr, 0));
  net->graph_x = x;
  net->graph_H = H;
  net->graph_W = W;
  net->graph_h = h;
  NET_TRY(hipGraphLaunch(net->graph_exec, net->stream));
  return MGWR_OK;
}
int net_signal_channels(const mgwr_net* net) { return net->nsig; }
int net_input_channels(const mgwr_net* net) { return net->in_channels(); }
int net_out_channels(const mgwr_net* net) { return net->ch.back(); }
long long net_capacity(const mgwr_net* net) { return net->bound ? net->cap : 0; }
hipStream_t net_stream(const mgwr_net* net) { return net->stream; }
std::mutex& net_mutex(mgwr_net* net) { return net->mu; }
float* net_input_stage(mgwr_net* net) { return net->xstage; }
bool net_same_shape(const mgwr_net* net, int layers, const int* channels, int nsignal) {
  if (net->L() != layers || net->nsig != nsignal) return false;
  for (int l = 0; l <= layers; ++l)
    if (net->ch[l] != channels[l]) return false;
  return true;
}
bool net_is_bound(const mgwr_net* net) { return net->bound; }
float* net_params(mgwr_net* net) { return net->params; }
size_t net_param_count(const mgwr_net* net) { return net->nparam; }
}  // namespace mgwr
