// Learned initial guess: a small convolution network on the gfx950, with
// hand-written forward, backward and Adam kernels.
//
// Layers l = 0..L-1: 3x3 convolution (zero padding, stride 1) from c_l to
// c_{l+1} channels, tanh after every layer but the last.  Tensors are
// [batch][channel][H][W] float32; a 1D grid is an image of height 1.  The
// forward pass and the data gradient use bfloat16 copies of the weights
// (refreshed after every update) with float32 accumulation; the master
// weights, their gradients and the Adam moments are float32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
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

// y[b][co][p] = bias[co] + sum_ci sum_k w[co][ci][k] x[b][ci][p + off(k)], optional tanh
__global__ void conv_fwd_kernel(const float* __restrict__ x, const uint16_t* __restrict__ w,
                                const float* __restrict__ bias, float* __restrict__ y, int B, int cin, int cout,
                                int H, int W, int act) {
  const long long HW = (long long)H * W;
  const long long total = (long long)B * cout * HW;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long p = idx % HW;
    const int co = (int)((idx / HW) % cout);
    const int b = (int)(idx / (HW * cout));
    const int py = (int)(p / W), px = (int)(p % W);
    float acc = bias[co];
    const float* xb = x + (long long)b * cin * HW;
    const uint16_t* wc = w + (long long)co * cin * 9;
    for (int ci = 0; ci < cin; ++ci) {
      const float* xc = xb + ci * HW;
      const uint16_t* wk = wc + ci * 9;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const int yy = py + ky - 1;
        if (yy < 0 || yy >= H) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int xx = px + kx - 1;
          if (xx < 0 || xx >= W) continue;
          acc += bf16_to_f32(wk[ky * 3 + kx]) * xc[(long long)yy * W + xx];
        }
      }
    }
    y[idx] = act ? tanhf(acc) : acc;
  }
}

// dx[b][ci][p] = sum_co sum_k w[co][ci][k] dy[b][co][p - off(k)]; times (1 - a^2)
// when the input of this layer is the tanh output a of the previous layer
__global__ void conv_bwd_data_kernel(const float* __restrict__ dy, const uint16_t* __restrict__ w,
                                     const float* __restrict__ a_prev, float* __restrict__ dx, int B, int cin,
                                     int cout, int H, int W, int act_prev) {
  const long long HW = (long long)H * W;
  const long long total = (long long)B * cin * HW;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long p = idx % HW;
    const int ci = (int)((idx / HW) % cin);
    const int b = (int)(idx / (HW * cin));
    const int py = (int)(p / W), px = (int)(p % W);
    float acc = 0.0f;
    const float* db = dy + (long long)b * cout * HW;
    for (int co = 0; co < cout; ++co) {
      const float* dc = db + co * HW;
      const uint16_t* wk = w + ((long long)co * cin + ci) * 9;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const int yy = py - (ky - 1);
        if (yy < 0 || yy >= H) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int xx = px - (kx - 1);
          if (xx < 0 || xx >= W) continue;
          acc += bf16_to_f32(wk[ky * 3 + kx]) * dc[(long long)yy * W + xx];
        }
      }
    }
    if (act_prev) {
      const float a = a_prev[idx];
      acc *= 1.0f - a * a;
    }
    dx[idx] = acc;
  }
}

// dw[co][ci][k] = sum_{b,p} dy[b][co][p] x[b][ci][p + off(k)]  (one block per weight),
// db[co] = sum_{b,p} dy[b][co][p]  (blocks with ci == cin)
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const float* __restrict__ dy,
                                                              const float* __restrict__ x, float* __restrict__ dw,
                                                              float* __restrict__ dbias, int B, int cin, int cout,
                                                              int H, int W) {
  __shared__ float red[256];
  const int blk = blockIdx.x;  // co * (cin*9 + 1) + j
  const int per = cin * 9 + 1;
  const int co = blk / per, j = blk % per;
  const long long HW = (long long)H * W;
  const long long total = (long long)B * HW;
  float acc = 0.0f;
  if (j == cin * 9) {
    for (long long t = threadIdx.x; t < total; t += blockDim.x) {
      const long long b = t / HW, p = t % HW;
      acc += dy[(b * cout + co) * HW + p];
    }
  } else {
    const int ci = j / 9, k = j % 9, ky = k / 3, kx = k % 3;
    for (long long t = threadIdx.x; t < total; t += blockDim.x) {
      const long long b = t / HW, p = t % HW;
      const int py = (int)(p / W), px = (int)(p % W);
      const int yy = py + ky - 1, xx = px + kx - 1;
      if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
      acc += dy[(b * cout + co) * HW + p] * x[(b * cin + ci) * HW + (long long)yy * W + xx];
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (j == cin * 9) dbias[co] = red[0];
    else dw[(long long)co * cin * 9 + j] = red[0];
  }
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

// Input channels of the warm start for one instance: f at the slice rows
// divided by `scale`, then constant channels alpha and r / 10.
__global__ void gather_slices_kernel(const double* __restrict__ b, const int* __restrict__ rows, int nslices,
                                     long long N, double scale, float alpha, float rdiv, float* __restrict__ x) {
  const long long total = (long long)(nslices + 2) * N;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(idx / N);
    const long long q = idx % N;
    float v;
    if (c < nslices) v = (float)(b[(long long)rows[c] * N + q] / scale);
    else v = c == nslices ? alpha : rdiv;
    x[idx] = v;
  }
}

// u[m][q] = scale * linear interpolation in the row index of the predicted
// slices (value 0 at row -1, i.e. at t = 0 for a zero initial value; constant
// after the last slice row)
__global__ void time_interp_kernel(const float* __restrict__ y, const int* __restrict__ rows, int nslices,
                                   long long M, long long N, double scale, double* __restrict__ u) {
  const long long total = M * N;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long m = idx / N, q = idx % N;
    int s = 0;
    while (s < nslices && rows[s] < m) ++s;
    double v;
    if (s == nslices) v = y[(long long)(nslices - 1) * N + q];
    else if (rows[s] == m) v = y[(long long)s * N + q];
    else {
      const double r0 = s == 0 ? -1.0 : (double)rows[s - 1];
      const double y0 = s == 0 ? 0.0 : (double)y[(long long)(s - 1) * N + q];
      const double r1 = rows[s], y1 = y[(long long)s * N + q];
      v = y0 + (y1 - y0) * ((double)m - r0) / (r1 - r0);
    }
    u[idx] = scale * v;
  }
}

static inline int grid_of(long long total) {
  long long g = (total + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

hipError_t launch_gather_slices(const double* b, const int* rows, int nslices, long long N, double scale,
                                float alpha, float rdiv, float* x, hipStream_t s) {
  hipLaunchKernelGGL(gather_slices_kernel, dim3(grid_of((long long)(nslices + 2) * N)), dim3(256), 0, s, b, rows,
                     nslices, N, scale, alpha, rdiv, x);
  return hipGetLastError();
}

hipError_t launch_time_interp(const float* y, const int* rows, int nslices, long long M, long long N, double scale,
                              double* u, hipStream_t s) {
  hipLaunchKernelGGL(time_interp_kernel, dim3(grid_of(M * N)), dim3(256), 0, s, y, rows, nslices, M, N, scale, u);
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
}  // namespace

struct mgwr_net {
  std::vector<int> ch;              // channels c_0..c_L
  std::vector<size_t> woff, boff;   // parameter offsets (floats)
  size_t nparam = 0;
  long long cap_bhw = 0;            // capacity of the bound activation buffers (batch*H*W)
  int maxc = 0;
  bool bound = false;
  hipStream_t stream = nullptr;
  float* params = nullptr;          // caller-owned master weights
  uint16_t* wbf = nullptr;
  float *grad = nullptr, *m = nullptr, *v = nullptr;
  std::vector<float*> act;          // act[l]: output of layer l (l = 0..L-1), [cap_bhw * c_{l+1}]
  float *gbuf0 = nullptr, *gbuf1 = nullptr;
  double* norms = nullptr;          // per-sample loss norms (cap 4096 samples)
  size_t total = 0;
  long long layout(long long bhw, std::vector<size_t>* offs) const {
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off += (bytes + 255) & ~size_t(255);
      return o;
    };
    std::vector<size_t> o;
    o.push_back(take(nparam * 2));        // wbf
    o.push_back(take(nparam * 4));        // grad
    o.push_back(take(nparam * 4));        // m
    o.push_back(take(nparam * 4));        // v
    for (size_t l = 0; l + 1 < ch.size(); ++l) o.push_back(take((size_t)bhw * ch[l + 1] * 4));
    o.push_back(take((size_t)bhw * maxc * 4));
    o.push_back(take((size_t)bhw * maxc * 4));
    o.push_back(take(4096 * 2 * sizeof(double)));
    if (offs) *offs = o;
    return (long long)off;
  }
};

namespace {

// Forward pass; activations of every layer stay in net->act.
int net_forward(mgwr_net* net, const float* x, int B, int H, int W) {
  const int L = (int)net->ch.size() - 1;
  const float* in = x;
  for (int l = 0; l < L; ++l) {
    const long long total = (long long)B * net->ch[l + 1] * H * W;
    hipLaunchKernelGGL(conv_fwd_kernel, dim3(grid_of(total)), dim3(256), 0, net->stream, in,
                       net->wbf + net->woff[l], net->params + net->boff[l], net->act[l], B, net->ch[l], net->ch[l + 1],
                       H, W, l + 1 < L ? 1 : 0);
    NET_TRY(hipGetLastError());
    in = net->act[l];
  }
  return MGWR_OK;
}

int check_net(mgwr_net* net, int B, int H, int W) {
  if (!net || !net->bound) return nfail(MGWR_ERR_STATE, "network is not bound");
  if (B < 1 || H < 1 || W < 1 || (long long)B * H * W > net->cap_bhw || B > 4096)
    return nfail(MGWR_ERR_INVALID_ARG, "batch*H*W exceeds the bound capacity");
  return MGWR_OK;
}

}  // namespace

extern "C" {

int mgwr_net_create(int layers, const int* channels, mgwr_net** out) {
  if (!out || !channels || layers < 1 || layers > 16) return nfail(MGWR_ERR_INVALID_ARG, "bad network shape");
  *out = nullptr;
  mgwr_net* net = new (std::nothrow) mgwr_net();
  if (!net) return nfail(MGWR_ERR_INVALID_ARG, "out of host memory");
  for (int l = 0; l <= layers; ++l) {
    if (channels[l] < 1 || channels[l] > 1024) {
      delete net;
      return nfail(MGWR_ERR_INVALID_ARG, "channel counts must lie in [1, 1024]");
    }
    net->ch.push_back(channels[l]);
    net->maxc = std::max(net->maxc, channels[l]);
  }
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
  const int L = (int)net->ch.size() - 1;
  net->act.assign(L, nullptr);
  for (int l = 0; l < L; ++l) net->act[l] = (float*)(w + o[4 + l]);
  net->gbuf0 = (float*)(w + o[4 + L]);
  net->gbuf1 = (float*)(w + o[5 + L]);
  net->norms = (double*)(w + o[6 + L]);
  net->cap_bhw = max_bhw;
  net->total = (size_t)need;
  NET_TRY(hipMemsetAsync(net->m, 0, net->nparam * 4, net->stream));
  NET_TRY(hipMemsetAsync(net->v, 0, net->nparam * 4, net->stream));
  hipLaunchKernelGGL(round_bf16_kernel, dim3(grid_of((long long)net->nparam)), dim3(256), 0, net->stream,
                     net->params, net->wbf, (long long)net->nparam);
  NET_TRY(hipGetLastError());
  NET_TRY(hipStreamSynchronize(net->stream));
  net->bound = true;
  return MGWR_OK;
}

int mgwr_net_sync_weights(mgwr_net* net) {
  if (!net || !net->bound) return nfail(MGWR_ERR_STATE, "network is not bound");
  hipLaunchKernelGGL(round_bf16_kernel, dim3(grid_of((long long)net->nparam)), dim3(256), 0, net->stream,
                     net->params, net->wbf, (long long)net->nparam);
  NET_TRY(hipGetLastError());
  return MGWR_OK;
}

int mgwr_net_forward(mgwr_net* net, const float* x, int B, int H, int W, float* y) {
  int rc = check_net(net, B, H, W);
  if (rc) return rc;
  if (!x || !y) return nfail(MGWR_ERR_INVALID_ARG, "null array");
  if ((rc = net_forward(net, x, B, H, W))) return rc;
  const int L = (int)net->ch.size() - 1;
  NET_TRY(hipMemcpyAsync(y, net->act[L - 1], (size_t)B * net->ch[L] * H * W * 4, hipMemcpyDeviceToDevice,
                         net->stream));
  return MGWR_OK;
}

int mgwr_net_gradient(mgwr_net* net, const float* x, const float* target, int B, int H, int W, float* grad_out,
                      double* loss_host) {
  int rc = check_net(net, B, H, W);
  if (rc) return rc;
  if (!x || !target) return nfail(MGWR_ERR_INVALID_ARG, "null array");
  if ((rc = net_forward(net, x, B, H, W))) return rc;
  const int L = (int)net->ch.size() - 1;
  const long long HW = (long long)H * W;
  const long long per = (long long)net->ch[L] * HW;
  hipLaunchKernelGGL(loss_norms_kernel, dim3(B), dim3(256), 0, net->stream, net->act[L - 1], target, per, net->norms);
  NET_TRY(hipGetLastError());
  hipLaunchKernelGGL(loss_grad_kernel, dim3(grid_of(B * per)), dim3(256), 0, net->stream, net->act[L - 1], target,
                     net->norms, net->gbuf0, B, per, 1e-30);
  NET_TRY(hipGetLastError());
  float* dcur = net->gbuf0;
  float* dnext = net->gbuf1;
  for (int l = L - 1; l >= 0; --l) {
    const float* in = l == 0 ? x : net->act[l - 1];
    const int cin = net->ch[l], cout = net->ch[l + 1];
    hipLaunchKernelGGL(conv_bwd_weight_kernel, dim3(cout * (cin * 9 + 1)), dim3(256), 0, net->stream, dcur, in,
                       net->grad + net->woff[l], net->grad + net->boff[l], B, cin, cout, H, W);
    NET_TRY(hipGetLastError());
    if (l > 0) {
      hipLaunchKernelGGL(conv_bwd_data_kernel, dim3(grid_of((long long)B * cin * HW)), dim3(256), 0, net->stream,
                         dcur, net->wbf + net->woff[l], net->act[l - 1], dnext, B, cin, cout, H, W, 1);
      NET_TRY(hipGetLastError());
      std::swap(dcur, dnext);
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

int mgwr_net_adam_step(mgwr_net* net, float lr, float beta1, float beta2, float eps, int step) {
  if (!net || !net->bound) return nfail(MGWR_ERR_STATE, "network is not bound");
  if (step < 1) return nfail(MGWR_ERR_INVALID_ARG, "step counts from 1");
  const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_of((long long)net->nparam)), dim3(256), 0, net->stream, net->params,
                     net->grad, net->m, net->v, net->wbf, (long long)net->nparam, lr, beta1, beta2, eps, c1, c2);
  NET_TRY(hipGetLastError());
  return MGWR_OK;
}

int mgwr_net_destroy(mgwr_net* net) {
  delete net;
  return MGWR_OK;
}

}  // extern "C"

// internal: forward pass for the solver's warm start (x, y are net buffers)
namespace mgwr {
int net_infer(mgwr_net* net, const float* x, int H, int W, const float** y) {
  int rc = check_net(net, 1, H, W);
  if (rc) return rc;
  if ((rc = net_forward(net, x, 1, H, W))) return rc;
  *y = net->act[net->ch.size() - 2];
  return MGWR_OK;
}
int net_in_channels(const mgwr_net* net) { return net->ch.front(); }
int net_out_channels(const mgwr_net* net) { return net->ch.back(); }
hipStream_t net_stream(const mgwr_net* net) { return net->stream; }
}  // namespace mgwr
