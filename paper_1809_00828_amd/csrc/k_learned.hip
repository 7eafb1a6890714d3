// Learned coarse correction: a small 3-D U-Net on the coarse vertex grid,
// with its own forward, backward and Adam kernels, the transfers between
// unknowns and the coarse grid, and training data taken from the solver.
//
// Network (4 levels, widths c0..c3, in_ch input channels): 'same' 3x3x3
// convolutions with zero padding, ReLU, average pooling over the existing
// children, nearest upsampling, additive skips:
//   enc_l: h = relu(conv_b(relu(conv_a(x))))   (l = 0..2, pool after)
//   bottom: relu(conv_b(relu(conv_a(.))))
//   dec_l: h = relu(conv_a(up(h))) + s_l; h = relu(conv_b(h))  (l = 2,1,0)
//   head:  conv(c0 -> 1)
// Parameters: one flat FP32 master vector (per convolution W[co][ci][27]
// then b[co]; tap = dz*9 + dy*3 + dx), a BF16 copy used by every
// convolution, FP32 activations and FP32 accumulation.
//
// Convolution kernels: every lane owns one output voxel and 8 output
// channels, with the BF16 weights arriving through wave-uniform loads.
// The data gradient is the same kernel with the weights transposed and the
// taps mirrored; the weight gradient is one workgroup per (co, ci) pair
// reducing over voxels (fixed order, no atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "dev_common.h"
#include "learned.h"

namespace fc {

constexpr int kConvT = 64;   // lanes per workgroup (one wave)
constexpr int kWgradSlots = 4096;   // (co, ci, chunk) partials of the weight gradient

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// y[b][o][v] = act(bias[o] + sum_{i,t} w(o,i,t) x[b][i][v + off_t])
// One wave per workgroup, one voxel and CoT output channels per lane (CoT
// shrinks on the coarse levels so that the launch still spans the chip).  The
// weights are read at wave-uniform addresses from rows of 14 dwords (27
// BF16 taps and one pad per (co, ci) pair), so they arrive through scalar
// loads and feed the FMAs as scalar operands; the 27 neighbour values of
// an input channel are loaded once and reused for all CoT outputs.
// kTrans: w(o,i,t) = W[i][o][26-t] (data gradient of a convolution whose
// input width is this kernel's Co), no bias, no activation.
template <bool kTrans, int kCoT>
__global__ __launch_bounds__(kConvT) void k_conv3d(const float* __restrict__ x, int Ci,
                                                   const uint32_t* __restrict__ W,
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ y, int Co, int N,
                                                   int relu) {
  const int V = N * N * N;
  const int b = blockIdx.z;
  const int o0 = blockIdx.y * kCoT;
  const int v = blockIdx.x * kConvT + threadIdx.x;
  const bool active = v < V;
  const int vv = active ? v : 0;
  const int xx = vv % N, yy = (vv / N) % N, zz = vv / (N * N);
  float acc[kCoT];
#pragma unroll
  for (int o = 0; o < kCoT; ++o) acc[o] = (!kTrans && bias && o0 + o < Co) ? bias[o0 + o] : 0.f;
  const float* xb = x + (int64_t)b * Ci * V;
  for (int i = 0; i < Ci; ++i) {
    const float* xi = xb + (int64_t)i * V;
    float xv[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const int z2 = zz + k / 9 - 1, y2 = yy + (k / 3) % 3 - 1, x2 = xx + k % 3 - 1;
      const bool in = z2 >= 0 && z2 < N && y2 >= 0 && y2 < N && x2 >= 0 && x2 < N;
      xv[k] = in ? xi[(z2 * N + y2) * N + x2] : 0.f;
    }
#pragma unroll
    for (int o = 0; o < kCoT; ++o) {
      if (o0 + o >= Co) break;
      const int64_t row = kTrans ? ((int64_t)i * Co + (o0 + o)) : ((int64_t)(o0 + o) * Ci + i);
      const uint32_t* wr = W + row * kRowDw;
#pragma unroll
      for (int j = 0; j < kRowDw; ++j) {
        const uint32_t pr = wr[j];
        const float wlo = __uint_as_float(pr << 16), whi = __uint_as_float(pr & 0xffff0000u);
        const int k0 = 2 * j, k1 = 2 * j + 1;
        acc[o] = fmaf(wlo, xv[kTrans ? 26 - k0 : k0], acc[o]);
        if (k1 < 27) acc[o] = fmaf(whi, xv[kTrans ? 26 - k1 : k1], acc[o]);
      }
    }
  }
  if (!active) return;
  float* yb = y + (int64_t)b * Co * V;
#pragma unroll
  for (int o = 0; o < kCoT; ++o)
    if (o0 + o < Co) yb[(int64_t)(o0 + o) * V + v] = relu ? fmaxf(acc[o], 0.f) : acc[o];
}

// BF16 rows of 14 dwords from the FP32 weights W[rows][27]
__global__ void k_pack_w(const float* __restrict__ w, uint32_t* __restrict__ out, int64_t rows) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < rows * kRowDw;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / kRowDw;
    const int j = (int)(t % kRowDw);
    const uint32_t lo = f2bf(w[row * 27 + 2 * j]);
    const uint32_t hi = 2 * j + 1 < 27 ? f2bf(w[row * 27 + 2 * j + 1]) : 0u;
    out[t] = lo | (hi << 16);
  }
}

// Weight gradient, gw[co][ci][t] = sum_{b,v} g[b][co][v] x[b][ci][v + off_t]
// and gb[co] = sum g, in two deterministic passes: workgroup (ci, co, c)
// sums chunk c of the (b, v) range into 28 partials, then one thread per
// (co, ci, t) adds the chunks in order.
__global__ __launch_bounds__(256) void k_conv3d_wgrad(const float* __restrict__ x, int Ci,
                                                      const float* __restrict__ g, int Co, int B,
                                                      int D, int H, int Wd, int nchunk,
                                                      float* __restrict__ part) {
  __shared__ float red[16];
  const int ci = blockIdx.x, co = blockIdx.y, c = blockIdx.z;
  const int V = D * H * Wd;
  const int64_t total = (int64_t)B * V;
  const int64_t len = (total + nchunk - 1) / nchunk;
  const int64_t lo = (int64_t)c * len, hi = lo + len < total ? lo + len : total;
  float acc[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) acc[k] = 0.f;
  float accb = 0.f;
  for (int64_t idx = lo + threadIdx.x; idx < hi; idx += blockDim.x) {
    const int b = (int)(idx / V), v = (int)(idx % V);
    const float gv = g[((int64_t)b * Co + co) * V + v];
    accb += gv;
    if (gv == 0.f) continue;
    const int xx = v % Wd, yy = (v / Wd) % H, zz = v / (Wd * H);
    const float* xi = x + ((int64_t)b * Ci + ci) * V;
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
      const int z2 = zz + dz, y2 = yy + dy, x2 = xx + dx;
      if (z2 >= 0 && z2 < D && y2 >= 0 && y2 < H && x2 >= 0 && x2 < Wd)
        acc[k] = fmaf(gv, xi[(z2 * H + y2) * Wd + x2], acc[k]);
    }
  }
  float* out = part + (((int64_t)co * Ci + ci) * nchunk + c) * 28;
  for (int k = 0; k < 27; ++k) {
    const float s = block_sum(acc[k], red);
    if (threadIdx.x == 0) out[k] = s;
  }
  const float sb = block_sum(accb, red);
  if (threadIdx.x == 0) out[27] = sb;
}

__global__ void k_wgrad_reduce(const float* __restrict__ part, int Ci, int Co, int nchunk,
                               float* __restrict__ gw, float* __restrict__ gb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = (int64_t)Co * Ci;
  if (t >= rows * 28) return;
  const int64_t row = t / 28;
  const int k = (int)(t % 28);
  const float* p = part + row * nchunk * 28 + k;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += p[(int64_t)c * 28];
  const int co = (int)(row / Ci), ci = (int)(row % Ci);
  if (k < 27) gw[row * 27 + k] = s;
  else if (ci == 0) {
    // the bias gradient is the same sum for every ci; keep ci = 0's
    gb[co] = s;
  }
}

// average over the existing children: (D,H,W) -> ceil halves
__global__ void k_pool(const float* __restrict__ x, float* __restrict__ y, int BC, int D, int H,
                       int Wd) {
  const int d = (D + 1) / 2, h = (H + 1) / 2, w = (Wd + 1) / 2;
  const int64_t total = (int64_t)BC * d * h * w;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bc = t / ((int64_t)d * h * w);
    const int rem = (int)(t % ((int64_t)d * h * w));
    const int X = rem % w, Y = (rem / w) % h, Z = rem / (w * h);
    float s = 0.f;
    int cnt = 0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
          const int z = 2 * Z + a, yy = 2 * Y + b, xx = 2 * X + c;
          if (z < D && yy < H && xx < Wd) {
            s += x[bc * D * H * Wd + ((int64_t)z * H + yy) * Wd + xx];
            ++cnt;
          }
        }
    y[t] = s / (float)cnt;
  }
}

__global__ void k_pool_bwd(const float* __restrict__ gy, float* __restrict__ gx, int BC, int D,
                           int H, int Wd) {
  const int d = (D + 1) / 2, h = (H + 1) / 2, w = (Wd + 1) / 2;
  const int64_t total = (int64_t)BC * D * H * Wd;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bc = t / ((int64_t)D * H * Wd);
    const int rem = (int)(t % ((int64_t)D * H * Wd));
    const int xx = rem % Wd, yy = (rem / Wd) % H, z = rem / (Wd * H);
    const int X = xx / 2, Y = yy / 2, Z = z / 2;
    const int cz = (2 * Z + 1 < D) ? 2 : 1, cy = (2 * Y + 1 < H) ? 2 : 1, cx = (2 * X + 1 < Wd) ? 2 : 1;
    gx[t] = gy[bc * d * h * w + ((int64_t)Z * h + Y) * w + X] / (float)(cz * cy * cx);
  }
}

// nearest upsampling (d,h,w) -> (D,H,W): y[i] = x[i/2]; with accumulate
// into y (mode 1) for the additive use
__global__ void k_upsample(const float* __restrict__ x, float* __restrict__ y, int BC, int D,
                           int H, int Wd) {
  const int d = (D + 1) / 2, h = (H + 1) / 2, w = (Wd + 1) / 2;
  const int64_t total = (int64_t)BC * D * H * Wd;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bc = t / ((int64_t)D * H * Wd);
    const int rem = (int)(t % ((int64_t)D * H * Wd));
    const int xx = rem % Wd, yy = (rem / Wd) % H, z = rem / (Wd * H);
    y[t] = x[bc * d * h * w + ((int64_t)(z / 2) * h + yy / 2) * w + xx / 2];
  }
}

__global__ void k_upsample_bwd(const float* __restrict__ gy, float* __restrict__ gx, int BC,
                               int D, int H, int Wd) {
  const int d = (D + 1) / 2, h = (H + 1) / 2, w = (Wd + 1) / 2;
  const int64_t total = (int64_t)BC * d * h * w;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bc = t / ((int64_t)d * h * w);
    const int rem = (int)(t % ((int64_t)d * h * w));
    const int X = rem % w, Y = (rem / w) % h, Z = rem / (w * h);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
          const int z = 2 * Z + a, yy = 2 * Y + b, xx = 2 * X + c;
          if (z < D && yy < H && xx < Wd) s += gy[bc * D * H * Wd + ((int64_t)z * H + yy) * Wd + xx];
        }
    gx[t] = s;
  }
}

// a = a + b
__global__ void k_add(float* __restrict__ a, const float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] += b[i];
}

// c = a + b
__global__ void k_add3(float* __restrict__ c, const float* __restrict__ a,
                       const float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    c[i] = a[i] + b[i];
}

// g *= (act > 0)
__global__ void k_relu_mask(float* __restrict__ g, const float* __restrict__ act, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!(act[i] > 0.f)) g[i] = 0.f;
}

// mean squared error: per-workgroup partial sums and g = 2 (y - t) / n
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y,
                                             const float* __restrict__ t, float* __restrict__ g,
                                             int64_t n, double* __restrict__ partial) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    s += (double)d * d;
    g[i] = 2.f * d / (float)n;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// omb1 = 1 - beta1, omb2 = 1 - beta2, c1 = 1 - beta1^t, c2 = 1 - beta2^t are
// formed in FP64 by the host: in FP32 the differences from 1 lose about
// 1e-5 of their value to cancellation (1 - 0.999f is off by 1.3e-5
// relative), which would bias every update by that much.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float omb1,
                       float omb2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

static inline dim3 grid1(int64_t n) {
  return dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192));
}

// ------------------------------------------------------------ network
static const int kLayerIO[15][2] = {{-1, 0}, {0, 0}, {0, 1}, {1, 1}, {1, 2}, {2, 2}, {2, 3},
                                    {3, 3}, {3, 2}, {2, 2}, {2, 1}, {1, 1}, {1, 0}, {0, 0},
                                    {0, -2}};

void Net::init(const int32_t* c, int32_t in_channels) {
  for (int i = 0; i < 4; ++i) ch[i] = c[i];
  in_ch = in_channels;
  int64_t off = 0;
  for (int l = 0; l < 15; ++l) {
    ci[l] = kLayerIO[l][0] == -1 ? in_ch : ch[kLayerIO[l][0]];
    co[l] = kLayerIO[l][1] == -2 ? 1 : ch[kLayerIO[l][1]];
    woff[l] = off;
    off += (int64_t)ci[l] * co[l] * 27;
    boff[l] = off;
    off += co[l];
  }
  nparam = off;
  int64_t dw = 0;
  for (int l = 0; l < 15; ++l) {
    wpoff[l] = dw;
    dw += (int64_t)ci[l] * co[l] * kRowDw;
  }
  nwpk = dw;
}

int64_t net_param_count(const int32_t* c, int32_t in_channels) {
  Net n;
  n.init(c, in_channels);
  return n.nparam;
}

// Output channels per lane: the largest of 8, 4, 2, 1 that still gives at
// least 1024 workgroups (the coarse levels hold few voxels).
template <bool kTrans>
static hipError_t launch_conv(const float* x, int cin, const uint32_t* W, const float* bias,
                              float* y, int cout, int N, int B, int relu, hipStream_t s) {
  const int V = N * N * N;
  const int64_t vb = (V + kConvT - 1) / kConvT;
  int cot = 8;
  while (cot > 1 && vb * ((cout + cot - 1) / cot) * B < 1024) cot /= 2;
  dim3 g((unsigned)vb, (unsigned)((cout + cot - 1) / cot), (unsigned)B);
  switch (cot) {
    case 8:
      hipLaunchKernelGGL((k_conv3d<kTrans, 8>), g, dim3(kConvT), 0, s, x, cin, W, bias, y, cout,
                         N, relu);
      break;
    case 4:
      hipLaunchKernelGGL((k_conv3d<kTrans, 4>), g, dim3(kConvT), 0, s, x, cin, W, bias, y, cout,
                         N, relu);
      break;
    case 2:
      hipLaunchKernelGGL((k_conv3d<kTrans, 2>), g, dim3(kConvT), 0, s, x, cin, W, bias, y, cout,
                         N, relu);
      break;
    default:
      hipLaunchKernelGGL((k_conv3d<kTrans, 1>), g, dim3(kConvT), 0, s, x, cin, W, bias, y, cout,
                         N, relu);
  }
  return hipGetLastError();
}

static hipError_t conv_fwd(const Net& net, int l, const float* x, float* y, int B, int N, bool relu,
                           hipStream_t s) {
  return launch_conv<false>(x, net.ci[l], net.wpk + net.wpoff[l], net.p + net.boff[l], y,
                            net.co[l], N, B, relu ? 1 : 0, s);
}

// data gradient of layer l: gx (Ci channels) from gy (Co channels)
static hipError_t conv_bwd_data(const Net& net, int l, const float* gy, float* gx, int B, int N,
                                hipStream_t s) {
  return launch_conv<true>(gy, net.co[l], net.wpk + net.wpoff[l], nullptr, gx, net.ci[l], N, B,
                           0, s);
}

static hipError_t conv_bwd_weight(Net& net, NetWs& ws, int l, const float* x, const float* gy,
                                  int B, int N, hipStream_t s) {
  const int Ci = net.ci[l], Co = net.co[l];
  const int64_t total = (int64_t)B * N * N * N;
  const int64_t pairs = (int64_t)Ci * Co;
  // chunks of at least 1024 (b, v) points, at most ws.wslots partial rows
  int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(ws.wslots / pairs, total / 1024));
  hipLaunchKernelGGL(k_conv3d_wgrad, dim3(Ci, Co, (unsigned)nchunk), dim3(256), 0, s, x, Ci, gy,
                     Co, B, N, N, N, (int)nchunk, ws.wpart);
  const int64_t nt = pairs * 28;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, ws.wpart,
                     Ci, Co, (int)nchunk, net.g + net.woff[l], net.g + net.boff[l]);
  return hipGetLastError();
}

fc_status NetWs::ensure(const Net& net, int B_, int N0) {
  if (B_ <= capB && N0 == N[0] && buf) return FC_OK;
  release();
  B = B_;
  capB = B_;
  N[0] = N0;
  for (int l = 1; l < 4; ++l) N[l] = (N[l - 1] + 1) / 2;
  // per-level tensor sizes (max channels of that level) for every saved
  // activation and two gradient scratch tensors per level
  int64_t total = 0;
  auto vox = [&](int l) { return (int64_t)N[l] * N[l] * N[l]; };
  for (int l = 0; l < 4; ++l) {
    // widths present at level l: its own, the pooled input from above (or
    // the network input) and the upsampled tensor from below
    int64_t cmax = net.ch[l];
    cmax = std::max<int64_t>(cmax, l == 0 ? net.in_ch : net.ch[l - 1]);
    if (l < 3) cmax = std::max<int64_t>(cmax, net.ch[l + 1]);
    for (int k = 0; k < kSlots; ++k) {
      off[l][k] = total;
      total += (int64_t)B * cmax * vox(l);
    }
  }
  off_y = total;
  total += 2 * (int64_t)B * vox(0);   // output and its gradient
  hipError_t e = hipMalloc(&buf, total * sizeof(float));
  if (e != hipSuccess) {
    buf = nullptr;
    set_error("network workspace allocation failed");
    return FC_E_NOMEM;
  }
  if (hipMalloc(&partial, 1024 * sizeof(double)) != hipSuccess) return FC_E_NOMEM;
  // partial rows of the weight gradient: at least one per (co, ci) pair
  wslots = kWgradSlots;
  for (int l = 0; l < 15; ++l) wslots = std::max<int64_t>(wslots, (int64_t)net.ci[l] * net.co[l]);
  if (hipMalloc(&wpart, (size_t)wslots * 28 * sizeof(float)) != hipSuccess) return FC_E_NOMEM;
  return FC_OK;
}

void NetWs::release() {
  if (buf) (void)hipFree(buf);
  if (partial) (void)hipFree(partial);
  if (wpart) (void)hipFree(wpart);
  buf = nullptr;
  partial = nullptr;
  wpart = nullptr;
  capB = 0;
}

// slots per level: 0 in, 1 a, 2 b (skip), 3 u (up), 4 da, 5 m, 6 db,
// 7, 8 gradient scratch
hipError_t net_forward(const Net& net, NetWs& ws, const float* x, int B, hipStream_t s) {
  const int* N = ws.N;
  hipError_t e;
  const float* in = x;
  for (int l = 0; l < 3; ++l) {
    float* a = ws.t(l, 1);
    float* b = ws.t(l, 2);
    if ((e = conv_fwd(net, 2 * l, in, a, B, N[l], true, s)) != hipSuccess) return e;
    if ((e = conv_fwd(net, 2 * l + 1, a, b, B, N[l], true, s)) != hipSuccess) return e;
    float* nxt = ws.t(l + 1, 0);
    const int64_t bc = (int64_t)B * net.ch[l];
    hipLaunchKernelGGL(k_pool, grid1(bc * ws.vox(l + 1)), dim3(256), 0, s, b, nxt, (int)bc, N[l],
                       N[l], N[l]);
    in = nxt;
  }
  if ((e = conv_fwd(net, 6, in, ws.t(3, 1), B, N[3], true, s)) != hipSuccess) return e;
  if ((e = conv_fwd(net, 7, ws.t(3, 1), ws.t(3, 2), B, N[3], true, s)) != hipSuccess) return e;
  const float* h = ws.t(3, 2);
  int hc = net.ch[3];
  for (int l = 2; l >= 0; --l) {
    float* u = ws.t(l, 3);
    const int64_t bc = (int64_t)B * hc;
    hipLaunchKernelGGL(k_upsample, grid1(bc * ws.vox(l)), dim3(256), 0, s, h, u, (int)bc, N[l],
                       N[l], N[l]);
    const int la = 8 + 2 * (2 - l), lb = la + 1;
    float* da = ws.t(l, 4);
    if ((e = conv_fwd(net, la, u, da, B, N[l], true, s)) != hipSuccess) return e;
    float* m = ws.t(l, 5);
    const int64_t n = (int64_t)B * net.ch[l] * ws.vox(l);
    hipLaunchKernelGGL(k_add3, grid1(n), dim3(256), 0, s, m, da, ws.t(l, 2), n);
    float* db = ws.t(l, 6);
    if ((e = conv_fwd(net, lb, m, db, B, N[l], true, s)) != hipSuccess) return e;
    h = db;
    hc = net.ch[l];
  }
  return conv_fwd(net, 14, h, ws.y(), B, N[0], false, s);
}

// Backward from gy (B,1,N0^3) into net.g (parameters); x is the input.
hipError_t net_backward(Net& net, NetWs& ws, const float* x, float* gy, int B, hipStream_t s) {
  const int* N = ws.N;
  hipError_t e;
  // head
  float* g = ws.t(0, 7);
  if ((e = conv_bwd_weight(net, ws, 14, ws.t(0, 6), gy, B, N[0], s)) != hipSuccess) return e;
  if ((e = conv_bwd_data(net, 14, gy, g, B, N[0], s)) != hipSuccess) return e;
  std::vector<float*> gskip(3, nullptr);
  int gc = net.ch[0];
  for (int l = 0; l < 3; ++l) {
    const int la = 8 + 2 * (2 - l), lb = la + 1;
    const int64_t n = (int64_t)B * net.ch[l] * ws.vox(l);
    hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(256), 0, s, g, ws.t(l, 6), n);
    if ((e = conv_bwd_weight(net, ws, lb, ws.t(l, 5), g, B, N[l], s)) != hipSuccess) return e;
    float* gm = ws.t(l, 8);
    if ((e = conv_bwd_data(net, lb, g, gm, B, N[l], s)) != hipSuccess) return e;
    // gm flows to the skip (kept in slot 8) and to da
    float* gda = ws.t(l, 7);
    (void)hipMemcpyAsync(gda, gm, n * sizeof(float), hipMemcpyDeviceToDevice, s);
    gskip[l] = gm;
    hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(256), 0, s, gda, ws.t(l, 4), n);
    if ((e = conv_bwd_weight(net, ws, la, ws.t(l, 3), gda, B, N[l], s)) != hipSuccess) return e;
    // data gradient of up_a lands on the upsampled tensor (Ci = width below)
    float* gu = ws.t(l, 3);   // the upsampled input is no longer needed
    if ((e = conv_bwd_data(net, la, gda, gu, B, N[l], s)) != hipSuccess) return e;
    const int cbelow = net.ci[la];
    float* gnext = ws.t(l + 1, 7);
    const int64_t bc = (int64_t)B * cbelow;
    hipLaunchKernelGGL(k_upsample_bwd, grid1(bc * ws.vox(l + 1)), dim3(256), 0, s, gu, gnext,
                       (int)bc, N[l], N[l], N[l]);
    g = gnext;
    gc = cbelow;
  }
  (void)gc;
  // bottom
  {
    const int64_t n = (int64_t)B * net.ch[3] * ws.vox(3);
    hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(256), 0, s, g, ws.t(3, 2), n);
    if ((e = conv_bwd_weight(net, ws, 7, ws.t(3, 1), g, B, N[3], s)) != hipSuccess) return e;
    float* g2 = ws.t(3, 8);
    if ((e = conv_bwd_data(net, 7, g, g2, B, N[3], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(256), 0, s, g2, ws.t(3, 1), n);
    if ((e = conv_bwd_weight(net, ws, 6, ws.t(3, 0), g2, B, N[3], s)) != hipSuccess) return e;
    g = ws.t(3, 7);
    if ((e = conv_bwd_data(net, 6, g2, g, B, N[3], s)) != hipSuccess) return e;
  }
  for (int l = 2; l >= 0; --l) {
    const int64_t bc = (int64_t)B * net.ch[l];
    const int64_t n = bc * ws.vox(l);
    float* gb = ws.t(l, 7);
    // gradient of pool input, plus the skip's gradient
    hipLaunchKernelGGL(k_pool_bwd, grid1(n), dim3(256), 0, s, g, gb, (int)bc, N[l], N[l], N[l]);
    hipLaunchKernelGGL(k_add, grid1(n), dim3(256), 0, s, gb, gskip[l], n);
    hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(256), 0, s, gb, ws.t(l, 2), n);
    if ((e = conv_bwd_weight(net, ws, 2 * l + 1, ws.t(l, 1), gb, B, N[l], s)) != hipSuccess) return e;
    float* g2 = ws.t(l, 8);
    if ((e = conv_bwd_data(net, 2 * l + 1, gb, g2, B, N[l], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(256), 0, s, g2, ws.t(l, 1), n);
    const float* xin = l == 0 ? x : ws.t(l, 0);
    if ((e = conv_bwd_weight(net, ws, 2 * l, xin, g2, B, N[l], s)) != hipSuccess) return e;
    if (l > 0) {
      g = ws.t(l, 7);   // reuse: data gradient into the pooled input of level l
      if ((e = conv_bwd_data(net, 2 * l, g2, g, B, N[l], s)) != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t net_mse(NetWs& ws, const float* target, float* gy, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1024), dim3(256), 0, s, ws.y(), target, gy, n, ws.partial);
  return hipGetLastError();
}

hipError_t net_adam(Net& net, float lr, int64_t step, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, (double)step));
  const float c2 = (float)(1.0 - std::pow(b2, (double)step));
  hipLaunchKernelGGL(k_adam, grid1(net.nparam), dim3(256), 0, s, net.p, net.g, net.m, net.v,
                     net.nparam, lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2),
                     1e-8f, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return net_sync_bf16(net, s);
}

hipError_t net_sync_bf16(Net& net, hipStream_t s) {
  for (int l = 0; l < 15; ++l) {
    const int64_t rows = (int64_t)net.ci[l] * net.co[l];
    hipLaunchKernelGGL(k_pack_w, grid1(rows * kRowDw), dim3(256), 0, s, net.p + net.woff[l],
                       net.wpk + net.wpoff[l], rows);
  }
  return hipGetLastError();
}

}  // namespace fc
