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
// Convolution kernels: implicit GEMMs on the BF16 matrix cores (MFMA) with
// FP32 accumulation.  A workgroup stages a 4x4x4 brick of its input with a
// one-voxel halo in LDS, split into BF16 terms (three for the forward and
// data-gradient passes, which keeps FP32 accuracy with BF16 weights; two
// for the weight gradient), and runs the 27 taps from there.  The data
// gradient is the forward kernel on weights packed transposed with the taps
// mirrored; the weight gradient sums brick ranges into partials that a
// second kernel adds in a fixed order (no atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "dev_common.h"
#include "learned.h"

namespace fc {

constexpr int kWgradRanges = 512;   // brick ranges of one weight-gradient launch, at most

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------- MFMA convolutions
// Every convolution is an implicit GEMM on the 16x16x16 BF16 matrix cores
// with FP32 accumulation.  Operand layouts of v_mfma_f32_16x16x16_bf16 (one
// wave): lane l supplies A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j]
// [l % 16], j = 0..3, and holds D[4 (l / 16) + j][l % 16].
//
// A workgroup owns a brick of 4x4x4 voxels; its input, with a one-voxel
// halo (6x6x6), is staged once in LDS, already split into BF16 terms, and
// every tap of the stencil reads it there.  A 16-voxel row tile of the GEMM
// is one 4x4 (y, x) plane of the brick.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kHaloVox = 216;   // 6^3 halo voxels of a 4^3 brick

// v = h0 + h1 + h2 in BF16 with |v - (h0 + h1 + h2)| <= 2^-24 |v| (each
// term the BF16 rounding of what the earlier ones leave; the remainders are
// exact in FP32).  Products of BF16 numbers are exact in FP32, so three
// MFMAs over the three terms give the FP32-accurate product with a BF16
// weight.  Two terms leave 2^-16 |v|.
struct Split3 {
  uint16_t h[3];
};

__device__ __forceinline__ Split3 split3(float v) {
  Split3 r;
  r.h[0] = f2bf(v);
  const float ra = v - __uint_as_float((uint32_t)r.h[0] << 16);
  r.h[1] = f2bf(ra);
  const float rb = ra - __uint_as_float((uint32_t)r.h[1] << 16);
  r.h[2] = f2bf(rb);
  return r;
}

__device__ __forceinline__ void split2(float v, uint16_t& h0, uint16_t& h1) {
  h0 = f2bf(v);
  h1 = f2bf(v - __uint_as_float((uint32_t)h0 << 16));
}

// offset of tap t = dz*9 + dy*3 + dx in a 6x6x6 halo (taps past 26 are
// padding with zero weight and read the corner)
__device__ __forceinline__ int halo_tap_offset(int t) {
  if (t >= 27) return 0;
  const int dz = t / 9, r = t - 9 * dz, dy = r / 3;
  return dz * 36 + dy * 6 + (r - 3 * dy);
}

// Reduction layout of a convolution with cin input channels: chunks of cc
// channels (4, 8 or 16), each chunk a run of ksteps * 16 reduction indices
// k = tap * cc + c (c the channel within the chunk), zero weights past
// 27 * cc.
struct ConvK {
  int cc, nchunk, ksteps, krow;
};

inline ConvK conv_k(int cin) {
  ConvK g;
  g.cc = cin <= 4 ? 4 : cin <= 8 ? 8 : 16;
  g.nchunk = (cin + g.cc - 1) / g.cc;
  g.ksteps = (27 * g.cc + 15) / 16;
  g.krow = g.nchunk * g.ksteps * 16;
  return g;
}

// y[b][o][v] = act(bias[o] + sum_{i,t} w(o,i,t) x[b][i][v + off_t]) with the
// weights packed by k_pack_conv (rows o of krow BF16 values, chunks of kCc
// input channels) and the input split into three BF16 terms.  Workgroup:
// brick blockIdx.x (nb^3 per sample), output channels 16 blockIdx.y .. + 15
// (one column tile), sample blockIdx.z; wave w computes plane z = w of the
// brick.  Per chunk, the halo input and the tile's weights are staged in
// LDS, the loads of a thread all issued before the first is used.
template <int kCc>
__global__ __launch_bounds__(256) void k_conv3d(const float* __restrict__ x, int Ci, int nchunk,
                                                const uint16_t* __restrict__ W, int krow,
                                                const float* __restrict__ bias,
                                                float* __restrict__ y, int Co, int N, int nb,
                                                int relu) {
  constexpr int kRs = kCc + 4;                   // LDS row of a halo voxel (pad: banks)
  constexpr int kSteps = (27 * kCc + 15) / 16;
  constexpr int kWRow = kSteps * 16 + 4;         // LDS row of one output channel
  constexpr int kItems = kHaloVox * kCc / 4;     // (halo voxel, 4 channels) items
  constexpr int kIter = (kItems + 255) / 256;
  constexpr int kWItems = 16 * kSteps * 2;       // 8 weights per item
  constexpr int kWIter = (kWItems + 255) / 256;
  __shared__ __align__(16) uint16_t xs[3][kHaloVox * kRs];   // [term][voxel][channel]
  __shared__ __align__(16) uint16_t wl[16 * kWRow];          // [column][k]
  const int V = N * N * N;
  const int brick = blockIdx.x, b = blockIdx.z, o0 = blockIdx.y * 16;
  const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
  const int x0 = 4 * bx - 1, y0 = 4 * by - 1, z0 = 4 * bz - 1;   // halo corner
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, r16 = l & 15, kg = l >> 4;
  const int hv0 = (w * 6 + (r16 >> 2)) * 6 + (r16 & 3);   // this lane's A row, tap 0
  // one accumulator per input term (independent MFMA chains), added
  // smallest term first at the end
  f32x4 acc[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float* xb = x + (int64_t)b * Ci * V;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int c0 = ch * kCc;
    float v[kIter][4];
    int dst[kIter];
#pragma unroll
    for (int it = 0; it < kIter; ++it) {
      const int e = tid + 256 * it;
      const int q = e / kHaloVox, hv = e - q * kHaloVox;
      const int hz = hv / 36, hr = hv - 36 * hz, hy = hr / 6, hx = hr - 6 * hy;
      const int gz = z0 + hz, gy = y0 + hy, gx = x0 + hx;
      const bool in = e < kItems && gz >= 0 && gz < N && gy >= 0 && gy < N && gx >= 0 && gx < N;
      const float* src = xb + (int64_t)(c0 + 4 * q) * V + (in ? (gz * N + gy) * N + gx : 0);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[it][j] = (in && c0 + 4 * q + j < Ci) ? src[(int64_t)j * V] : 0.f;
      dst[it] = e < kItems ? hv * kRs + 4 * q : -1;
    }
    uint4 wv[kWIter];
    int wdst[kWIter];
#pragma unroll
    for (int it = 0; it < kWIter; ++it) {
      const int e = tid + 256 * it;
      const int r = e / (2 * kSteps), q = e - r * 2 * kSteps;
      wv[it] = uint4{0u, 0u, 0u, 0u};
      if (e < kWItems && o0 + r < Co)
        wv[it] = *reinterpret_cast<const uint4*>(W + (int64_t)(o0 + r) * krow +
                                                 (int64_t)ch * kSteps * 16 + 8 * q);
      wdst[it] = e < kWItems ? r * kWRow + 8 * q : -1;
    }
    __syncthreads();   // the previous chunk's reads are done
#pragma unroll
    for (int it = 0; it < kIter; ++it) {
      if (dst[it] < 0) continue;
      uint16_t h[3][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const Split3 sp = split3(v[it][j]);
        h[0][j] = sp.h[0];
        h[1][j] = sp.h[1];
        h[2][j] = sp.h[2];
      }
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        uint2 pk;
        pk.x = (uint32_t)h[s][0] | ((uint32_t)h[s][1] << 16);
        pk.y = (uint32_t)h[s][2] | ((uint32_t)h[s][3] << 16);
        *reinterpret_cast<uint2*>(&xs[s][dst[it]]) = pk;
      }
    }
#pragma unroll
    for (int it = 0; it < kWIter; ++it) {
      if (wdst[it] < 0) continue;
      *reinterpret_cast<uint2*>(&wl[wdst[it]]) = uint2{wv[it].x, wv[it].y};
      *reinterpret_cast<uint2*>(&wl[wdst[it] + 4]) = uint2{wv[it].z, wv[it].w};
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
      const int k = 16 * s + 4 * kg;
      const int t = k / kCc, c = k - t * kCc;
      const int a = (hv0 + halo_tap_offset(t)) * kRs + c;
      const bf16x4 bw = *reinterpret_cast<const bf16x4*>(&wl[r16 * kWRow + k]);
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        const bf16x4 av = *reinterpret_cast<const bf16x4*>(&xs[h][a]);
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bw, acc[h], 0, 0, 0);
      }
    }
  }
  // D[4 kg + j][r16]: voxel (y = kg, x = j) of plane w, channel o0 + r16
  const int gz = z0 + 1 + w, gy = y0 + 1 + kg, o = o0 + r16;
  if (gz >= N || gy >= N || o >= Co) return;
  const float bo = bias ? bias[o] : 0.f;
  float* yo = y + ((int64_t)b * Co + o) * V + (gz * N + gy) * N;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int gx = x0 + 1 + j;
    if (gx < N) {
      const float val = (acc[2][j] + acc[1][j]) + acc[0][j] + bo;
      yo[gx] = relu ? fmaxf(val, 0.f) : val;
    }
  }
}

// Packed BF16 weights of one layer for k_conv3d.  Forward (trans = 0): row
// o of Co rows, reduction over the Ci input channels, value W[o][i][t].
// Data gradient (trans = 1): row i of Ci rows, reduction over the Co output
// channels with the taps mirrored, value W[o][i][26 - t] (the adjoint of a
// 'same' convolution is the convolution with the mirrored stencil).
__global__ void k_pack_conv(const float* __restrict__ w, int Co, int Ci, int trans, int cc,
                            int ksteps, int krow, uint16_t* __restrict__ out) {
  const int rows = trans ? Ci : Co, cin = trans ? Co : Ci;
  const int64_t total = (int64_t)rows * krow;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / krow), k = (int)(e - (int64_t)r * krow);
    const int chunk = k / (ksteps * 16), kk = k - chunk * ksteps * 16;
    const int t = kk / cc, c = chunk * cc + kk % cc;
    float v = 0.f;
    if (t < 27 && c < cin)
      v = trans ? w[((int64_t)c * Ci + r) * 27 + 26 - t] : w[((int64_t)r * Ci + c) * 27 + t];
    out[e] = f2bf(v);
  }
}

// Weight gradient gw[o][i][t] = sum_{b,v} g[b][o][v] x[b][i][v + off_t] and
// gb[o] = sum g[b][o][v], on the matrix cores: rows o, columns the 16
// input channels i of one chunk per tap, reduction over the voxels of a
// brick (16 per step: one 4x4 plane), both operands split into two BF16
// terms and the three products above 2^-16 summed.  Workgroup: input
// channels 16 blockIdx.x .., output channels 32 blockIdx.y .., a range of
// bricks (over samples and space) blockIdx.z; wave w owns taps w, w + 4, ..
// (wave 3 also the bias, as a column of ones).  Each workgroup writes its
// sums to part[z][o][i][28] (slot 27 of i = 0: bias); k_wgrad_reduce adds
// the ranges in order (deterministic, no atomics).
__global__ __launch_bounds__(256, 2) void k_conv3d_wgrad(const float* __restrict__ x, int Ci,
                                                      const float* __restrict__ g, int Co,
                                                      int N, int nb, int64_t nbricks,
                                                      int64_t per, int Cip,
                                                      float* __restrict__ part) {
  // input terms by x shift: xs[term][dx][i][row (z, y) of the halo][4]
  // holds x at halo x = dx .. dx + 3, so each shifted 4-voxel run is one
  // aligned 8-byte read; rows of 148 values per channel spread the banks
  constexpr int kXRow = 148;
  constexpr int kGRow = 68;
  constexpr int kXItems = 16 * kHaloVox;
  constexpr int kXIter = (kXItems + 255) / 256;
  constexpr int kGIter = 32 * 64 / 256;
  __shared__ __align__(16) uint16_t xs[2][3][16 * kXRow];
  __shared__ __align__(16) uint16_t gs[2][32 * kGRow];   // [term][o][voxel]
  const int V = N * N * N, nb3 = nb * nb * nb;
  const int i0 = blockIdx.x * 16, o0 = blockIdx.y * 32;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, r16 = l & 15, kg = l >> 4;
  const bool two = o0 + 16 < Co;
  const bool with_bias = w == 3 && blockIdx.x == 0;
  f32x4 acc[7][2];
#pragma unroll
  for (int q = 0; q < 7; ++q) acc[q][0] = acc[q][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t lo = (int64_t)blockIdx.z * per;
  const int64_t hi = lo + per < nbricks ? lo + per : nbricks;
  // the raw values of one brick, loaded one brick ahead of the compute
  float xv[kXIter], gv[kGIter];
  auto load = [&](int64_t bi) {
    const int b = (int)(bi / nb3), brick = (int)(bi - (int64_t)b * nb3);
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int x0 = 4 * bx - 1, y0 = 4 * by - 1, z0 = 4 * bz - 1;
    const float* xb = x + (int64_t)b * Ci * V;
#pragma unroll
    for (int it = 0; it < kXIter; ++it) {
      const int e = tid + 256 * it;
      const int i = e / kHaloVox, hv = e - i * kHaloVox;
      const int hz = hv / 36, hr = hv - 36 * hz, hy = hr / 6, hx = hr - 6 * hy;
      const int gz = z0 + hz, gy = y0 + hy, gx = x0 + hx;
      xv[it] = (e < kXItems && i0 + i < Ci && gz >= 0 && gz < N && gy >= 0 && gy < N &&
                gx >= 0 && gx < N)
                   ? xb[(int64_t)(i0 + i) * V + (gz * N + gy) * N + gx]
                   : 0.f;
    }
    const float* gb = g + (int64_t)b * Co * V;
#pragma unroll
    for (int it = 0; it < kGIter; ++it) {
      const int e = tid + 256 * it;
      const int o = e >> 6, v = e & 63;
      const int gz = z0 + 1 + (v >> 4), gy = y0 + 1 + ((v >> 2) & 3), gx = x0 + 1 + (v & 3);
      gv[it] = (o0 + o < Co && gz < N && gy < N && gx < N)
                   ? gb[(int64_t)(o0 + o) * V + (gz * N + gy) * N + gx]
                   : 0.f;
    }
  };
  if (lo < hi) load(lo);
  for (int64_t bi = lo; bi < hi; ++bi) {
    __syncthreads();   // the previous brick's reads are done
#pragma unroll
    for (int it = 0; it < kXIter; ++it) {
      const int e = tid + 256 * it;
      if (e >= kXItems) continue;
      const int i = e / kHaloVox, hv = e - i * kHaloVox;
      const int hz = hv / 36, hr = hv - 36 * hz, hy = hr / 6, hx = hr - 6 * hy;
      uint16_t h0, h1;
      split2(xv[it], h0, h1);
      const int base = i * kXRow + (hz * 6 + hy) * 4 + hx;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int xq = hx - dx;
        if (xq >= 0 && xq < 4) {
          xs[0][dx][base - dx] = h0;
          xs[1][dx][base - dx] = h1;
        }
      }
    }
#pragma unroll
    for (int it = 0; it < kGIter; ++it) {
      const int e = tid + 256 * it;
      const int o = e >> 6, v = e & 63;
      uint16_t h0, h1;
      split2(gv[it], h0, h1);
      gs[0][o * kGRow + v] = h0;
      gs[1][o * kGRow + v] = h1;
    }
    __syncthreads();
    if (bi + 1 < hi) load(bi + 1);   // in flight during the products below
#pragma unroll 1
    for (int pz = 0; pz < 4; ++pz) {
      // A: g[o][voxels (y = kg, x = 0..3) of plane pz]
      const int ga = r16 * kGRow + 16 * pz + 4 * kg;
      const bf16x4 g0a = *reinterpret_cast<const bf16x4*>(&gs[0][ga]);
      const bf16x4 g1a = *reinterpret_cast<const bf16x4*>(&gs[1][ga]);
      const bf16x4 g0b = *reinterpret_cast<const bf16x4*>(&gs[0][ga + 16 * kGRow]);
      const bf16x4 g1b = *reinterpret_cast<const bf16x4*>(&gs[1][ga + 16 * kGRow]);
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        const int t = w + 4 * q;
        if (t < 27) {
          const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
          const int xa = r16 * kXRow + ((pz + dz) * 6 + kg + dy) * 4;
          const bf16x4 x0v = *reinterpret_cast<const bf16x4*>(&xs[0][dx][xa]);
          const bf16x4 x1v = *reinterpret_cast<const bf16x4*>(&xs[1][dx][xa]);
          acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g1a, x0v, acc[q][0], 0, 0, 0);
          acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g0a, x1v, acc[q][0], 0, 0, 0);
          acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g0a, x0v, acc[q][0], 0, 0, 0);
          if (two) {
            acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g1b, x0v, acc[q][1], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g0b, x1v, acc[q][1], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g0b, x0v, acc[q][1], 0, 0, 0);
          }
        } else if (with_bias) {
          const short one = (short)0x3f80;   // BF16 1.0
          const bf16x4 ones = {one, one, one, one};
          acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g1a, ones, acc[q][0], 0, 0, 0);
          acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g0a, ones, acc[q][0], 0, 0, 0);
          if (two) {
            acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g1b, ones, acc[q][1], 0, 0, 0);
            acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(g0b, ones, acc[q][1], 0, 0, 0);
          }
        }
      }
    }
  }
  // D[4 kg + j][r16]: output channel o0 + 16 ct + 4 kg + j, input channel
  // i0 + r16
  float* pz = part + (int64_t)blockIdx.z * Co * Cip * 28;
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int t = w + 4 * q;
    if (t >= 27 && !with_bias) continue;
    if (t >= 27 && r16 != 0) continue;
    const int tt = t < 27 ? t : 27;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int o = o0 + 16 * ct + 4 * kg + j;
        if (o < Co && (ct == 0 || two))
          pz[((int64_t)o * Cip + i0 + r16) * 28 + tt] = acc[q][ct][j];
      }
    }
  }
}

// gw[o][i][t] and gb[o] from the per-range sums: 16 outputs per workgroup
// of 256 threads, thread (slice, output) adds ranges slice, slice + 16, ..
// in order, then the 16 slice sums are added in order (deterministic).
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int Ci,
                                                      int Co, int Cip, int nrange,
                                                      float* __restrict__ gw,
                                                      float* __restrict__ gb) {
  __shared__ float sums[16][17];
  const int lane = threadIdx.x & 15, slice = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + lane;
  const int64_t nout = (int64_t)Co * Ci * 28;
  int o = 0, i = 0, t = 0;
  float s = 0.f;
  if (e < nout) {
    o = (int)(e / (Ci * 28));
    const int r = (int)(e - (int64_t)o * Ci * 28);
    i = r / 28;
    t = r - 28 * i;
    const int64_t stride = (int64_t)Co * Cip * 28;
    const float* p = part + ((int64_t)o * Cip + i) * 28 + t;
    for (int c = slice; c < nrange; c += 16) s += p[c * stride];
  }
  sums[slice][lane] = s;
  __syncthreads();
  if (slice != 0 || e >= nout || (t == 27 && i != 0)) return;
  float tot = 0.f;
  for (int k = 0; k < 16; ++k) tot += sums[k][lane];
  if (t < 27) gw[((int64_t)o * Ci + i) * 27 + t] = tot;
  else gb[o] = tot;
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
  int64_t e = 0;
  for (int l = 0; l < 15; ++l) {
    wfoff[l] = e;
    e += (int64_t)co[l] * conv_k(ci[l]).krow;
    wtoff[l] = e;
    e += (int64_t)ci[l] * conv_k(co[l]).krow;
  }
  nwpk = e;
}

int64_t net_param_count(const int32_t* c, int32_t in_channels) {
  Net n;
  n.init(c, in_channels);
  return n.nparam;
}

// One workgroup per 4^3 brick and 16 output channels; cin input channels
// with weights packed for that width.
static hipError_t launch_conv(const float* x, int cin, const uint16_t* W, const float* bias,
                              float* y, int cout, int N, int B, int relu, hipStream_t s) {
  const ConvK k = conv_k(cin);
  const int nb = (N + 3) / 4;
  dim3 g((unsigned)(nb * nb * nb), (unsigned)((cout + 15) / 16), (unsigned)B);
  if (k.cc == 4)
    hipLaunchKernelGGL(k_conv3d<4>, g, dim3(256), 0, s, x, cin, k.nchunk, W, k.krow, bias, y,
                       cout, N, nb, relu);
  else if (k.cc == 8)
    hipLaunchKernelGGL(k_conv3d<8>, g, dim3(256), 0, s, x, cin, k.nchunk, W, k.krow, bias, y,
                       cout, N, nb, relu);
  else
    hipLaunchKernelGGL(k_conv3d<16>, g, dim3(256), 0, s, x, cin, k.nchunk, W, k.krow, bias, y,
                       cout, N, nb, relu);
  return hipGetLastError();
}

static hipError_t conv_fwd(const Net& net, int l, const float* x, float* y, int B, int N, bool relu,
                           hipStream_t s) {
  return launch_conv(x, net.ci[l], net.wpk + net.wfoff[l], net.p + net.boff[l], y, net.co[l], N,
                     B, relu ? 1 : 0, s);
}

// data gradient of layer l: gx (Ci channels) from gy (Co channels)
static hipError_t conv_bwd_data(const Net& net, int l, const float* gy, float* gx, int B, int N,
                                hipStream_t s) {
  return launch_conv(gy, net.co[l], net.wpk + net.wtoff[l], nullptr, gx, net.ci[l], N, B, 0, s);
}

static int64_t wgrad_row_floats(int Ci, int Co) {
  return (int64_t)Co * ((Ci + 15) / 16 * 16) * 28;
}

// brick ranges of a weight-gradient launch: about 1024 workgroups
static int64_t wgrad_max_ranges(int Ci, int Co) {
  const int64_t tiles = (int64_t)((Ci + 15) / 16) * ((Co + 31) / 32);
  return std::min<int64_t>(kWgradRanges, std::max<int64_t>(1, 1024 / tiles));
}

static hipError_t conv_bwd_weight(Net& net, NetWs& ws, int l, const float* x, const float* gy,
                                  int B, int N, hipStream_t s) {
  const int Ci = net.ci[l], Co = net.co[l];
  const int nb = (N + 3) / 4;
  const int64_t nbricks = (int64_t)B * nb * nb * nb;
  const int nic = (Ci + 15) / 16, nop = (Co + 31) / 32;
  int64_t nrange = std::min<int64_t>(wgrad_max_ranges(Ci, Co), nbricks);
  const int64_t per = (nbricks + nrange - 1) / nrange;
  nrange = (nbricks + per - 1) / per;
  dim3 g((unsigned)nic, (unsigned)nop, (unsigned)nrange);
  hipLaunchKernelGGL(k_conv3d_wgrad, g, dim3(256), 0, s, x, Ci, gy, Co, N, nb, nbricks, per,
                     nic * 16, ws.wpart);
  const int64_t nt = (int64_t)Co * Ci * 28;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nt + 15) / 16)), dim3(256), 0, s, ws.wpart,
                     Ci, Co, nic * 16, (int)nrange, net.g + net.woff[l], net.g + net.boff[l]);
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
  // weight-gradient partials of the largest layer
  wslots = 0;
  for (int l = 0; l < 15; ++l)
    wslots = std::max<int64_t>(wslots, wgrad_max_ranges(net.ci[l], net.co[l]) *
                                           wgrad_row_floats(net.ci[l], net.co[l]));
  if (hipMalloc(&wpart, (size_t)wslots * sizeof(float)) != hipSuccess) return FC_E_NOMEM;
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
    const int ci = net.ci[l], co = net.co[l];
    const ConvK kf = conv_k(ci), kt = conv_k(co);
    hipLaunchKernelGGL(k_pack_conv, grid1((int64_t)co * kf.krow), dim3(256), 0, s,
                       net.p + net.woff[l], co, ci, 0, kf.cc, kf.ksteps, kf.krow,
                       net.wpk + net.wfoff[l]);
    hipLaunchKernelGGL(k_pack_conv, grid1((int64_t)ci * kt.krow), dim3(256), 0, s,
                       net.p + net.woff[l], co, ci, 1, kt.cc, kt.ksteps, kt.krow,
                       net.wpk + net.wtoff[l]);
  }
  return hipGetLastError();
}

}  // namespace fc
