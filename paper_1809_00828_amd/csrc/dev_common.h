// Device helpers shared by the libfc kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fc_internal.h"

namespace fc {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;   // MI355X: 8 XCDs, workgroups dispatched round-robin

// Map the hardware workgroup id to a logical tile id so that the
// workgroups that land on one XCD (ids congruent mod 8) process one
// contiguous range of tiles and share that XCD's L2.  A bijection on
// [0, nwg) for any nwg.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nwg) {
  const uint32_t x = bid % kNumXcd, j = bid / kNumXcd;
  const uint32_t q = nwg / kNumXcd, r = nwg % kNumXcd;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// Deterministic sum over the workgroup (blockDim.x a multiple of 64, at
// most 1024).  Every thread receives the result.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* lds /* >= 16 */) {
  v = group_sum<kWave>(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  __syncthreads();
  if (l == 0) lds[w] = v;
  __syncthreads();
  T t = 0;
  for (int i = 0; i < nw; ++i) t += lds[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ double load_relaxed(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-workgroup election: every workgroup calls this once after writing
// its partial results; returns true in exactly one workgroup, the last to
// arrive, which may then read every partial.  The ticket is reset for the
// next use by the winner.
__device__ __forceinline__ bool last_block(uint32_t* ticket, uint32_t nblocks,
                                           int* lds_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                          __HIP_MEMORY_SCOPE_AGENT);
    int win = (old == nblocks - 1) ? 1 : 0;
    if (win) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *lds_flag = win;
  }
  __syncthreads();
  bool win = *lds_flag != 0;
  if (win) __threadfence();
  return win;
}

// Fixed-order sum of n partials by the whole workgroup.
__device__ __forceinline__ double sum_partials(const double* part, int n,
                                               double* lds) {
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) t += load_relaxed(part + i);
  return block_sum(t, lds);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}

}  // namespace fc
