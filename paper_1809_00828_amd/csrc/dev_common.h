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

// Lattice box of row node `row`: for every direction the range of lattice
// indices of the functions whose support meets the row's support (a vertex
// index reaches one cell to each side, an interior index only its cell).
struct RowBox {
  int lo[3], len[3];
};

__device__ __forceinline__ RowBox row_box(int64_t row, const LatticeInfo lat) {
  RowBox b;
  int64_t r = row;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = 0;
    b.len[k] = 1;
    if (k < lat.dim) {
      const int g = (int)(r % lat.n1);
      r /= lat.n1;
      if (g % lat.p == 0) {
        const int lo = max(0, g - lat.p), hi = min(lat.n1 - 1, g + lat.p);
        b.lo[k] = lo;
        b.len[k] = hi - lo + 1;
      } else {
        b.lo[k] = (g / lat.p) * lat.p;
        b.len[k] = lat.p + 1;
      }
    }
  }
  return b;
}

// column of the k-th block of the row (first direction fastest)
__device__ __forceinline__ int lattice_col(const RowBox& b, int k, int n1) {
  const int kx = k % b.len[0], r = k / b.len[0];
  const int ky = r % b.len[1], kz = r / b.len[1];
  return (b.lo[0] + kx) + n1 * ((b.lo[1] + ky) + n1 * (b.lo[2] + kz));
}

__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}

}  // namespace fc
