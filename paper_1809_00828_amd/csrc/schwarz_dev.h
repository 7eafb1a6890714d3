// Device helpers of the Schwarz block products shared by the single-problem
// and batched kernels.
#pragma once
#include "dev_common.h"

namespace fc {

// Elements per block of the wrapped-diagonal symmetric layout.
__host__ __device__ __forceinline__ int64_t sym_block_stride_dev(int m) {
  return (int64_t)(m / 2 + 1) * m;
}

template <typename T>
__device__ __forceinline__ double to_f64(T v);
template <>
__device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <>
__device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double to_f64<uint16_t>(uint16_t v) { return (double)bf16_to_f32(v); }

template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<uint16_t>(uint16_t v) { return bf16_to_f32(v); }
template <>
__device__ __forceinline__ float to_f32<double>(double v) { return (float)v; }

// Accumulator: FP64 for FP64 storage, FP32 for the low-precision copies.
template <typename T>
struct Acc {
  using type = float;
};
template <>
struct Acc<double> {
  using type = double;
};

template <typename A, typename T>
__device__ __forceinline__ A madd(T a, double r, A acc) {
  if constexpr (sizeof(A) == 8)
    return fma(to_f64<T>(a), r, acc);
  else
    return fmaf(to_f32<T>(a), (float)r, acc);
}

__device__ __forceinline__ double gather_r(const double* r, const double* q, double alpha,
                                           int64_t dof) {
  double v = r[dof];
  if (q) v = fma(-alpha, q[dof], v);
  return v;
}

// Rows of the wrapped-diagonal layout staged through LDS per chunk: 16 KB
// of LDS, 8 rows of FP64 or 16 of FP32.
template <typename T>
struct StageRows {
  static constexpr int value = sizeof(T) == 8 ? 8 : 16;
};

// Symmetric product of one block (m > 64) by a whole workgroup, one output
// row i per thread (threads with i >= m take part in the barriers only):
// chunks of stored rows are loaded with coalesced non-temporal loads, every
// thread its own entry, written to LDS, and the rotated entries are read
// back from LDS, so HBM and L2 see each stored entry exactly once.  rB holds
// the block's gathered right-hand side (m entries, in LDS).  The stored
// entries are streamed non-temporally (each is read once per product).
template <typename T, typename RB>
__device__ __forceinline__ double sym_block_staged(const T* __restrict__ Qb, const RB* rB,
                                                   int m, int i,
                                                   T (*tile)[256]) {
  using A = typename Acc<T>::type;
  constexpr int kStageRows = StageRows<T>::value;
  const bool act = i < m;
  const int h = m / 2;
  const bool even = (m & 1) == 0;
  A acc0 = 0, acc1 = 0;
  int ip = i, im = i;
  for (int k0 = 0; k0 <= h; k0 += kStageRows) {
    T v[kStageRows];
#pragma unroll
    for (int kk = 0; kk < kStageRows; ++kk) {
      const int k = k0 + kk;
      const T* src = Qb + (int64_t)k * m + i;
      v[kk] = (act && k <= h) ? __builtin_nontemporal_load(src) : T(0);
    }
    __syncthreads();   // previous chunk's rotated reads are done
#pragma unroll
    for (int kk = 0; kk < kStageRows; ++kk) tile[kk][i] = v[kk];
    __syncthreads();
    if (act) {
#pragma unroll
      for (int kk = 0; kk < kStageRows; ++kk) {
        const int k = k0 + kk;
        if (k > h) break;
        if (k == 0) {
          acc0 = madd<A>(v[kk], rB[i], acc0);
          continue;
        }
        ip = (ip + 1 == m) ? 0 : ip + 1;
        im = (im == 0) ? m - 1 : im - 1;
        acc0 = madd<A>(v[kk], rB[ip], acc0);
        if (!(even && k == h)) acc1 = madd<A>(tile[kk][im], rB[im], acc1);
      }
    }
  }
  return (double)acc0 + (double)acc1;
}

// Wrapped-diagonal symmetric product for one block row i (0 <= i < m).
template <typename T>
__device__ __forceinline__ double sym_row(const T* __restrict__ Qb, const double* rb, int m,
                                          int i) {
  using A = typename Acc<T>::type;
  const int h = m / 2;
  const bool even = (m & 1) == 0;
  A acc0 = 0, acc1 = 0;
  acc0 = madd<A>(Qb[i], rb[i], acc0);
  int ip = i, im = i;
#pragma unroll 4
  for (int k = 1; k <= h; ++k) {
    ip = (ip + 1 == m) ? 0 : ip + 1;   // (i + k) mod m
    im = (im == 0) ? m - 1 : im - 1;   // (i - k) mod m
    const T* row = Qb + (int64_t)k * m;
    acc0 = madd<A>(row[i], rb[ip], acc0);
    if (!(even && k == h)) acc1 = madd<A>(row[im], rb[im], acc1);
  }
  return (double)acc0 + (double)acc1;
}

// Dense product for one block row i.
template <typename T>
__device__ __forceinline__ double dense_row(const T* __restrict__ Pb, const double* rb, int m,
                                            int i) {
  using A = typename Acc<T>::type;
  A acc0 = 0, acc1 = 0;
  int j = 0;
#pragma unroll 8
  for (; j + 1 < m; j += 2) {
    acc0 = madd<A>(__builtin_nontemporal_load(Pb + (int64_t)j * m + i), rb[j], acc0);
    acc1 = madd<A>(__builtin_nontemporal_load(Pb + (int64_t)(j + 1) * m + i), rb[j + 1], acc1);
  }
  if (j < m) acc0 = madd<A>(__builtin_nontemporal_load(Pb + (int64_t)j * m + i), rb[j], acc0);
  return (double)acc0 + (double)acc1;
}

}  // namespace fc
