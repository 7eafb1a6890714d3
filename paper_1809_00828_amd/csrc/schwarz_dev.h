// Device helpers of the Schwarz block products shared by the single-problem
// and batched kernels.
#pragma once
#include "dev_common.h"

namespace fc {

// Elements per block of the wrapped-diagonal symmetric layout.
__host__ __device__ __forceinline__ int64_t sym_block_stride_dev(int m) {
  return (int64_t)(m / 2 + 1) * m;
}

// Offset of stored entry (k, i) = P_B[i][(i + k) mod m] of a block in the
// wrapped-diagonal layout.  m > 64 (one block per workgroup): stored row by
// stored row.  m <= 64 (one lane per column i): stored rows 2j and 2j + 1
// interleaved column by column, so a lane's two entries are adjacent and
// one two-wide load; an odd last stored row follows alone.
__host__ __device__ __forceinline__ int64_t sym_offset(int k, int i, int m) {
  if (m > 64) return (int64_t)k * m + i;
  const int npair = (m / 2 + 1) & ~1;   // stored rows that come in pairs
  return k < npair ? (int64_t)(k & ~1) * m + 2 * i + (k & 1) : (int64_t)k * m + i;
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

// Symmetric product of one block (m > 64) by a whole workgroup of
// 64 ceil(m/64) threads, one output row i per thread (threads with i >= m
// take part in the loads and barriers only).  A chunk of stored rows is one
// contiguous run of the block; every thread loads 16-byte pieces of it
// (half the load instructions of one entry per thread, and no idle lanes),
// non-temporally, into LDS, and each thread then reads its own entry and
// the rotated one back from LDS, so HBM and L2 see each stored entry exactly
// once.  The next chunk's loads are issued before the current chunk is
// summed.  rB holds the block's gathered right-hand side (m entries, in
// LDS).  tile (16-byte aligned) holds kStageRows * m <= kStageRows * 256 entries,
// as tile[kk * m + j] for stored row k0 + kk.
template <typename T, typename RB>
__device__ __forceinline__ double sym_block_staged_runs(const T* __restrict__ Qb, const RB* rB,
                                                   int m, int i, T* tile) {
  using A = typename Acc<T>::type;
  constexpr int kStageRows = StageRows<T>::value;
  constexpr int V = 16 / sizeof(T);                // entries per 16-byte piece
  constexpr int kPer = kStageRows / V;             // pieces per thread per chunk (m <= threads)
  typedef T tv __attribute__((ext_vector_type(V), aligned(sizeof(T))));
  typedef T tva __attribute__((ext_vector_type(V), aligned(16)));
  const int nt = blockDim.x, t = threadIdx.x;
  const bool act = i < m;
  const int h = m / 2;
  const bool even = (m & 1) == 0;
  A acc0 = 0, acc1 = 0;
  int ip = i, im = i;
  // chunk k0's pieces are loaded while chunk k0 - kStageRows is summed
  auto load_chunk = [&](int k0, tv* v) {
    const int cnt = min(kStageRows, h + 1 - k0) * m;
    const T* src = Qb + (int64_t)k0 * m;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = (t + nt * u) * V;
      if (e + V <= cnt) {
        v[u] = __builtin_nontemporal_load(reinterpret_cast<const tv*>(src + e));
      } else {
#pragma unroll
        for (int c = 0; c < V; ++c) v[u][c] = e + c < cnt ? __builtin_nontemporal_load(src + e + c) : T(0);
      }
    }
  };
  tv v[kPer];
  load_chunk(0, v);
  for (int k0 = 0; k0 <= h; k0 += kStageRows) {
    const int cnt = min(kStageRows, h + 1 - k0) * m;   // entries of this chunk
    __syncthreads();   // previous chunk's reads are done
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = (t + nt * u) * V;
      if (e < cnt) *reinterpret_cast<tva*>(tile + e) = v[u];   // the pad past cnt is never read
    }
    __syncthreads();
    if (k0 + kStageRows <= h) load_chunk(k0 + kStageRows, v);
    if (act) {
#pragma unroll
      for (int kk = 0; kk < kStageRows; ++kk) {
        const int k = k0 + kk;
        if (k > h) break;
        const T* row = tile + kk * m;
        if (k == 0) {
          acc0 = madd<A>(row[i], rB[i], acc0);
          continue;
        }
        ip = (ip + 1 == m) ? 0 : ip + 1;
        im = (im == 0) ? m - 1 : im - 1;
        acc0 = madd<A>(row[i], rB[ip], acc0);
        if (!(even && k == h)) acc1 = madd<A>(row[im], rB[im], acc1);
      }
    }
  }
  return (double)acc0 + (double)acc1;
}

// The same with every thread loading its own entry of each stored row of
// the chunk (8-byte loads) and keeping it in a register; only the rotated
// entries are read back from LDS (tile[kk * 256 + j]).
template <typename T, typename RB>
__device__ __forceinline__ double sym_block_staged_rows(const T* __restrict__ Qb, const RB* rB,
                                                        int m, int i, T* tile) {
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
    for (int kk = 0; kk < kStageRows; ++kk) tile[kk * 256 + i] = v[kk];
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
        if (!(even && k == h)) acc1 = madd<A>(tile[kk * 256 + im], rB[im], acc1);
      }
    }
  }
  return (double)acc0 + (double)acc1;
}

// Wrapped-diagonal symmetric product for one block row i (0 <= i < m), in
// either layout of sym_offset.
template <typename T>
__device__ __forceinline__ double sym_row(const T* __restrict__ Qb, const double* rb, int m,
                                          int i) {
  using A = typename Acc<T>::type;
  const int h = m / 2;
  const bool even = (m & 1) == 0;
  A acc0 = 0, acc1 = 0;
  acc0 = madd<A>(Qb[sym_offset(0, i, m)], rb[i], acc0);
  int ip = i, im = i;
#pragma unroll 4
  for (int k = 1; k <= h; ++k) {
    ip = (ip + 1 == m) ? 0 : ip + 1;   // (i + k) mod m
    im = (im == 0) ? m - 1 : im - 1;   // (i - k) mod m
    acc0 = madd<A>(Qb[sym_offset(k, i, m)], rb[ip], acc0);
    if (!(even && k == h)) acc1 = madd<A>(Qb[sym_offset(k, im, m)], rb[im], acc1);
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
