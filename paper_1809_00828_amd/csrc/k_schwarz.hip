// Application of the additive Schwarz preconditioner
//     z = S r = sum_B R_B^T P_B R_B r  (+ diagonal scaling)   (Sec. 3.1, Eq. 6)
// with the element-block local inverses P_B kept as dense blocks instead of
// being summed into one global sparse S (Algorithm 1 prolongates them into
// S; keeping them apart lets the gather, the block product and the scatter
// stream each block once).
//
// Phase 1 (one pass over the local inverses): per block, gather
// r_B = R_B r into LDS and write y_B = P_B r_B.
//   * Symmetric (default) layout.  P_B is symmetric, so only its m(m+1)/2
//     distinct entries are stored, as "wrapped diagonals":
//         Q_B[k][i] = P_B[i][(i + k) mod m],   k = 0 .. floor(m/2).
//     Thread i then needs, for every k, Q_B[k][i] (the entry P[i][i+k]) and
//     Q_B[k][(i - k) mod m] (the entry P[i][i-k] by symmetry): both are
//     reads of the same stored row k, one of them rotated, so every wave
//     load is a contiguous segment, no cross-lane reduction is needed, and
//     HBM delivers each stored entry once (the rotated read hits the cache
//     line the direct read of a neighbouring thread brought in).  When m is
//     even the row k = m/2 holds every pair twice and is used once.
//   * Dense layout: lane i accumulates sum_j P_B[j][i] r_B[j] (row j of a
//     symmetric matrix is its column j) reading P_B row by row.
// Phase 2 (pull): every unknown sums the y_B entries of the blocks that
// contain it, in a fixed order (no atomics, bitwise reproducible), and adds
// its diagonal-scaling term.
#include <cstdlib>

#include "dev_common.h"
#include "k_schwarz.h"

namespace fc {

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

// m > 64: one workgroup of 64*ceil(m/64) threads per block.
template <typename T, bool kSym>
__global__ __launch_bounds__(256) void k_schwarz_large(
    const T* __restrict__ P, int64_t block_stride, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    const double* __restrict__ r, const double* __restrict__ q,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks) {
  __shared__ double rB[256];
  if (sc && sc->done) return;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  if (blk >= n_blocks) return;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int i = threadIdx.x;
  const int64_t e = block_elem[blk];
  if (i < m) {
    const int64_t dof = (int64_t)elem_nodes[e * nn + i / bd] * bd + (i % bd);
    rB[i] = gather_r(r, q, alpha, dof);
  }
  __syncthreads();
  if (i >= m) return;
  const T* Pb = P + blk * block_stride;
  y[blk * m + i] = kSym ? sym_row<T>(Pb, rB, m, i) : dense_row<T>(Pb, rB, m, i);
}

// m > 64, symmetric layout staged through LDS: chunks of kRows stored rows
// are loaded with coalesced non-temporal loads (every thread its own entry),
// written to LDS, and the rotated entries are read back from LDS, so HBM
// and L2 see each stored entry exactly once.
constexpr int kStageRows = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_schwarz_sym_staged(
    const T* __restrict__ P, int64_t block_stride, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    const double* __restrict__ r, const double* __restrict__ q,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks) {
  using A = typename Acc<T>::type;
  __shared__ double rB[256];
  __shared__ T tile[kStageRows][256];
  if (sc && sc->done) return;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  if (blk >= n_blocks) return;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int i = threadIdx.x;
  const bool act = i < m;
  const int64_t e = block_elem[blk];
  if (act) {
    const int64_t dof = (int64_t)elem_nodes[e * nn + i / bd] * bd + (i % bd);
    rB[i] = gather_r(r, q, alpha, dof);
  }
  const T* Qb = P + blk * block_stride;
  const int h = m / 2;
  const bool even = (m & 1) == 0;
  A acc0 = 0, acc1 = 0;
  int ip = i, im = i;
  for (int k0 = 0; k0 <= h; k0 += kStageRows) {
    T v[kStageRows];
#pragma unroll
    for (int kk = 0; kk < kStageRows; ++kk) {
      const int k = k0 + kk;
      v[kk] = (act && k <= h) ? __builtin_nontemporal_load(Qb + (int64_t)k * m + i) : T(0);
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
  if (act) y[blk * m + i] = (double)acc0 + (double)acc1;
}

// m <= 64: each wave handles floor(64/m) blocks, one lane per output row.
template <typename T, bool kSym>
__global__ __launch_bounds__(256) void k_schwarz_small(
    const T* __restrict__ P, int64_t block_stride, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    const double* __restrict__ r, const double* __restrict__ q,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks) {
  __shared__ double rB[4][64];
  if (sc && sc->done) return;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int bpw = 64 / m;
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  const int lb = l / m, i = l % m;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t blk = (tile * 4 + w) * bpw + lb;
  const bool active = lb < bpw && blk < n_blocks;
  if (active) {
    const int64_t e = block_elem[blk];
    const int64_t dof = (int64_t)elem_nodes[e * nn + i / bd] * bd + (i % bd);
    rB[w][l] = gather_r(r, q, alpha, dof);
  }
  __syncthreads();
  if (!active) return;
  const double* rb = &rB[w][lb * m];
  const T* Pb = P + blk * block_stride;
  y[blk * m + i] = kSym ? sym_row<T>(Pb, rb, m, i) : dense_row<T>(Pb, rb, m, i);
}

// Phase 2: z_i = sum over blocks containing i of y_B[slot] + fb_i * r_i.
__global__ __launch_bounds__(256) void k_schwarz_pull(
    const double* __restrict__ y, const int32_t* __restrict__ inv_ptr,
    const int32_t* __restrict__ inv_idx, const double* __restrict__ fb, int bd,
    int64_t n_dofs, const double* __restrict__ r, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_dofs) return;
  const int64_t node = i / bd;
  const int c = (int)(i - node * bd);
  double s = 0.0;
  for (int32_t e = inv_ptr[node]; e < inv_ptr[node + 1]; ++e) s += y[(int64_t)inv_idx[e] + c];
  z[i] = fma(fb[i], r[i], s);
}

// Wrapped-diagonal copy: Q[blk][k][i] = P[blk][i][(i+k) mod m], k <= m/2.
template <typename T>
__global__ void k_pack_sym(const double* __restrict__ P, T* __restrict__ Q, int m,
                           int64_t n_blocks) {
  const int h = m / 2;
  const int64_t per = (int64_t)(h + 1) * m;
  const int64_t total = per * n_blocks;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = t / per;
    const int64_t rem = t - blk * per;
    const int k = (int)(rem / m), i = (int)(rem - (int64_t)k * m);
    int j = i + k;
    if (j >= m) j -= m;
    const double v = P[blk * (int64_t)m * m + (int64_t)i * m + j];
    if constexpr (sizeof(T) == 8) {
      Q[t] = v;
    } else if constexpr (sizeof(T) == 4) {
      Q[t] = (float)v;
    } else {
      // FP64 -> BF16 through FP32, round to nearest even
      uint32_t u = __float_as_uint((float)v);
      u += 0x7fffu + ((u >> 16) & 1u);
      Q[t] = (T)(u >> 16);
    }
  }
}

int64_t sym_block_stride(int m) { return (int64_t)(m / 2 + 1) * m; }

hipError_t launch_pack_sym(const double* P, void* Q, int precision, int m, int64_t n_blocks,
                           hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  dim3 g(8192), b(256);
  switch (precision) {
    case 0: hipLaunchKernelGGL(k_pack_sym<double>, g, b, 0, s, P, (double*)Q, m, n_blocks); break;
    case 1: hipLaunchKernelGGL(k_pack_sym<float>, g, b, 0, s, P, (float*)Q, m, n_blocks); break;
    case 2: hipLaunchKernelGGL(k_pack_sym<uint16_t>, g, b, 0, s, P, (uint16_t*)Q, m, n_blocks); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool kSym>
static hipError_t phase1(const fc_precond_s& pc, const T* P, const double* r, const double* q,
                         const CgScalars* sc, hipStream_t s) {
  const fc_problem_s& pb = *pc.pb;
  if (pc.n_blocks == 0) return hipSuccess;
  const int64_t stride = kSym ? sym_block_stride(pc.m) : (int64_t)pc.m * pc.m;
  static const int variant = [] {
    const char* v = std::getenv("FC_SCHWARZ_STAGED");
    return v ? std::atoi(v) : 1;
  }();
  if (pc.m > 64) {
    const int threads = 64 * ((pc.m + 63) / 64);
    if (kSym && variant)
      hipLaunchKernelGGL((k_schwarz_sym_staged<T>), dim3((unsigned)pc.n_blocks), dim3(threads),
                         0, s, P, stride, pb.elem_nodes, pc.block_elem, pc.nn, pc.bdim, pc.m, r,
                         q, sc, pc.y, pc.n_blocks);
    else
      hipLaunchKernelGGL((k_schwarz_large<T, kSym>), dim3((unsigned)pc.n_blocks), dim3(threads),
                         0, s, P, stride, pb.elem_nodes, pc.block_elem, pc.nn, pc.bdim, pc.m, r,
                         q, sc, pc.y, pc.n_blocks);
  } else {
    const int bpw = 64 / pc.m;
    const int64_t per_wg = 4 * (int64_t)bpw;
    const int64_t nwg = (pc.n_blocks + per_wg - 1) / per_wg;
    hipLaunchKernelGGL((k_schwarz_small<T, kSym>), dim3((unsigned)nwg), dim3(256), 0, s, P, stride,
                       pb.elem_nodes, pc.block_elem, pc.nn, pc.bdim, pc.m, r, q, sc, pc.y,
                       pc.n_blocks);
  }
  return hipGetLastError();
}

hipError_t launch_schwarz_phase1(const fc_precond_s& pc, int precision, const double* r,
                                 const double* q, const CgScalars* sc, hipStream_t s) {
  switch (precision) {
    case 0:
      if (pc.Q) return phase1<double, true>(pc, pc.Q, r, q, sc, s);
      return phase1<double, false>(pc, pc.P, r, q, sc, s);
    case 1:
      if (!pc.Q32) return hipErrorInvalidValue;
      return phase1<float, true>(pc, pc.Q32, r, q, sc, s);
    case 2:
      if (!pc.Qbf) return hipErrorInvalidValue;
      return phase1<uint16_t, true>(pc, pc.Qbf, r, q, sc, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_schwarz_pull(const fc_precond_s& pc, const double* r, double* z,
                               hipStream_t s) {
  const int64_t n = pc.pb->n_dofs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_schwarz_pull, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pc.y,
                     pc.inv_ptr, pc.inv_idx, pc.fallback, pc.bdim, n, r, z);
  return hipGetLastError();
}

hipError_t launch_schwarz_apply(const fc_precond_s& pc, const double* r, double* z,
                                hipStream_t s) {
  hipError_t e = launch_schwarz_phase1(pc, 0, r, nullptr, nullptr, s);
  if (e != hipSuccess) return e;
  return launch_schwarz_pull(pc, r, z, s);
}

}  // namespace fc
