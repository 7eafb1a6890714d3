// Application of the additive Schwarz preconditioner
//     z = S r = sum_B R_B^T P_B R_B r  (+ diagonal scaling)   (Sec. 3.1, Eq. 6)
// with the element-block local inverses P_B kept as dense m x m blocks
// instead of being summed into one global sparse S (Algorithm 1 prolongates
// them into S; keeping them apart costs the same bytes per product and lets
// the gather, the dense product and the scatter stream each block once).
//
// Phase 1 (one pass over P): per block, gather r_B = R_B r into LDS and
// write y_B = P_B r_B.  P_B is symmetric, so lane i accumulates
// sum_j P_B[j][i] r_B[j] and the lanes of a wave read row j contiguously.
// Phase 2 (pull): every unknown sums the y_B entries of the blocks that
// contain it, in a fixed order (no atomics, bitwise reproducible), and adds
// its diagonal-scaling term.
#include "dev_common.h"
#include "k_schwarz.h"

namespace fc {

template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<uint16_t>(uint16_t v) { return bf16_to_f32(v); }

// Gathered residual entry of block slot t (optionally r - alpha q).
__device__ __forceinline__ double gather_r(const double* r, const double* q, double alpha,
                                           int64_t dof) {
  double v = r[dof];
  if (q) v = fma(-alpha, q[dof], v);
  return v;
}

// m > 64: one workgroup of 64*ceil(m/64) threads per block.
template <typename T>
__global__ __launch_bounds__(256) void k_schwarz_large(
    const T* __restrict__ P, const int32_t* __restrict__ elem_nodes,
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
  const T* Pb = P + blk * (int64_t)m * m + i;
  if constexpr (sizeof(T) == 8) {
    double acc0 = 0.0, acc1 = 0.0;
    int j = 0;
#pragma unroll 8
    for (; j + 1 < m; j += 2) {
      acc0 = fma((double)__builtin_nontemporal_load(Pb + (int64_t)j * m), rB[j], acc0);
      acc1 = fma((double)__builtin_nontemporal_load(Pb + (int64_t)(j + 1) * m), rB[j + 1], acc1);
    }
    if (j < m) acc0 = fma((double)__builtin_nontemporal_load(Pb + (int64_t)j * m), rB[j], acc0);
    y[blk * m + i] = acc0 + acc1;
  } else {
    float acc0 = 0.f, acc1 = 0.f;
    int j = 0;
#pragma unroll 8
    for (; j + 1 < m; j += 2) {
      acc0 = fmaf(to_f32<T>(__builtin_nontemporal_load(Pb + (int64_t)j * m)), (float)rB[j], acc0);
      acc1 = fmaf(to_f32<T>(__builtin_nontemporal_load(Pb + (int64_t)(j + 1) * m)),
                  (float)rB[j + 1], acc1);
    }
    if (j < m) acc0 = fmaf(to_f32<T>(__builtin_nontemporal_load(Pb + (int64_t)j * m)), (float)rB[j], acc0);
    y[blk * m + i] = (double)(acc0 + acc1);
  }
}

// m <= 64: each wave handles floor(64/m) blocks, one lane per output.
template <typename T>
__global__ __launch_bounds__(256) void k_schwarz_small(
    const T* __restrict__ P, const int32_t* __restrict__ elem_nodes,
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
  const T* Pb = P + blk * (int64_t)m * m + i;
  if constexpr (sizeof(T) == 8) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j)
      acc = fma((double)__builtin_nontemporal_load(Pb + (int64_t)j * m), rb[j], acc);
    y[blk * m + i] = acc;
  } else {
    float acc = 0.f;
    for (int j = 0; j < m; ++j)
      acc = fmaf(to_f32<T>(__builtin_nontemporal_load(Pb + (int64_t)j * m)), (float)rb[j], acc);
    y[blk * m + i] = (double)acc;
  }
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

template <typename T>
static hipError_t phase1(const fc_precond_s& pc, const T* P, const double* r, const double* q,
                         const CgScalars* sc, hipStream_t s) {
  const fc_problem_s& pb = *pc.pb;
  if (pc.n_blocks == 0) return hipSuccess;
  if (pc.m > 64) {
    const int threads = 64 * ((pc.m + 63) / 64);
    hipLaunchKernelGGL(k_schwarz_large<T>, dim3((unsigned)pc.n_blocks), dim3(threads), 0, s, P,
                       pb.elem_nodes, pc.block_elem, pc.nn, pc.bdim, pc.m, r, q, sc, pc.y,
                       pc.n_blocks);
  } else {
    const int bpw = 64 / pc.m;
    const int64_t per_wg = 4 * (int64_t)bpw;
    const int64_t nwg = (pc.n_blocks + per_wg - 1) / per_wg;
    hipLaunchKernelGGL(k_schwarz_small<T>, dim3((unsigned)nwg), dim3(256), 0, s, P,
                       pb.elem_nodes, pc.block_elem, pc.nn, pc.bdim, pc.m, r, q, sc, pc.y,
                       pc.n_blocks);
  }
  return hipGetLastError();
}

hipError_t launch_schwarz_phase1(const fc_precond_s& pc, int precision, const double* r,
                                 const double* q, const CgScalars* sc, hipStream_t s) {
  switch (precision) {
    case 0: return phase1<double>(pc, pc.P, r, q, sc, s);
    case 1: return phase1<float>(pc, pc.P32, r, q, sc, s);
    case 2: return phase1<uint16_t>(pc, pc.Pbf, r, q, sc, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_schwarz_apply(const fc_precond_s& pc, const double* r, double* z,
                                hipStream_t s) {
  hipError_t e = launch_schwarz_phase1(pc, 0, r, nullptr, nullptr, s);
  if (e != hipSuccess) return e;
  const int64_t n = pc.pb->n_dofs;
  hipLaunchKernelGGL(k_schwarz_pull, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pc.y,
                     pc.inv_ptr, pc.inv_idx, pc.fallback, pc.bdim, n, r, z);
  return hipGetLastError();
}

}  // namespace fc
