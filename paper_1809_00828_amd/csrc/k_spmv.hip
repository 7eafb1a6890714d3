// Block-sparse (BSR) matrix-vector product y = A x for the assembled finite
// cell stiffness matrix (Sec. 3.1, Eq. 2); the product with A is half of
// every PCG iteration (Sec. 5.4 names the matrix-vector products as the
// dominant work of the solver).
//
// Layout (row-SoA BSR): the values of block row i are stored entry-major,
// val[rowptr[i]*B*B + e*L + k] for entry e of the k-th block of the row,
// so G lanes sweeping the blocks of one row read G consecutive values per
// entry.  A group of G lanes owns one block row; its partial sums are
// combined with a butterfly reduction.  Values and column indices are read
// once per product and streamed with non-temporal loads, which leaves the
// cache to the gathered x entries (neighbouring rows of the lattice share
// most of their columns).
#include "dev_common.h"
#include "k_spmv.h"

namespace fc {

template <int B, int G, typename T>
__global__ __launch_bounds__(256) void k_spmv_bsr(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, const double* __restrict__ x,
    double* __restrict__ y, int64_t n_rows, const CgScalars* sc,
    double* __restrict__ partial, CgScalars* scw) {
  constexpr int BB = B * B;
  constexpr int RPW = 256 / G;   // rows per workgroup
  __shared__ double lds[16];
  __shared__ int flag;
  const bool fused = partial != nullptr;
  if (fused && sc->done) return;
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t row = (int64_t)tile * RPW + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  double dot = 0.0;
  if (row < n_rows) {
    const int64_t base = rowptr[row];
    const int L = rowptr[row + 1] - (int32_t)base;
    const T* v = val + base * BB;
    float accf[B];
    double acc[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      acc[i] = 0.0;
      accf[i] = 0.0f;
    }
    for (int k = lane; k < L; k += G) {
      const int c = __builtin_nontemporal_load(col + base + k);
      double xv[B];
#pragma unroll
      for (int j = 0; j < B; ++j) xv[j] = x[(int64_t)c * B + j];
#pragma unroll
      for (int i = 0; i < B; ++i)
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const T a = __builtin_nontemporal_load(v + (int64_t)(i * B + j) * L + k);
          if constexpr (sizeof(T) == 8)
            acc[i] = fma((double)a, xv[j], acc[i]);
          else
            accf[i] = fmaf((float)a, (float)xv[j], accf[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      double t = (sizeof(T) == 8) ? acc[i] : (double)accf[i];
      if constexpr (sizeof(T) == 8)
        t = group_sum<G>(t);
      else
        t = (double)group_sum<G>((float)t);
      acc[i] = t;
    }
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < B; ++i) {
        y[row * B + i] = acc[i];
        if (fused) dot = fma(x[row * B + i], acc[i], dot);
      }
    }
  }
  if (!fused) return;
  // fused (p, A p) for PCG: per-workgroup partial, last workgroup finalises
  dot = block_sum(dot, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = dot;
  if (!last_block(&scw->ticket, gridDim.x, &flag)) return;
  const double pq = sum_partials(partial, gridDim.x, lds);
  if (threadIdx.x == 0) {
    scw->pq = pq;
    scw->iter += 1;
    const double rz = scw->rz;
    if (!(pq > 0.0) || !(rz > 0.0)) {
      scw->done = (pq != pq || rz != rz) ? 4 : 3;
    } else {
      scw->alpha = rz / pq;
    }
  }
}

template <int B, typename T>
static hipError_t spmv_dispatch(const DeviceBsr& A, const T* val, const double* x,
                                double* y, hipStream_t s, const CgScalars* sc,
                                double* partial, CgScalars* scw, int* nblocks_out) {
  // group width from the mean row length
  const double mean = A.n_rows ? double(A.nnzb) / double(A.n_rows) : 1.0;
  int G = 64;
  if (mean < 12) G = 8;
  else if (mean < 24) G = 16;
  else if (mean < 48) G = 32;
  const int rpw = 256 / G;
  const int64_t nb = (A.n_rows + rpw - 1) / rpw;
  if (nblocks_out) *nblocks_out = (int)nb;
  if (nb == 0) return hipSuccess;
  dim3 grid((unsigned)nb), block(256);
#define FC_SPMV_CASE(GG)                                                           \
  case GG:                                                                         \
    hipLaunchKernelGGL((k_spmv_bsr<B, GG, T>), grid, block, 0, s, A.rowptr, A.col, \
                       val, x, y, A.n_rows, sc, partial, scw);                    \
    break;
  switch (G) {
    FC_SPMV_CASE(8)
    FC_SPMV_CASE(16)
    FC_SPMV_CASE(32)
    FC_SPMV_CASE(64)
  }
#undef FC_SPMV_CASE
  return hipGetLastError();
}

template <typename T>
static hipError_t spmv_any(const DeviceBsr& A, const T* val, const double* x,
                           double* y, hipStream_t s, const CgScalars* sc,
                           double* partial, CgScalars* scw, int* nb) {
  switch (A.bdim) {
    case 1: return spmv_dispatch<1, T>(A, val, x, y, s, sc, partial, scw, nb);
    case 2: return spmv_dispatch<2, T>(A, val, x, y, s, sc, partial, scw, nb);
    case 3: return spmv_dispatch<3, T>(A, val, x, y, s, sc, partial, scw, nb);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spmv(const DeviceBsr& A, const double* x, double* y, hipStream_t s) {
  return spmv_any<double>(A, A.val, x, y, s, nullptr, nullptr, nullptr, nullptr);
}

hipError_t launch_spmv_f32(const DeviceBsr& A, const double* x, double* y,
                           hipStream_t s) {
  return spmv_any<float>(A, A.val32, x, y, s, nullptr, nullptr, nullptr, nullptr);
}

int spmv_num_blocks(const DeviceBsr& A) {
  int nb = 0;
  const double mean = A.n_rows ? double(A.nnzb) / double(A.n_rows) : 1.0;
  int G = 64;
  if (mean < 12) G = 8;
  else if (mean < 24) G = 16;
  else if (mean < 48) G = 32;
  nb = (int)((A.n_rows + 256 / G - 1) / (256 / G));
  return nb;
}

hipError_t launch_spmv_pq(const DeviceBsr& A, bool f32, const double* p, double* q,
                          CgScalars* sc, double* partial, hipStream_t s) {
  if (f32) return spmv_any<float>(A, A.val32, p, q, s, sc, partial, sc, nullptr);
  return spmv_any<double>(A, A.val, p, q, s, sc, partial, sc, nullptr);
}

}  // namespace fc
