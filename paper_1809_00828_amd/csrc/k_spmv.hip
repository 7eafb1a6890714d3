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
// most of their columns).  When block rows repeat (every row whose cells are
// uncut repeats one of a few stencils of the cell grid), the products read
// one stored copy per distinct row through a per-row offset; rows with one
// copy and one lattice box shape are taken four at a time, each value loaded
// once for the four (k_spmv_bsr_grp), and the caches serve the repeats.
//
// Tiles of 256/G rows are dealt out so that the workgroups resident on one
// XCD (hardware ids congruent mod 8) walk one contiguous range of rows and
// share that XCD's L2 for x.  The PCG variant leaves one partial (x, y)
// per workgroup; a one-workgroup kernel of the solver sums them in a fixed
// order (no atomics).
#include <cstdlib>
#include <type_traits>

#include "dev_common.h"
#include "k_spmv.h"

namespace fc {

// Matrix data is read once per product.  FP64 3x3 blocks read it
// non-temporally; scalar rows and the FP32 copy read it through the caches,
// which is 13 % faster at 64^3 p = 2 and 3.5 % for the FP32 rows of the
// mixed product (measured; there the non-temporal stream costs more than
// it saves).
template <bool kNT, typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  if constexpr (kNT) return __builtin_nontemporal_load(p);
  else return *p;
}

// rows (may be null): the launch covers only these n_rows block rows
// (ascending), the others of y are left alone.
// kLat: columns computed from the lattice box (col is not read).
// XT: type of x (FP32 for the FP32 rows of the mixed product, which round
// x to FP32 before every product anyway).
// kShared: a row's values start at val + vofs[row] (bitwise-equal rows share
// one copy) instead of val + rowptr[row]*B*B; shared values are read
// through the caches, where the rows that repeat stay resident.
template <int B, int G, typename T, bool kLat, typename XT, bool kShared>
__global__ __launch_bounds__(256) void k_spmv_bsr(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, const XT* __restrict__ x,
    double* __restrict__ y, int64_t n_rows, const CgScalars* __restrict__ sc,
    double* __restrict__ partial, const int32_t* __restrict__ rows, const LatticeInfo lat,
    const int64_t* __restrict__ vofs) {
  constexpr bool kNT = B != 1 && sizeof(T) == 8 && !kShared;
  constexpr int BB = B * B;
  constexpr int RPW = 256 / G;   // rows per tile
  __shared__ double lds[16];
  if (sc && sc->done) return;
  const int64_t ntiles = (n_rows + RPW - 1) / RPW;
  // XCD-contiguous tile ranges
  const uint32_t nwg = gridDim.x, xcd = blockIdx.x % kNumXcd, j = blockIdx.x / kNumXcd;
  const uint32_t per = nwg / kNumXcd + (xcd < nwg % kNumXcd ? 1u : 0u);
  const int64_t t0 = ntiles * xcd / kNumXcd, t1 = ntiles * (xcd + 1) / kNumXcd;
  const int lane = threadIdx.x % G;
  double dot = 0.0;
  for (int64_t tile = t0 + j; tile < t1; tile += per) {
    const int64_t idx = tile * RPW + threadIdx.x / G;
    if (idx >= n_rows) continue;
    const int64_t row = rows ? (int64_t)rows[idx] : idx;
    const int64_t base = rowptr[row];
    const int L = rowptr[row + 1] - (int32_t)base;
    const T* v = val + (kShared ? vofs[row] : base * BB);
    RowBox box;
    if constexpr (kLat) box = row_box(row, lat);
    double acc[B];
    float accf[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      acc[i] = 0.0;
      accf[i] = 0.0f;
    }
    // U blocks per lane per pass: all loads of a pass are in flight
    // together (scalar rows: eight, which on 64^3-cell p = 2 rows is 6 %
    // faster than four; 3x3 blocks carry nine values each, so two)
    constexpr int U = B == 1 ? 8 : 2;
    for (int k = lane; k < L; k += U * G) {
      int c[U];
      T a[U][BB];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ku = k + u * G;
        const bool on = ku < L;
        if constexpr (kLat)
          c[u] = on ? lattice_col(box, ku, lat.n1) : -1;
        else
          c[u] = on ? stream_load<kNT>(col + base + ku) : -1;
#pragma unroll
        for (int e = 0; e < BB; ++e)
          a[u][e] = on ? stream_load<kNT>(v + (int64_t)e * L + ku) : T(0);
      }
      XT xv[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int jj = 0; jj < B; ++jj) xv[u][jj] = c[u] >= 0 ? x[(int64_t)c[u] * B + jj] : XT(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
          for (int jj = 0; jj < B; ++jj) {
            if constexpr (sizeof(T) == 8)
              acc[i] = fma((double)a[u][i * B + jj], (double)xv[u][jj], acc[i]);
            else
              accf[i] = fmaf((float)a[u][i * B + jj], (float)xv[u][jj], accf[i]);
          }
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      if constexpr (sizeof(T) == 8)
        acc[i] = group_sum<G>(acc[i]);
      else
        acc[i] = (double)group_sum<G>(accf[i]);
    }
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < B; ++i) {
        y[row * B + i] = acc[i];
        if (partial) dot = fma((double)x[row * B + i], acc[i], dot);
      }
    }
  }
  if (!partial) return;
  dot = block_sum(dot, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = dot;
}

// Rows that read one shared copy, R at a time (grp: R row indices per
// group, -1 padding; with lattice columns the rows of a group have one box
// shape, so a column is the first row's plus a fixed shift).  Each value is
// loaded once for the R rows; every row keeps the lane order, the order of
// its fused multiply-adds and the reduction of k_spmv_bsr, so its result is
// bitwise that kernel's at the same G.
template <int B, int G, bool kLat, int R, typename T = double, typename XT = double>
__global__ __launch_bounds__(256) void k_spmv_bsr_grp(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, const int64_t* __restrict__ vofs,
    const int32_t* __restrict__ grp, int64_t n_grp, const XT* __restrict__ x,
    double* __restrict__ y, const CgScalars* __restrict__ sc, const LatticeInfo lat) {
  // FP32 values accumulate in FP32, as in k_spmv_bsr
  using AC = typename std::conditional<sizeof(T) == 8, double, float>::type;
  constexpr int BB = B * B;
  constexpr int RPW = 256 / G;
  if (sc && sc->done) return;
  const int64_t ntiles = (n_grp + RPW - 1) / RPW;
  const uint32_t nwg = gridDim.x, xcd = blockIdx.x % kNumXcd, j = blockIdx.x / kNumXcd;
  const uint32_t per = nwg / kNumXcd + (xcd < nwg % kNumXcd ? 1u : 0u);
  const int64_t t0 = ntiles * xcd / kNumXcd, t1 = ntiles * (xcd + 1) / kNumXcd;
  const int lane = threadIdx.x % G;
  for (int64_t tile = t0 + j; tile < t1; tile += per) {
    const int64_t gi = tile * RPW + threadIdx.x / G;
    if (gi >= n_grp) continue;
    int64_t row[R];
#pragma unroll
    for (int q = 0; q < R; ++q) row[q] = grp[gi * R + q];
    const int64_t r0 = row[0];
    const int L = rowptr[r0 + 1] - rowptr[r0];
    const T* v = val + vofs[r0];
    // kLat: shift of each row's columns against row 0's; else the start of
    // each row's column list
    int64_t cb[R];
    RowBox box;
    if constexpr (kLat) {
      box = row_box(r0, lat);
      const int64_t b0 = box.lo[0] + (int64_t)lat.n1 * (box.lo[1] + (int64_t)lat.n1 * box.lo[2]);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        cb[q] = 0;
        if (row[q] >= 0) {
          const RowBox bq = row_box(row[q], lat);
          cb[q] = bq.lo[0] + (int64_t)lat.n1 * (bq.lo[1] + (int64_t)lat.n1 * bq.lo[2]) - b0;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) cb[q] = row[q] >= 0 ? (int64_t)rowptr[row[q]] : 0;
    }
    AC acc[R][B];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int i = 0; i < B; ++i) acc[q][i] = AC(0);
    constexpr int U = B == 1 ? 8 : 2;
    for (int k = lane; k < L; k += U * G) {
      T a[U][BB];
      int c0[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ku = k + u * G;
        const bool on = ku < L;
        if constexpr (kLat) c0[u] = on ? lattice_col(box, ku, lat.n1) : -1;
        else c0[u] = on ? ku : -1;
#pragma unroll
        for (int e = 0; e < BB; ++e) a[u][e] = on ? v[(int64_t)e * L + ku] : T(0);
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if (row[q] < 0) continue;
        XT xv[U][B];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          int64_t c = -1;
          if (c0[u] >= 0) c = kLat ? c0[u] + cb[q] : (int64_t)col[cb[q] + c0[u]];
#pragma unroll
          for (int jj = 0; jj < B; ++jj) xv[u][jj] = c >= 0 ? x[c * B + jj] : XT(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int i = 0; i < B; ++i)
#pragma unroll
            for (int jj = 0; jj < B; ++jj) {
              if constexpr (sizeof(T) == 8)
                acc[q][i] = fma((double)a[u][i * B + jj], (double)xv[u][jj], acc[q][i]);
              else
                acc[q][i] = fmaf((float)a[u][i * B + jj], (float)xv[u][jj], acc[q][i]);
            }
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (row[q] < 0) continue;
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const double s = (double)group_sum<G>(acc[q][i]);
        if (lane == 0) y[row[q] * B + i] = s;
      }
    }
  }
}

// Launch shape.  Group width chosen per matrix by spmv_autotune at set-up,
// else from the mean row length (FC_SPMV_GROUP overrides both); the PCG
// variant uses one tile per workgroup unless
// FC_SPMV_FUSED_GRID caps the grid (then workgroups loop over tiles).
static int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

static int group_width(const DeviceBsr& A) {
  static const int forced = env_int("FC_SPMV_GROUP", 0);
  if (forced == 8 || forced == 16 || forced == 32 || forced == 64) return forced;
  if (A.group) return A.group;
  const double mean = A.n_rows ? double(A.nnzb) / double(A.n_rows) : 1.0;
  if (mean < 12) return 8;
  if (mean < 24) return 16;
  if (mean < 48) return 32;
  return 64;
}

static int64_t num_tiles(const DeviceBsr& A) {
  const int rpw = 256 / group_width(A);
  return (A.n_rows + rpw - 1) / rpw;
}

static int64_t fused_grid(const DeviceBsr& A) {
  static const int cap = env_int("FC_SPMV_FUSED_GRID", 0);
  const int64_t nt = num_tiles(A);
  return cap > 0 ? std::min<int64_t>(nt, cap) : nt;
}

template <int B, typename T, typename XT>
static hipError_t spmv_dispatch(const DeviceBsr& A, const T* val, const XT* x,
                                double* y, hipStream_t s, const CgScalars* sc,
                                double* partial, const int32_t* rows, int64_t n_list,
                                const int64_t* vofs) {
  const int G = group_width(A);
  const int64_t n_rows = rows ? n_list : A.n_rows;
  const int64_t nt = (n_rows + 256 / G - 1) / (256 / G);
  if (nt == 0) return hipSuccess;
  const int64_t nb = (partial && !rows) ? fused_grid(A) : nt;
  static const bool lat_allowed = env_int("FC_SPMV_LATTICE", 1) != 0;
  const bool lat = lat_allowed && A.lat.dim > 0;
  // full FP64 products over shared rows: grouped rows (the groups were
  // formed for lattice columns only when the lattice is in use)
  // (full FP64 products over all rows; FP32 products over the FP32 rows of
  // the mixed product, grouped among those rows)
  const int32_t* gl = nullptr;
  int64_t gn = 0;
  if constexpr (std::is_same<T, double>::value && std::is_same<XT, double>::value) {
    if (vofs && val == A.vsh && !rows) {
      gl = A.grp;
      gn = A.n_grp;
    }
  } else if constexpr (std::is_same<T, float>::value && std::is_same<XT, float>::value) {
    if (vofs && val == A.vsh32 && rows == A.rows_lo) {
      gl = A.grp_lo;
      gn = A.n_grp_lo;
    }
  }
  {
    if (gl && gn > 0 && !partial && lat == (A.lat.dim > 0)) {
      const int64_t ng = (gn + 256 / G - 1) / (256 / G);
      dim3 gg((unsigned)ng), bb(256);
#define FC_SPMV_GRP(GG)                                                                    \
  case GG:                                                                                 \
    if (lat)                                                                               \
      hipLaunchKernelGGL((k_spmv_bsr_grp<B, GG, true, kShareGroup, T, XT>), gg, bb, 0, s,   \
                         A.rowptr, A.col, val, vofs, gl, gn, x, y, sc, A.lat);              \
    else                                                                                   \
      hipLaunchKernelGGL((k_spmv_bsr_grp<B, GG, false, kShareGroup, T, XT>), gg, bb, 0, s,  \
                         A.rowptr, A.col, val, vofs, gl, gn, x, y, sc, A.lat);              \
    break;
      switch (G) {
        FC_SPMV_GRP(8)
        FC_SPMV_GRP(16)
        FC_SPMV_GRP(32)
        FC_SPMV_GRP(64)
      }
#undef FC_SPMV_GRP
      return hipGetLastError();
    }
  }
  dim3 grid((unsigned)nb), block(256);
#define FC_SPMV_LAUNCH(GG, SH)                                                             \
  if (lat)                                                                                 \
    hipLaunchKernelGGL((k_spmv_bsr<B, GG, T, true, XT, SH>), grid, block, 0, s, A.rowptr,   \
                       A.col, val, x, y, n_rows, sc, partial, rows, A.lat, vofs);          \
  else                                                                                     \
    hipLaunchKernelGGL((k_spmv_bsr<B, GG, T, false, XT, SH>), grid, block, 0, s, A.rowptr,  \
                       A.col, val, x, y, n_rows, sc, partial, rows, A.lat, vofs);
#define FC_SPMV_CASE(GG)                                                                   \
  case GG:                                                                                 \
    if (vofs) {                                                                            \
      FC_SPMV_LAUNCH(GG, true)                                                             \
    } else {                                                                               \
      FC_SPMV_LAUNCH(GG, false)                                                            \
    }                                                                                      \
    break;
  switch (G) {
    FC_SPMV_CASE(8)
    FC_SPMV_CASE(16)
    FC_SPMV_CASE(32)
    FC_SPMV_CASE(64)
  }
#undef FC_SPMV_CASE
#undef FC_SPMV_LAUNCH
  return hipGetLastError();
}

template <typename T, typename XT = double>
static hipError_t spmv_any(const DeviceBsr& A, const T* val, const XT* x, double* y,
                           hipStream_t s, const CgScalars* sc, double* partial,
                           const int32_t* rows = nullptr, int64_t n_list = 0,
                           const int64_t* vofs = nullptr) {
  switch (A.bdim) {
    case 1: return spmv_dispatch<1, T, XT>(A, val, x, y, s, sc, partial, rows, n_list, vofs);
    case 2: return spmv_dispatch<2, T, XT>(A, val, x, y, s, sc, partial, rows, n_list, vofs);
    case 3: return spmv_dispatch<3, T, XT>(A, val, x, y, s, sc, partial, rows, n_list, vofs);
  }
  return hipErrorInvalidValue;
}

// FP64 values: the shared rows when set-up kept them, else the full matrix
static const double* f64_values(const DeviceBsr& A) { return A.vofs ? A.vsh : A.val; }

hipError_t launch_spmv(const DeviceBsr& A, const double* x, double* y, hipStream_t s) {
  return spmv_any<double>(A, f64_values(A), x, y, s, nullptr, nullptr, nullptr, 0, A.vofs);
}

int spmv_num_blocks(const DeviceBsr& A) { return (int)fused_grid(A); }

// mismatches between stored columns and lattice boxes (counted with an
// atomic only where one occurs)
__global__ void k_check_lattice(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                int64_t n_rows, const LatticeInfo lat,
                                unsigned long long* __restrict__ bad) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n_rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    const RowBox b = row_box(row, lat);
    const int64_t base = rowptr[row];
    const int L = rowptr[row + 1] - (int32_t)base;
    int miss = L != b.len[0] * b.len[1] * b.len[2];
    for (int k = 0; k < L && !miss; ++k) miss = col[base + k] != lattice_col(b, k, lat.n1);
    if (miss) atomicAdd(bad, 1ull);
  }
}

hipError_t spmv_enable_lattice(DeviceBsr& A, int dim, int n1, int p, hipStream_t s) {
  A.lat = LatticeInfo{};
  if (dim < 1 || dim > 3 || p < 1 || A.n_rows == 0) return hipSuccess;
  int64_t nodes = 1;
  for (int k = 0; k < dim; ++k) nodes *= n1;
  if (nodes != A.n_rows) return hipSuccess;
  unsigned long long* bad = nullptr;
  hipError_t e = hipMalloc(&bad, sizeof(*bad));
  if (e != hipSuccess) return e;
  unsigned long long hbad = 1;
  const LatticeInfo lat{dim, n1, p};
  e = hipMemsetAsync(bad, 0, sizeof(*bad), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_check_lattice, dim3(2048), dim3(256), 0, s, A.rowptr, A.col, A.n_rows,
                       lat, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(bad);
  if (e == hipSuccess && hbad == 0) A.lat = lat;
  return e;
}

// Group width of this matrix: time every width on the matrix itself
// (x = 0, so only the memory traffic counts) and keep the fastest.
hipError_t spmv_autotune(DeviceBsr& A, hipStream_t s) {
  A.group = 0;
  const int64_t n = A.n_rows * A.bdim;
  if (n == 0) return hipSuccess;
  double *x = nullptr, *y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipMalloc(&x, n * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&y, n * sizeof(double));
  if (err == hipSuccess) err = hipMemsetAsync(x, 0, n * sizeof(double), s);
  if (err == hipSuccess) err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  float best = 1e30f;
  int best_g = 0;
  for (int G : {8, 16, 32, 64}) {
    if (err != hipSuccess) break;
    A.group = G;
    err = launch_spmv(A, x, y, s);
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && err == hipSuccess; ++r) err = launch_spmv(A, x, y, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && ms < best) {
      best = ms;
      best_g = G;
    }
  }
  A.group = err == hipSuccess ? best_g : 0;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (x) (void)hipFree(x);
  if (y) (void)hipFree(y);
  return err;
}

hipError_t launch_spmv_pq(const DeviceBsr& A, const double* p, double* q, CgScalars* sc,
                          double* partial, hipStream_t s) {
  return spmv_any<double>(A, f64_values(A), p, q, s, sc, partial, nullptr, 0, A.vofs);
}

hipError_t launch_spmv_mixed(const DeviceBsr& A, const double* p, const float* p32, double* q,
                             const CgScalars* sc, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (A.n_hi > 0 &&
      (e = spmv_any<double>(A, f64_values(A), p, q, s, sc, nullptr, A.rows_hi, A.n_hi,
                            A.vofs)) != hipSuccess)
    return e;
  if (A.n_lo > 0)
    e = spmv_any<float, float>(A, A.vsh32 ? A.vsh32 : A.val32, p32, q, s, sc, nullptr, A.rows_lo,
                               A.n_lo, A.vsh32 ? A.vofs : nullptr);
  return e;
}

}  // namespace fc
