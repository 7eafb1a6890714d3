// Block-sparse (BSR) matrix-vector product y = A x for the assembled finite
// cell stiffness matrix (Sec. 3.1, Eq. 2); the product with A is half of
// every PCG iteration (Sec. 5.4 names the matrix-vector products as the
// dominant work of the solver).
//
// Layout (row-SoA BSR): the values of block row i are stored entry-major,
// val[rowptr[i]*B*B + e*L + k] for entry e of the k-th block of the row,
// so G lanes sweeping the blocks of one row read G consecutive values per
// entry.  A group of G lanes owns one block row; its partial sums are
// combined with a butterfly reduction.  Every block row reads its own
// stored values once per product; FP64 3x3 values and column indices are
// streamed with non-temporal loads, which leaves the cache to the gathered x
// entries (neighbouring rows of the lattice share most of their columns).
// The group width G is fixed at set-up from the mean row length, so the
// summation order of a row, and with it every result, is the same in every
// process.
//
// Tiles of 256/G rows are dealt out so that the workgroups resident on one
// XCD (hardware ids congruent mod 8) walk one contiguous range of rows and
// share that XCD's L2 for x.  The PCG variant leaves one partial (x, y)
// per workgroup; a one-workgroup kernel of the solver sums them in a fixed
// order (no atomics).
#include <cstdlib>

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
// U: blocks per lane per pass (all loads of a pass are in flight together).
// kNT: stream the matrix values non-temporally.
template <int B, int G, typename T, bool kLat, typename XT, int U, bool kNT>
__global__ __launch_bounds__(256) void k_spmv_bsr(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, const XT* __restrict__ x,
    double* __restrict__ y, int64_t n_rows, const CgScalars* __restrict__ sc,
    double* __restrict__ partial, const int32_t* __restrict__ rows, const LatticeInfo lat) {
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
    // on the lattice the row's start and length follow from its indices,
    // so the value stream does not wait for a row-pointer load
    RowBox box;
    int64_t base;
    int L;
    if constexpr (kLat) {
      int c[3];
      lattice_coords(row, lat, c);
      box = row_box_at(c, lat);
      base = lattice_row_start_at(c, box, lat);
      L = box.len[0] * box.len[1] * box.len[2];
    } else {
      base = rowptr[row];
      L = rowptr[row + 1] - (int32_t)base;
    }
    const T* v = val + base * BB;
    double acc[B];
    float accf[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      acc[i] = 0.0;
      accf[i] = 0.0f;
    }
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

// Launch shape.  G lanes per block row: enough lanes that one pass of U
// blocks per lane (eight scalar blocks, two 3x3 blocks) covers the mean row,
// rounded up to 8, 16, 32 or 64 (FC_SPMV_GROUP overrides it).  Measured on
// MI355X this picks the fastest width for both FP64 workloads: 64 for the
// 3x3 rows of 32^3-cell p = 3 elasticity (about 122 blocks), 8 for the
// scalar rows of 64^3-cell p = 2 Poisson (about 63).  The PCG variant uses
// one tile per workgroup unless FC_SPMV_FUSED_GRID caps the grid (then
// workgroups loop over tiles).
static int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

int spmv_group_for(const DeviceBsr& A) {
  const double mean = A.n_rows ? double(A.nnzb) / double(A.n_rows) : 1.0;
  const int U = A.bdim == 1 ? 8 : 2;
  const double lanes = mean / U;
  if (lanes <= 8) return 8;
  if (lanes <= 16) return 16;
  if (lanes <= 32) return 32;
  return 64;
}

static int group_width(const DeviceBsr& A) {
  static const int forced = env_int("FC_SPMV_GROUP", 0);
  if (forced == 8 || forced == 16 || forced == 32 || forced == 64) return forced;
  return A.group ? A.group : spmv_group_for(A);
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
                                double* partial, const int32_t* rows, int64_t n_list) {
  const int G = group_width(A);
  const int64_t n_rows = rows ? n_list : A.n_rows;
  const int64_t nt = (n_rows + 256 / G - 1) / (256 / G);
  if (nt == 0) return hipSuccess;
  const int64_t nb = (partial && !rows) ? fused_grid(A) : nt;
  static const bool lat_allowed = env_int("FC_SPMV_LATTICE", 1) != 0;
  const bool lat = lat_allowed && A.lat.dim > 0;
  dim3 grid((unsigned)nb), block(256);
  // 3x3 blocks: two per lane per pass (nine values each), FP64 values
  // non-temporal.  Scalar rows: eight per lane per pass through the caches
  // (FC_SPMV_PASS=16 and FC_SPMV_NT=1 select sixteen and the non-temporal
  // stream for FP64 scalar rows on the lattice).
  static const int pass16 = env_int("FC_SPMV_PASS", 8) == 16;
  static const int nt1 = env_int("FC_SPMV_NT", 0) == 1;
  constexpr bool kNT3 = B != 1 && sizeof(T) == 8;
  constexpr int kU = B == 1 ? 8 : 2;
#define FC_SPMV_LAUNCH(GG, LAT, UU, NT)                                                      \
  hipLaunchKernelGGL((k_spmv_bsr<B, GG, T, LAT, XT, UU, NT>), grid, block, 0, s, A.rowptr,   \
                     A.col, val, x, y, n_rows, sc, partial, rows, A.lat)
#define FC_SPMV_CASE(GG)                                                                     \
  case GG:                                                                                   \
    if (lat) {                                                                               \
      if constexpr (B == 1 && sizeof(T) == 8) {                                              \
        if (pass16 && nt1) FC_SPMV_LAUNCH(GG, true, 16, true);                               \
        else if (pass16) FC_SPMV_LAUNCH(GG, true, 16, false);                                \
        else if (nt1) FC_SPMV_LAUNCH(GG, true, 8, true);                                     \
        else FC_SPMV_LAUNCH(GG, true, 8, false);                                             \
      } else {                                                                               \
        FC_SPMV_LAUNCH(GG, true, kU, kNT3);                                                  \
      }                                                                                      \
    } else {                                                                                 \
      FC_SPMV_LAUNCH(GG, false, kU, kNT3);                                                   \
    }                                                                                        \
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
                           const int32_t* rows = nullptr, int64_t n_list = 0) {
  switch (A.bdim) {
    case 1: return spmv_dispatch<1, T, XT>(A, val, x, y, s, sc, partial, rows, n_list);
    case 2: return spmv_dispatch<2, T, XT>(A, val, x, y, s, sc, partial, rows, n_list);
    case 3: return spmv_dispatch<3, T, XT>(A, val, x, y, s, sc, partial, rows, n_list);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spmv(const DeviceBsr& A, const double* x, double* y, hipStream_t s) {
  return spmv_any<double>(A, A.val, x, y, s, nullptr, nullptr);
}

int spmv_num_blocks(const DeviceBsr& A) { return (int)fused_grid(A); }

// mismatches between stored rows and lattice boxes: length, start and
// columns (counted with an atomic only where one occurs)
__global__ void k_check_lattice(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                int64_t n_rows, const LatticeInfo lat,
                                unsigned long long* __restrict__ bad) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n_rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    const RowBox b = row_box(row, lat);
    const int64_t base = rowptr[row];
    const int L = rowptr[row + 1] - (int32_t)base;
    int miss = L != b.len[0] * b.len[1] * b.len[2] || base != lattice_row_start(row, lat);
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
  const LatticeInfo lat = make_lattice_info(dim, n1, p);
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

hipError_t launch_spmv_pq(const DeviceBsr& A, const double* p, double* q, CgScalars* sc,
                          double* partial, hipStream_t s) {
  return spmv_any<double>(A, A.val, p, q, s, sc, partial);
}

hipError_t launch_spmv_mixed(const DeviceBsr& A, const double* p, const float* p32, double* q,
                             const CgScalars* sc, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (A.n_hi > 0 &&
      (e = spmv_any<double>(A, A.val, p, q, s, sc, nullptr, A.rows_hi, A.n_hi)) != hipSuccess)
    return e;
  if (A.n_lo > 0)
    e = spmv_any<float, float>(A, A.val32, p32, q, s, sc, nullptr, A.rows_lo, A.n_lo);
  return e;
}

}  // namespace fc
