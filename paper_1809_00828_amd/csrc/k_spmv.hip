// Block-sparse (BSR) matrix-vector product y = A x for the assembled finite
// cell stiffness matrix (Sec. 3.1, Eq. 2); the product with A is half of
// every PCG iteration (Sec. 5.4 names the matrix-vector products as the
// dominant work of the solver).
//
// Layout (row-SoA BSR): the values of block row i are stored entry-major,
// val[rowptr[i]*B*B + e*L + k] for entry e of the k-th block of the row,
// so G lanes sweeping the blocks of one row read G consecutive values per
// entry (two adjacent blocks per lane for 2x2 and 3x3 blocks, so each entry
// of a lane is one 16-byte load).  A group of G lanes owns one block row;
// its partial sums are combined with a butterfly reduction.  Every block row reads its own
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
//
// Matrices assembled from a problem description have lattice rows: the
// columns and the start of each row follow from the row's lattice indices
// and are computed, not read.  Scalar ones (degree p <= 4) also keep a
// sliced copy, 64 rows of one lattice line with equal boxes per slice, for
// the whole-matrix product (k_spmv_sell below).
#include <cstdlib>
#include <vector>

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

// Sum over a wave with DPP moves (row shifts within rows of 16 lanes, then
// row broadcasts): the total lands in lane 63, in a fixed order.
template <int C, int RM>
__device__ __forceinline__ double dpp64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, C, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), C, RM, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_sum_last(double v) {
  v += dpp64<0x111, 0xf>(v);   // row_shr:1
  v += dpp64<0x112, 0xf>(v);   // row_shr:2
  v += dpp64<0x114, 0xf>(v);   // row_shr:4
  v += dpp64<0x118, 0xf>(v);   // row_shr:8
  v += dpp64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// rows (may be null): the launch covers only these n_rows block rows
// (ascending), the others of y are left alone.
// kLat: columns computed from the lattice box (col is not read).
// XT: type of x (FP32 for the FP32 rows of the mixed product, which round
// x to FP32 before every product anyway).
// U: blocks per lane per pass (all loads of a pass are in flight together);
// U = 2 takes two adjacent blocks, so each entry is one two-wide load (half
// the load instructions of two separate blocks: 5.5 % faster for the 3x3
// rows of 32^3-cell p = 3 elasticity).
// kNT: stream the matrix values non-temporally.
// At most 96 VGPRs, five waves per SIMD: the paired loads otherwise take 105
// VGPRs and four waves, which is 3 % slower.
template <int B, int G, typename T, bool kLat, typename XT, int U, bool kNT>
__global__ __launch_bounds__(256, 5) void k_spmv_bsr(
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
  const XcdRange xr_ = xcd_range(blockIdx.x, gridDim.x, ntiles);
  const uint32_t j = xr_.j, per = xr_.per;
  const int64_t t0 = xr_.t0, t1 = xr_.t1;
  const int lane = threadIdx.x % G;
  double dot = 0.0;
  for (int64_t tile = t0 + j; tile < t1; tile += per) {
    // one row per wave (G = 64): the row and everything derived from it are
    // wave-uniform, so they are computed once per wave in scalar registers
    const int wrow = G == 64 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.x / G)
                             : (int)(threadIdx.x / G);
    const int64_t idx = tile * RPW + wrow;
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
    // U == 2: a lane takes two adjacent blocks, so each entry of the pair
    // is one 2-wide load (16 bytes for FP64; 8-byte aligned, which the
    // hardware loads as one access)
    constexpr bool kPair = U == 2;
    const int k0 = kPair ? 2 * lane : lane;
    for (int k = k0; k < L; k += U * G) {
      int c[U];
      T a[U][BB];
      if constexpr (kPair) {
        typedef T t2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const bool on = k + u < L;
          if constexpr (kLat)
            c[u] = on ? lattice_col(box, k + u, lat.n1) : -1;
          else
            c[u] = on ? stream_load<kNT>(col + base + k + u) : -1;
        }
        if (k + 1 < L) {
#pragma unroll
          for (int e = 0; e < BB; ++e) {
            const t2* p = reinterpret_cast<const t2*>(v + (int64_t)e * L + k);
            const t2 t = kNT ? __builtin_nontemporal_load(p) : *p;
            a[0][e] = t.x;
            a[1][e] = t.y;
          }
        } else {
#pragma unroll
          for (int e = 0; e < BB; ++e) {
            a[0][e] = stream_load<kNT>(v + (int64_t)e * L + k);
            a[1][e] = T(0);
          }
        }
      } else {
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
      }
      XT xv[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (B == 3) {
          typedef XT x2 __attribute__((ext_vector_type(2), aligned(sizeof(XT))));
          const int64_t cc = c[u] >= 0 ? (int64_t)c[u] * B : 0;
          const x2 t = *reinterpret_cast<const x2*>(x + cc);
          const XT t2 = x[cc + 2];
          xv[u][0] = c[u] >= 0 ? t.x : XT(0);
          xv[u][1] = c[u] >= 0 ? t.y : XT(0);
          xv[u][2] = c[u] >= 0 ? t2 : XT(0);
        } else {
#pragma unroll
          for (int jj = 0; jj < B; ++jj) xv[u][jj] = c[u] >= 0 ? x[(int64_t)c[u] * B + jj] : XT(0);
        }
      }
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
    constexpr int kOut = G == 64 ? 63 : 0;   // the lane that holds the row's sums
#pragma unroll
    for (int i = 0; i < B; ++i) {
      if constexpr (G == 64)
        acc[i] = wave_sum_last(sizeof(T) == 8 ? acc[i] : (double)accf[i]);
      else if constexpr (sizeof(T) == 8)
        acc[i] = group_sum<G>(acc[i]);
      else
        acc[i] = (double)group_sum<G>(accf[i]);
    }
    if (lane == kOut) {
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

// ---------------------------------------------------------------- sliced
// x index of lane row i of a class: interior vertices x = p (i + 1), other
// interior indices in ascending order (p - 1 per cell; none when p = 1)
__device__ __forceinline__ int sell_x(bool vertex, int i, int p) {
  if (vertex || p == 1) return p * (i + 1);
  return (i / (p - 1)) * p + 1 + i % (p - 1);
}

template <int P>
__device__ __forceinline__ int sell_x_p(bool vertex, int i) {
  if constexpr (P == 1) {
    return i + 1;
  } else {
    return vertex ? P * (i + 1) : (i / (P - 1)) * P + 1 + i % (P - 1);
  }
}

// Lattice range of the functions whose support meets that of index g along
// one direction (as in row_box_at), for degree P.
template <int P>
__device__ __forceinline__ void dir_box_p(int g, int n1, int* lo, int* len) {
  if (g % P == 0) {
    const int a = max(0, g - P), b = min(n1 - 1, g + P);
    *lo = a;
    *len = b - a + 1;
  } else {
    *lo = (g / P) * P;
    *len = P + 1;
  }
}

struct SellSlice {
  int64_t line;
  bool vertex;
  int chunk;
};

__device__ __forceinline__ SellSlice sell_slice(int64_t s, int cv, int cn) {
  SellSlice r;
  const int spl = cv + cn;
  r.line = s / spl;
  const int loc = (int)(s - r.line * spl);
  r.vertex = loc < cv;
  r.chunk = r.vertex ? loc : loc - cv;
  return r;
}

// The same for the product kernel: fewer than 2^31 slices, and the slices
// per line divided by multiply-shift.
__device__ __forceinline__ SellSlice sell_slice_fast(uint32_t s, int cv, const FastDiv dspl) {
  SellSlice r;
  const uint32_t line = fdiv(s, dspl);
  const int loc = (int)(s - line * dspl.d);
  r.line = line;
  r.vertex = loc < cv;
  r.chunk = r.vertex ? loc : loc - cv;
  return r;
}

// sell_val from the row layout, one workgroup per slice
__global__ __launch_bounds__(256) void k_sell_build(const double* __restrict__ val,
                                                    const int64_t* __restrict__ off,
                                                    int64_t n_slices, int cv, int cn, int nv,
                                                    int nn, const LatticeInfo lat,
                                                    double* __restrict__ sv) {
  for (int64_t s = blockIdx.x; s < n_slices; s += gridDim.x) {
    const SellSlice sl = sell_slice(s, cv, cn);
    const int n1 = lat.n1;
    const int y0 = lat.dim >= 2 ? (int)(sl.line % n1) : 0;
    const int z0 = lat.dim == 3 ? (int)(sl.line / n1) : 0;
    const int64_t len = (off[s + 1] - off[s]) / 64;
    for (int64_t e = threadIdx.x; e < 64 * len; e += blockDim.x) {
      const int k = (int)(e / 64), l = (int)(e % 64);
      const int i = sl.chunk * 64 + l;
      double v = 0.0;
      if (i < (sl.vertex ? nv : nn)) {
        const int c[3] = {sell_x(sl.vertex, i, lat.p), y0, z0};
        v = val[lattice_row_start_at(c, row_box_at(c, lat), lat) + k];
      }
      // entries in pairs: lane l holds entries 2j, 2j + 1 at 128 j + 2 l + 0/1;
      // an odd last entry alone at 128 j + l
      const int64_t dst = (k == len - 1 && (len & 1)) ? (int64_t)(k / 2) * 128 + l
                                                      : (int64_t)(k / 2) * 128 + 2 * l + (k & 1);
      sv[off[s] + dst] = v;
    }
  }
}

// y = A x on the sliced rows: one wave per slice, one row per lane.  The
// box entries run x-pencil by x-pencil (kx fastest); every lane of a slice
// has the same pencil count and length, so the pencil's column offset in y
// and z is the same for all lanes.  Pencils go two per round, all their
// loads issued before the first FMA: a round's 2K entries are K paired
// values per lane (one 16-byte load each, 1 KB contiguous per wave; 8 %
// faster than one 8-byte load per entry at 64^3 cells, p = 2), and each
// pencil's x run is read two entries per load.  A last round with one
// pencil reads its odd last entry alone.  kNT: the values (read once) are
// streamed non-temporally.  The pencil's (y, z) offsets are stepped, not
// divided out of its index.
template <int K, bool kNT>
__device__ __forceinline__ double sell_pencils(const double* __restrict__ vs, int l,
                                               const double* __restrict__ xb, int len1,
                                               int npen, int64_t n1) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef double d2a8 __attribute__((ext_vector_type(2), aligned(8)));
  double acc = 0.0;
  int qy = 0, qz = 0;   // offsets of pencil q
  for (int q = 0; q < npen; q += 2) {
    const double* vr = vs + (int64_t)128 * K * (q / 2) + 2 * l;
    const double* xp0 = xb + n1 * (qy + n1 * qz);
    if (++qy == len1) {
      qy = 0;
      ++qz;
    }
    if (q + 1 < npen) {
      const double* xp1 = xb + n1 * (qy + n1 * qz);
      if (++qy == len1) {
        qy = 0;
        ++qz;
      }
      double a[2 * K], b[2 * K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const d2* p = reinterpret_cast<const d2*>(vr + 128 * j);
        const d2 t = kNT ? __builtin_nontemporal_load(p) : *p;
        a[2 * j] = t.x;
        a[2 * j + 1] = t.y;
      }
#pragma unroll
      for (int kx = 0; kx + 1 < K; kx += 2) {
        const d2a8 t0 = *reinterpret_cast<const d2a8*>(xp0 + kx);
        const d2a8 t1 = *reinterpret_cast<const d2a8*>(xp1 + kx);
        b[kx] = t0.x;
        b[kx + 1] = t0.y;
        b[K + kx] = t1.x;
        b[K + kx + 1] = t1.y;
      }
      if (K & 1) {
        b[K - 1] = xp0[K - 1];
        b[2 * K - 1] = xp1[K - 1];
      }
#pragma unroll
      for (int e = 0; e < 2 * K; ++e) acc = fma(a[e], b[e], acc);
    } else {
      double a[K], b[K];
#pragma unroll
      for (int j = 0; j < K / 2; ++j) {
        const d2* p = reinterpret_cast<const d2*>(vr + 128 * j);
        const d2 t = kNT ? __builtin_nontemporal_load(p) : *p;
        a[2 * j] = t.x;
        a[2 * j + 1] = t.y;
      }
      if (K & 1) {
        const double* p = vr - l + 128 * (K / 2);   // the odd last entry, alone
        a[K - 1] = kNT ? __builtin_nontemporal_load(p) : *p;
      }
#pragma unroll
      for (int kx = 0; kx + 1 < K; kx += 2) {
        const d2a8 t0 = *reinterpret_cast<const d2a8*>(xp0 + kx);
        b[kx] = t0.x;
        b[kx + 1] = t0.y;
      }
      if (K & 1) b[K - 1] = xp0[K - 1];
#pragma unroll
      for (int e = 0; e < K; ++e) acc = fma(a[e], b[e], acc);
    }
  }
  return acc;
}

template <int P, bool kNT>
__global__ __launch_bounds__(256) void k_spmv_sell(const double* __restrict__ sv,
                                                   const int64_t* __restrict__ off,
                                                   int64_t n_slices, int cv, const FastDiv dspl,
                                                   int nv, int nn, const double* __restrict__ x,
                                                   double* __restrict__ y,
                                                   const CgScalars* __restrict__ sc,
                                                   const LatticeInfo lat) {
  if (sc && sc->done) return;
  // the slice of this wave (wave-uniform, so everything derived from it
  // stays in scalar registers; no division by a run-time value)
  const int64_t s = xcd_remap(blockIdx.x, gridDim.x) * 4 +
                    __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  if (s >= n_slices) return;
  const int l = threadIdx.x % 64;
  const SellSlice sl = sell_slice_fast((uint32_t)s, cv, dspl);
  const int n1 = lat.n1;
  const uint32_t lz = fdiv((uint32_t)sl.line, lat.dn1);
  const int y0 = lat.dim >= 2 ? (int)((uint32_t)sl.line - lz * (uint32_t)n1) : 0;
  const int z0 = lat.dim == 3 ? (int)lz : 0;
  int lo1 = 0, len1 = 1, lo2 = 0, len2 = 1;
  if (lat.dim >= 2) dir_box_p<P>(y0, n1, &lo1, &len1);
  if (lat.dim == 3) dir_box_p<P>(z0, n1, &lo2, &len2);
  const int count = sl.vertex ? nv : nn;
  const int i = sl.chunk * 64 + l;
  const bool valid = i < count;
  const int xr = sell_x_p<P>(sl.vertex, valid ? i : count - 1);
  const int lo0 = sl.vertex ? xr - P : (xr / P) * P;
  const double* vs = sv + off[s];
  const double* xb = x + lo0 + (int64_t)n1 * (lo1 + (int64_t)n1 * lo2);
  const int npen = len1 * len2;
  // two pencils per round: 1 % faster than four and 3 % faster than eight
  // at 64^3 cells, p = 2
  const double acc = sl.vertex ? sell_pencils<2 * P + 1, kNT>(vs, l, xb, len1, npen, n1)
                               : sell_pencils<P + 1, kNT>(vs, l, xb, len1, npen, n1);
  if (valid) y[xr + (int64_t)n1 * (y0 + (int64_t)n1 * z0)] = acc;
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
  // the whole scalar matrix with its sliced copy, no fused dot: the sliced
  // rows, then the boundary vertex rows from the row layout
  if constexpr (B == 1 && sizeof(T) == 8 && sizeof(XT) == 8) {
    if (lat && A.sell_val && !rows && !partial) {
      const int cn = A.sell_nn > 0 ? (A.sell_nn + 63) / 64 : 0;
      const FastDiv dspl = make_fastdiv((uint32_t)(A.sell_cv + cn));
      dim3 g((unsigned)((A.n_slices + 3) / 4)), b(256);
      // values streamed non-temporally (3 % faster at 64^3 cells, p = 2;
      // FC_SPMV_SELL_NT=0 reads them through the caches)
      static const bool sell_nt = env_int("FC_SPMV_SELL_NT", 1) != 0;
#define FC_SELL(PP)                                                                           \
  do {                                                                                        \
    if (sell_nt)                                                                              \
      hipLaunchKernelGGL((k_spmv_sell<PP, true>), g, b, 0, s, A.sell_val, A.sell_off,         \
                         A.n_slices, A.sell_cv, dspl, A.sell_nv, A.sell_nn, (const double*)x, y, \
                         sc, A.lat);                                                          \
    else                                                                                      \
      hipLaunchKernelGGL((k_spmv_sell<PP, false>), g, b, 0, s, A.sell_val, A.sell_off,        \
                         A.n_slices, A.sell_cv, dspl, A.sell_nv, A.sell_nn, (const double*)x, y, \
                         sc, A.lat);                                                          \
  } while (0)
      switch (A.lat.p) {
        case 1: FC_SELL(1); break;
        case 2: FC_SELL(2); break;
        case 3: FC_SELL(3); break;
        default: FC_SELL(4); break;
      }
#undef FC_SELL
      hipError_t e = hipGetLastError();
      if (e != hipSuccess || A.n_rest == 0) return e;
      return spmv_dispatch<B, T, XT>(A, val, x, y, s, sc, nullptr, A.sell_rest, A.n_rest);
    }
  }
  dim3 grid((unsigned)nb), block(256);
  // 3x3 blocks: two per lane per pass (nine values each), FP64 values
  // non-temporal; scalar rows: eight per lane per pass through the caches
  constexpr bool kNT = B != 1 && sizeof(T) == 8;
  constexpr int kU = B == 1 ? 8 : 2;
#define FC_SPMV_CASE(GG)                                                                     \
  case GG:                                                                                   \
    if (lat)                                                                                 \
      hipLaunchKernelGGL((k_spmv_bsr<B, GG, T, true, XT, kU, kNT>), grid, block, 0, s,       \
                         A.rowptr, A.col, val, x, y, n_rows, sc, partial, rows, A.lat);      \
    else                                                                                     \
      hipLaunchKernelGGL((k_spmv_bsr<B, GG, T, false, XT, kU, kNT>), grid, block, 0, s,      \
                         A.rowptr, A.col, val, x, y, n_rows, sc, partial, rows, A.lat);      \
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

// Host side of the sliced copy: slice offsets (each slice holds 64 lanes of
// its box size), the boundary vertex rows, then the copy on the device.
static hipError_t spmv_build_sell(DeviceBsr& A, hipStream_t s) {
  const LatticeInfo lat = A.lat;
  const int n1 = lat.n1, p = lat.p, n = (n1 - 1) / p;
  const int nv = n - 1, nn = n * (p - 1);
  const int cv = nv > 0 ? (nv + 63) / 64 : 0, cn = nn > 0 ? (nn + 63) / 64 : 0;
  const int64_t lines = lat.dim == 3 ? (int64_t)n1 * n1 : n1;
  if (cv + cn == 0) return hipSuccess;
  auto len = [&](int g) {
    if (g % p != 0) return p + 1;
    return std::min(n1 - 1, g + p) - std::max(0, g - p) + 1;
  };
  std::vector<int64_t> off;
  off.reserve((size_t)(lines * (cv + cn) + 1));
  off.push_back(0);
  std::vector<int32_t> rest;
  for (int64_t line = 0; line < lines; ++line) {
    const int y0 = (int)(line % n1), z0 = lat.dim == 3 ? (int)(line / n1) : 0;
    const int64_t yz = (int64_t)len(y0) * (lat.dim == 3 ? len(z0) : 1);
    for (int k = 0; k < cv; ++k) off.push_back(off.back() + 64 * yz * (2 * p + 1));
    for (int k = 0; k < cn; ++k) off.push_back(off.back() + 64 * yz * (p + 1));
    const int64_t r0 = (int64_t)n1 * (y0 + (int64_t)n1 * z0);
    rest.push_back((int32_t)r0);
    if (n1 > 1) rest.push_back((int32_t)(r0 + n1 - 1));
  }
  const int64_t ns = (int64_t)off.size() - 1;
  hipError_t e = hipMalloc(&A.sell_val, (size_t)off.back() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&A.sell_off, off.size() * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&A.sell_rest, rest.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpyAsync(A.sell_off, off.data(), off.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(A.sell_rest, rest.data(), rest.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sell_build, dim3(4096), dim3(256), 0, s, A.val, A.sell_off, ns, cv, cn,
                       nv, nn, lat, A.sell_val);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host vectors die here
  if (e != hipSuccess) {
    for (void* q : {(void*)A.sell_val, (void*)A.sell_off, (void*)A.sell_rest})
      if (q) (void)hipFree(q);
    A.sell_val = nullptr;
    A.sell_off = nullptr;
    A.sell_rest = nullptr;
    // without room for the copy the row layout serves every product
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return hipSuccess;
    }
    return e;
  }
  A.n_slices = ns;
  A.sell_cv = cv;
  A.sell_nv = nv;
  A.sell_nn = nn;
  A.n_rest = (int64_t)rest.size();
  return hipSuccess;
}

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
  if (e == hipSuccess && A.lat.dim >= 2 && A.bdim == 1 && p <= 4 && env_int("FC_SPMV_SELL", 1))
    e = spmv_build_sell(A, s);
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
