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

// Contiguous tile range [t0, t1) of the XCD of workgroup bid, walked by
// that XCD's workgroups from j with stride per.  Workgroups are dealt out
// round-robin over min(nwg, kNumXcd) XCDs, so a grid with fewer workgroups
// than XCDs still covers every tile.
struct XcdRange {
  int64_t t0, t1;
  uint32_t j, per;
};

__device__ __forceinline__ XcdRange xcd_range(uint32_t bid, uint32_t nwg, int64_t ntiles) {
  const uint32_t nx = nwg < (uint32_t)kNumXcd ? nwg : (uint32_t)kNumXcd;
  const uint32_t x = bid % nx;
  XcdRange r;
  r.j = bid / nx;
  r.per = nwg / nx + (x < nwg % nx ? 1u : 0u);
  // eight XCDs (every grid of eight workgroups or more): a shift instead of
  // a 64-bit division, which costs hundreds of scalar instructions per wave
  if (nx == (uint32_t)kNumXcd) {
    r.t0 = (ntiles * x) >> 3;
    r.t1 = (ntiles * (x + 1)) >> 3;
  } else {
    r.t0 = ntiles * x / nx;
    r.t1 = ntiles * (x + 1) / nx;
  }
  return r;
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

// n / d with the multiplier of make_fastdiv
__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv f) {
  const uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);   // v_mul_hi_u32 on the device
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Lattice indices of row node `row` (fewer than 2^31 rows: the row
// pointers are 32-bit), first direction fastest.
__device__ __forceinline__ void lattice_coords(int64_t row, const LatticeInfo& lat, int c[3]) {
  uint32_t r = (uint32_t)row;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c[k] = 0;
    if (k < lat.dim) {
      const uint32_t q = fdiv(r, lat.dn1);
      c[k] = (int)(r - q * (uint32_t)lat.n1);
      r = q;
    }
  }
}

struct RowBox {
  int lo[3], len[3];
  float inv[2];   // 1 / len[0], 1 / len[1] (approximate, see lattice_col)
};

__device__ __forceinline__ RowBox row_box_at(const int c[3], const LatticeInfo& lat) {
  RowBox b;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = 0;
    b.len[k] = 1;
    if (k < lat.dim) {
      const int g = c[k];
      const int q = (int)fdiv((uint32_t)g, lat.dp);
      if (g == q * lat.p) {
        const int lo = max(0, g - lat.p), hi = min(lat.n1 - 1, g + lat.p);
        b.lo[k] = lo;
        b.len[k] = hi - lo + 1;
      } else {
        b.lo[k] = q * lat.p;
        b.len[k] = lat.p + 1;
      }
    }
  }
  b.inv[0] = __builtin_amdgcn_rcpf((float)b.len[0]);
  b.inv[1] = __builtin_amdgcn_rcpf((float)b.len[1]);
  return b;
}

// Lattice box of row node `row`: for every direction the range of lattice
// indices of the functions whose support meets the row's support (a vertex
// index reaches one cell to each side, an interior index only its cell).
__device__ __forceinline__ RowBox row_box(int64_t row, const LatticeInfo& lat) {
  int c[3];
  lattice_coords(row, lat, c);
  return row_box_at(c, lat);
}

// Row start of a node in a matrix whose rows are the lattice nodes in order
// and hold exactly their lattice boxes (the layout the SpMV checks before it
// computes columns).  Along one direction, node g reaches len(g) nodes:
// 2p + 1 for an inner vertex index, p + 1 for a boundary vertex or any
// other index.  The box of node (x, y, z) holds len(x) len(y) len(z)
// entries, so with S(g) = sum_{j<g} len(j) and T = S(n1) the entries before
// it number S(z) T^2 + len(z) S(y) T + len(z) len(y) S(x).
__device__ __forceinline__ int64_t lattice_len(int g, const LatticeInfo& lat) {
  if (g != (int)fdiv((uint32_t)g, lat.dp) * lat.p) return lat.p + 1;
  return (g == 0 || g == lat.n1 - 1) ? lat.p + 1 : 2 * lat.p + 1;
}

__device__ __forceinline__ int64_t lattice_prefix(int g, const LatticeInfo& lat) {
  // every period of p indices holds one vertex and p - 1 other indices; the
  // boundary vertices 0 and n1 - 1 reach p fewer nodes (the last one lies
  // in a whole period only when p = 1)
  const int p = lat.p;
  const int q = (int)fdiv((uint32_t)g, lat.dp), rm = g - q * p;
  int64_t s = (int64_t)q * (2 * p + 1 + (int64_t)(p - 1) * (p + 1));
  if (q > 0) s -= p;
  if ((int64_t)q * p > lat.n1 - 1) s -= p;
  if (rm > 0) s += lattice_len(q * p, lat) + (int64_t)(rm - 1) * (p + 1);
  return s;
}

__device__ __forceinline__ int64_t lattice_row_start_at(const int c[3], const RowBox& b,
                                                        const LatticeInfo& lat) {
  const int64_t T = lattice_prefix(lat.n1, lat);
  // from the last direction down: S(c_k) T^k times the box lengths above k
  int64_t base = 0, outer = 1;
  if (lat.dim == 3) {
    base += lattice_prefix(c[2], lat) * T * T;
    outer = b.len[2];
  }
  if (lat.dim >= 2) {
    base += lattice_prefix(c[1], lat) * T * outer;
    outer *= b.len[1];
  }
  base += lattice_prefix(c[0], lat) * outer;
  return base;
}

__device__ __forceinline__ int64_t lattice_row_start(int64_t row, const LatticeInfo& lat) {
  int c[3];
  lattice_coords(row, lat, c);
  return lattice_row_start_at(c, row_box_at(c, lat), lat);
}

// column of the k-th block of the row (first direction fastest).  k < 2^12
// and the lengths are small, so floor((k + 1/2) / len) from the approximate
// reciprocal is exact: the quotient lies at least 1/(2 len) from an integer,
// far beyond the reciprocal's relative error of about 2^-22.
__device__ __forceinline__ int lattice_col(const RowBox& b, int k, int n1) {
  const int r = (int)(((float)k + 0.5f) * b.inv[0]);
  const int kx = k - r * b.len[0];
  const int kz = (int)(((float)r + 0.5f) * b.inv[1]);
  const int ky = r - kz * b.len[1];
  return (b.lo[0] + kx) + n1 * ((b.lo[1] + ky) + n1 * (b.lo[2] + kz));
}

// The cells holding lattice index g along one direction (at most two, in
// ascending order) and the function's local index on each: a vertex index
// (g a multiple of p) is local 1 (right end) of cell g/p - 1 and local 0 of
// cell g/p; any other index is local g % p + 1 of cell g/p alone.
struct CellsOf {
  int cnt;
  int cell[2], loc[2];
};

__device__ __forceinline__ CellsOf cells_of(int g, int n, int p, const FastDiv dp) {
  CellsOf c;
  c.cnt = 0;
  const int e = (int)fdiv((uint32_t)g, dp), rem = g - e * p;
  if (rem == 0) {
    if (e >= 1) {
      c.cell[c.cnt] = e - 1;
      c.loc[c.cnt] = 1;
      ++c.cnt;
    }
    if (e < n) {
      c.cell[c.cnt] = e;
      c.loc[c.cnt] = 0;
      ++c.cnt;
    }
  } else {
    c.cell[0] = e;
    c.loc[0] = rem + 1;
    c.cnt = 1;
  }
  return c;
}

// Node tiles of the lattice pull: 16 x 4 x 4 nodes (3-D) or 32 x 8 (2-D)
// per 256-thread workgroup, so the cells whose block outputs a workgroup
// sums are mostly summed by that workgroup alone.  The tile counts along the
// first two directions are the divisors of L.dtx and L.dty.
__host__ __device__ __forceinline__ int64_t pull_num_tiles(const PullLattice L) {
  const int64_t ntz = L.dim == 3 ? (L.n1 + 3) / 4 : 1;
  return (int64_t)L.dtx.d * L.dty.d * ntz;
}

// Node of slot `slot` (0 .. 255) of tile `tile` (one unknown per node: the
// lattice pull serves scalar problems): a tile's nodes are taken row by row
// (TX consecutive nodes), which keeps the vector accesses of consecutive
// lanes contiguous.  The tile sizes are powers of two and the tile counts
// are divided by multiply-shift.  False when the node lies outside the
// lattice.
__device__ __forceinline__ bool pull_node(const PullLattice L, int64_t tile, int slot, int* gx,
                                          int* gy, int* gz) {
  const uint32_t t = (uint32_t)tile;   // fewer than 2^31 tiles
  const uint32_t tyz = fdiv(t, L.dtx), bz = fdiv(tyz, L.dty);
  const int bx = (int)(t - tyz * L.dtx.d), by = (int)(tyz - bz * L.dty.d);
  const int sx = L.dim == 3 ? 4 : 5, sy = L.dim == 3 ? 2 : 3;   // log2 TX, log2 TY
  const int row = slot >> sx;
  *gx = (bx << sx) + (slot & ((1 << sx) - 1));
  *gy = (by << sy) + (row & ((1 << sy) - 1));
  *gz = L.dim == 3 ? (int)(bz << 2) + (row >> sy) : (int)bz + (row >> sy);
  return *gx < L.n1 && *gy < L.n1 && (L.dim < 3 ? *gz == 0 : *gz < L.n1);
}

// Sum of the block outputs y_B holding node (gx, gy, gz), in ascending
// block (= cell) order, as the node-to-block map lists them.  All (at most
// eight) loads are issued before the ordered sum.
__device__ __forceinline__ double pull_lattice_sum(const double* __restrict__ y,
                                                   const PullLattice L, int m, int gx, int gy,
                                                   int gz) {
  const CellsOf cx = cells_of(gx, L.n, L.p, L.dp);
  CellsOf cy{1, {0, 0}, {0, 0}}, cz{1, {0, 0}, {0, 0}};
  if (L.dim >= 2) cy = cells_of(gy, L.n, L.p, L.dp);
  if (L.dim >= 3) cz = cells_of(gz, L.n, L.p, L.dp);
  const int p1 = L.p + 1;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ix = k & 1, iy = (k >> 1) & 1, iz = k >> 2;
    const bool on = ix < cx.cnt && iy < cy.cnt && iz < cz.cnt;
    v[k] = 0.0;
    if (on) {
      const int64_t e =
          cx.cell[ix] + (int64_t)L.n * (cy.cell[iy] + (int64_t)L.n * cz.cell[iz]);
      const int loc = cx.loc[ix] + p1 * (cy.loc[iy] + p1 * cz.loc[iz]);
      v[k] = y[e * m + loc];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ix = k & 1, iy = (k >> 1) & 1, iz = k >> 2;
    if (ix < cx.cnt && iy < cy.cnt && iz < cz.cnt) s += v[k];
  }
  return s;
}

// Node of local function loc of cell e on a lattice whose cells are the
// blocks, in order (the inverse of cells_of: local index 0 is a cell's
// left vertex, 1 its right vertex, 2 .. p its interior indices, tensor
// order with the first direction fastest).
__device__ __forceinline__ int64_t lattice_cell_node(const PullLattice L, int e, int loc) {
  int64_t node = 0, stride = 1;
  uint32_t ee = (uint32_t)e, ll = (uint32_t)loc;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < L.dim) {
      const uint32_t eq = fdiv(ee, L.dn), lq = fdiv(ll, L.dp1);
      const int c = (int)(ee - eq * (uint32_t)L.n), l = (int)(ll - lq * (uint32_t)(L.p + 1));
      ee = eq;
      ll = lq;
      const int g = c * L.p + (l == 0 ? 0 : l == 1 ? L.p : l - 1);
      node += g * stride;
      stride *= L.n1;
    }
  }
  return node;
}

// Unknown of row i of a block whose node list starts at nodes[e * nn]
// (element blocks, or vertex patches whose lists are padded with -1 at the
// boundary): -1 for a padding row.
__device__ __forceinline__ int64_t block_dof(const int32_t* __restrict__ nodes, int64_t e, int nn,
                                             int bd, int i) {
  const int32_t nd = nodes[e * nn + i / bd];
  return nd < 0 ? int64_t(-1) : (int64_t)nd * bd + (i % bd);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}

}  // namespace fc
