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

// The cells holding lattice index g along one direction (at most two, in
// ascending order) and the function's local index on each: a vertex index
// (g a multiple of p) is local 1 (right end) of cell g/p - 1 and local 0 of
// cell g/p; any other index is local g % p + 1 of cell g/p alone.
struct CellsOf {
  int cnt;
  int cell[2], loc[2];
};

__device__ __forceinline__ CellsOf cells_of(int g, int n, int p) {
  CellsOf c;
  c.cnt = 0;
  if (g % p == 0) {
    const int e = g / p;
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
    c.cell[0] = g / p;
    c.loc[0] = g % p + 1;
    c.cnt = 1;
  }
  return c;
}

// Node tiles of the lattice pull: 16 x 4 x 4 nodes (3-D) or 32 x 8 (2-D)
// per 256-thread workgroup, so the cells whose block outputs a workgroup
// sums are mostly summed by that workgroup alone.
struct PullTiles {
  int TX, TY, TZ, ntx, nty, ntz;
};

__host__ __device__ __forceinline__ PullTiles pull_tiles(const PullLattice L) {
  PullTiles t;
  t.TX = L.dim == 3 ? 16 : 32;
  t.TY = L.dim == 3 ? 4 : 8;
  t.TZ = L.dim == 3 ? 4 : 1;
  t.ntx = (L.n1 + t.TX - 1) / t.TX;
  t.nty = (L.n1 + t.TY - 1) / t.TY;
  t.ntz = L.dim == 3 ? (L.n1 + t.TZ - 1) / t.TZ : 1;
  return t;
}

// Unknown of slot `slot` (0 .. TX*TY*TZ*BD - 1) of tile `tile`: a tile's
// unknowns are taken row by row (TX consecutive nodes, components
// interleaved, so each row is one contiguous run of TX*BD unknowns), which
// keeps the vector accesses of consecutive lanes contiguous.  False when the
// node lies outside the lattice.
template <int BD>
__device__ __forceinline__ bool pull_dof(const PullLattice L, const PullTiles T, int64_t tile,
                                         int slot, int* gx, int* gy, int* gz, int* c) {
  const int t = (int)tile;   // fewer than 2^31 tiles: n1 <= 2^21 nodes per direction
  const int bx = t % T.ntx, by = (t / T.ntx) % T.nty;
  const int bz = t / (T.ntx * T.nty);
  const int row = slot / (T.TX * BD), o = slot - row * (T.TX * BD);
  *gx = bx * T.TX + o / BD;
  *c = o % BD;
  *gy = by * T.TY + row % T.TY;
  *gz = bz * T.TZ + row / T.TY;
  return *gx < L.n1 && *gy < L.n1 && (L.dim < 3 ? *gz == 0 : *gz < L.n1);
}

// Sum of the block outputs y_B holding component c of node (gx, gy, gz), in
// ascending block (= cell) order, as the node-to-block map lists them.  All
// (at most eight) loads are issued before the ordered sum.
__device__ __forceinline__ double pull_lattice_sum(const double* __restrict__ y,
                                                   const PullLattice L, int m, int bd, int gx,
                                                   int gy, int gz, int c) {
  const CellsOf cx = cells_of(gx, L.n, L.p);
  CellsOf cy{1, {0, 0}, {0, 0}}, cz{1, {0, 0}, {0, 0}};
  if (L.dim >= 2) cy = cells_of(gy, L.n, L.p);
  if (L.dim >= 3) cz = cells_of(gz, L.n, L.p);
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
      v[k] = y[e * m + (int64_t)loc * bd + c];
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
