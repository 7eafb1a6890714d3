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
//     even the row k = m/2 holds every pair twice and is used once.  For
//     m <= 64 (one lane per column) the stored rows are kept in pairs,
//     rows 2j and 2j + 1 interleaved column by column, so a lane reads two
//     of its entries with one load (sym_offset).
//   * Dense layout: lane i accumulates sum_j P_B[j][i] r_B[j] (row j of a
//     symmetric matrix is its column j) reading P_B row by row.
//   * FP32: the same wrapped diagonals of the diagonally scaled inverse
//     D^{1/2} P_B D^{1/2} rounded to FP32 (FP32 accumulation), applied as
//     D^{-1/2} (.) D^{-1/2}; blocks whose rounded copy is not certified
//     positive definite are skipped there and done from the FP64 copy.
//   * BF16: the scaled Cholesky factor of the same matrix, two triangular
//     passes through LDS (positive semi-definite however rounded).
//   Every block reads its own stored inverse once per apply.
// Phase 2 (pull): every unknown sums the y_B entries of the blocks that
// contain it, in a fixed order (no atomics, bitwise reproducible), and adds
// its diagonal-scaling term.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "dev_common.h"
#include "k_schwarz.h"
#include "schwarz_dev.h"

namespace fc {

// m > 64: one workgroup of 64*ceil(m/64) threads per block.
template <typename T, bool kSym>
__global__ __launch_bounds__(256) void k_schwarz_large(
    const T* __restrict__ P, int64_t block_stride, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    const double* __restrict__ r, const double* __restrict__ q, const double* __restrict__ isd,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks) {
  __shared__ double rB[256];
  if (sc && sc->done) return;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  if (blk >= n_blocks) return;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int i = threadIdx.x;
  const int64_t e = block_elem[blk];
  int64_t dof = -1;
  if (i < m) {
    dof = block_dof(elem_nodes, e, nn, bd, i);
    rB[i] = dof >= 0 ? gather_r(r, q, alpha, dof) * (isd ? isd[dof] : 1.0) : 0.0;
  }
  __syncthreads();
  if (i >= m) return;
  const T* Pb = P + blk * block_stride;
  const double v = kSym ? sym_row<T>(Pb, rB, m, i) : dense_row<T>(Pb, rB, m, i);
  y[blk * m + i] = dof < 0 ? 0.0 : isd ? v * isd[dof] : v;
}

// m > 64, symmetric layout staged through LDS.  kRuns: 16-byte runs of the
// chunk per thread (sym_block_staged_runs), else every thread's own entry of
// each stored row (sym_block_staged_rows); launch_staged picks by block size.
template <typename T, bool kRuns>
__global__ __launch_bounds__(256) void k_schwarz_sym_staged(
    const T* __restrict__ P, int64_t block_stride, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    const double* __restrict__ r, const double* __restrict__ q, const double* __restrict__ isd,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks,
    const int32_t* __restrict__ list, const int32_t* __restrict__ skip) {
  using A = typename Acc<T>::type;
  constexpr int kStageRows = StageRows<T>::value;
  // the gathered residual is kept in the accumulation type: an FP32 copy
  // rounds it to FP32 at every use anyway, and half-width entries halve the
  // LDS traffic of the rotated reads
  __shared__ A rB[256];
  __shared__ __align__(16) T tile[kStageRows * 256];
  if (sc && sc->done) return;
  // list: the workgroups handle only the listed blocks; skip: blocks
  // flagged there are left to another launch
  const int64_t blk = list ? (int64_t)list[blockIdx.x] : xcd_remap(blockIdx.x, gridDim.x);
  if (blk >= n_blocks) return;
  if (skip && skip[blk]) return;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int i = threadIdx.x;
  const bool act = i < m;
  const int64_t e = block_elem[blk];
  int64_t dof = -1;
  if (act) {
    dof = block_dof(elem_nodes, e, nn, bd, i);
    rB[i] = dof >= 0 ? (A)(gather_r(r, q, alpha, dof) * (isd ? isd[dof] : 1.0)) : A(0);
  }
  const T* Qb = P + blk * block_stride;
  const double v = kRuns ? sym_block_staged_runs<T, A>(Qb, rB, m, i, tile)
                         : sym_block_staged_rows<T, A>(Qb, rB, m, i, tile);
  if (act) y[blk * m + i] = dof < 0 ? 0.0 : isd ? v * isd[dof] : v;
}

// m <= 64: each wave handles floor(64/m) blocks, one lane per output row.
// kM > 0 (symmetric layout, m = kM known at compile time): lane i loads its
// column of the stored rows (Q_B[k][i] = P_B[i][(i + k) mod m], k = 0 ..
// m/2; two rows per load, as sym_offset pairs them) into registers before
// it gathers r_B, so the block's stream is in
// flight during the gather; the entries P_B[i][(i - k) mod m] =
// Q_B[k][(i - k) mod m] are then read from the lane that loaded them (a
// cross-lane read within the wave).  kM = 0: any m, the stored rows read
// after the gather (sym_row / dense_row).  kLat: the blocks are the cells of
// a lattice in order, so a row's unknown follows from the block and row
// indices and the gather of r_B is issued together with the stored rows.
template <typename T, bool kSym, int kM, bool kLat>
__global__ __launch_bounds__(256) void k_schwarz_small(
    const T* __restrict__ P, int64_t block_stride, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m_arg,
    const double* __restrict__ r, const double* __restrict__ q, const double* __restrict__ isd,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks,
    const PullLattice lat) {
  __shared__ double rB[4][64];
  if (sc && sc->done) return;
  const int m = kM > 0 ? kM : m_arg;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int bpw = 64 / m;
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  const int lb = l / m, i = l % m;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t blk = (tile * 4 + w) * bpw + lb;
  const bool active = lb < bpw && blk < n_blocks;
  // lanes without a block read block 0 (always present) and store nothing
  const T* Pb = P + (active ? blk : 0) * block_stride;
  using A = typename Acc<T>::type;
  constexpr int kH = kM / 2;
  T v[kH + 1];
  int64_t dof = -1;
  double rv = 0.0;
  double g_r = 0.0, g_q = 0.0, g_s = 1.0;
  if constexpr (kLat) {
    // the gathered entries are loaded first and the stored rows next, all
    // without branches (a lane without a block reads unknown 0), and only
    // then combined: the wait for the gather does not wait for the rows
    // (the lattice is set for scalar problems only: one unknown per node)
    dof = active ? lattice_cell_node(lat, (int)blk, i) : 0;
    g_r = r[dof];
    g_q = (q ? q : r)[dof];
    g_s = (isd ? isd : r)[dof];
  }
  if constexpr (kSym && kM > 0) {
    // stored rows in pairs (sym_offset, m <= 64): one two-wide load each
    constexpr int kNP = (kH + 1) & ~1;
    typedef T t2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
#pragma unroll
    for (int k = 0; k < kNP; k += 2) {
      const t2 t = *reinterpret_cast<const t2*>(Pb + k * kM + 2 * i);
      v[k] = t.x;
      v[k + 1] = t.y;
    }
    if constexpr (kNP < kH + 1) v[kH] = Pb[kH * kM + i];
  }
  if constexpr (kLat) {
    rv = (q ? fma(-alpha, g_q, g_r) : g_r) * (isd ? g_s : 1.0);
  } else {
    if (active) {
      dof = block_dof(elem_nodes, block_elem[blk], nn, bd, i);
      rv = dof >= 0 ? gather_r(r, q, alpha, dof) * (isd ? isd[dof] : 1.0) : 0.0;
    }
  }
  if (active) rB[w][l] = rv;
  __syncthreads();
  double out;
  if constexpr (kSym && kM > 0) {
    // every lane takes part in the cross-lane reads; a lane without a block
    // reads its own group's entries and discards the result
    const int g0 = (active ? lb : 0) * kM;
    const double* rb = &rB[w][g0];
    A acc0 = madd<A>(v[0], rb[i], A(0)), acc1 = 0;
#pragma unroll
    for (int k = 1; k <= kH; ++k) {
      const int ip = i + k < kM ? i + k : i + k - kM;   // (i + k) mod m
      const int im = i >= k ? i - k : i - k + kM;       // (i - k) mod m
      const T vr = __shfl(v[k], g0 + im, 64);
      acc0 = madd<A>(v[k], rb[ip], acc0);
      if (!((kM & 1) == 0 && k == kH)) acc1 = madd<A>(vr, rb[im], acc1);
    }
    out = (double)acc0 + (double)acc1;
  } else {
    if (!active) return;
    const double* rb = &rB[w][lb * m];
    out = kSym ? sym_row<T>(Pb, rb, m, i) : dense_row<T>(Pb, rb, m, i);
  }
  if (!active) return;
  y[blk * m + i] = dof < 0 ? 0.0 : isd ? out * isd[dof] : out;
}

// Factored low-precision product y_B = D^{-1/2} Lt (Lt^T (D^{-1/2} r_B)) with
// Lt packed by subdiagonals (k_setup.hip).  The whole packed factor of a
// block is staged in LDS with 16-byte loads, then both triangular passes
// read it from LDS:
//   t_j = sum_d Lt[off_d + j] r_{j+d}        (lane j, d = 0 .. m-1-j)
//   y_i = sum_d Lt[off_d + i - d] t_{i-d}    (lane i, d = 0 .. i)
// Each pass reads consecutive LDS words across lanes.  FP32 accumulation.
template <typename T>
__device__ __forceinline__ void stage_packed(const T* __restrict__ src, T* dst, int64_t count,
                                             int tid, int nt) {
  // 16-byte chunks where the block start is 16-byte aligned, else scalar
  const uintptr_t addr = reinterpret_cast<uintptr_t>(src);
  constexpr int V = 16 / sizeof(T);
  if ((addr % 16) == 0) {
    const int64_t nv = count / V;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
    u32x4* d4 = reinterpret_cast<u32x4*>(dst);
    for (int64_t c = tid; c < nv; c += nt) d4[c] = __builtin_nontemporal_load(s4 + c);
    for (int64_t c = nv * V + tid; c < count; c += nt) dst[c] = src[c];
  } else {
    for (int64_t c = tid; c < count; c += nt) dst[c] = __builtin_nontemporal_load(src + c);
  }
}

template <typename T>
__device__ __forceinline__ float ld_f32(const T* p) {
  if constexpr (sizeof(T) == 4)
    return *p;
  else
    return bf16_to_f32(*p);
}

// One block per workgroup (m > 64) or several per wave (m <= 64): the
// caller sets up rb (scaled gathered residual) and the staged factor Lb.
template <typename T>
__device__ __forceinline__ float chol_pass1(const T* Lb, const float* rb, int m, int j) {
  float t0 = 0.f, t1 = 0.f;
  int64_t off = 0;
  int d = 0;
  for (; d + 1 <= m - 1 - j; d += 2) {
    t0 = fmaf(ld_f32(Lb + off + j), rb[j + d], t0);
    off += m - d;
    t1 = fmaf(ld_f32(Lb + off + j), rb[j + d + 1], t1);
    off += m - d - 1;
  }
  if (d <= m - 1 - j) t0 = fmaf(ld_f32(Lb + off + j), rb[j + d], t0);
  return t0 + t1;
}

template <typename T>
__device__ __forceinline__ float chol_pass2(const T* Lb, const float* tb, int m, int i) {
  float y0 = 0.f, y1 = 0.f;
  int64_t off = 0;
  int d = 0;
  for (; d + 1 <= i; d += 2) {
    y0 = fmaf(ld_f32(Lb + off + i - d), tb[i - d], y0);
    off += m - d;
    y1 = fmaf(ld_f32(Lb + off + i - d - 1), tb[i - d - 1], y1);
    off += m - d - 1;
  }
  if (d <= i) y0 = fmaf(ld_f32(Lb + off + i - d), tb[i - d], y0);
  return y0 + y1;
}

constexpr int kCholLdsBytes = 75000;   // FP32 factor of m = 192: 74,112 bytes

template <typename T>
__global__ __launch_bounds__(256) void k_schwarz_chol_large(
    const T* __restrict__ L, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    const double* __restrict__ r, const double* __restrict__ q, const double* __restrict__ isd,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  __shared__ float rb[256], tb[256];
  if (sc && sc->done) return;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  if (blk >= n_blocks) return;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int i = threadIdx.x;
  const int64_t per = (int64_t)m * (m + 1) / 2;
  T* Lb = reinterpret_cast<T*>(dyn_lds);
  stage_packed<T>(L + blk * per, Lb, per, i, blockDim.x);
  const int64_t e = block_elem[blk];
  int64_t dof = 0;
  double s = 1.0;
  if (i < m) {
    dof = (int64_t)elem_nodes[e * nn + i / bd] * bd + (i % bd);
    s = isd[dof];
    rb[i] = (float)(gather_r(r, q, alpha, dof) * s);
  }
  __syncthreads();
  if (i < m) tb[i] = chol_pass1<T>(Lb, rb, m, i);
  __syncthreads();
  if (i < m) y[blk * m + i] = (double)chol_pass2<T>(Lb, tb, m, i) * s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_schwarz_chol_small(
    const T* __restrict__ L, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    const double* __restrict__ r, const double* __restrict__ q, const double* __restrict__ isd,
    const CgScalars* __restrict__ sc, double* __restrict__ y, int64_t n_blocks) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  __shared__ float rb[4][64], tb[4][64];
  if (sc && sc->done) return;
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int bpw = 64 / m;
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  const int lb = l / m, i = l % m;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t blk0 = tile * 4 * bpw;                 // first block of the workgroup
  const int64_t nwb = std::min<int64_t>(4 * bpw, n_blocks - blk0);
  const int64_t per = (int64_t)m * (m + 1) / 2;
  T* Ls = reinterpret_cast<T*>(dyn_lds);
  if (nwb > 0) stage_packed<T>(L + blk0 * per, Ls, nwb * per, threadIdx.x, blockDim.x);
  const int64_t blk = (tile * 4 + w) * bpw + lb;
  const bool active = lb < bpw && blk < n_blocks;
  int64_t dof = 0;
  double s = 1.0;
  if (active) {
    const int64_t e = block_elem[blk];
    dof = (int64_t)elem_nodes[e * nn + i / bd] * bd + (i % bd);
    s = isd[dof];
    rb[w][l] = (float)(gather_r(r, q, alpha, dof) * s);
  }
  __syncthreads();
  const T* Lb = Ls + (blk - blk0) * per;
  if (active) tb[w][l] = chol_pass1<T>(Lb, &rb[w][lb * m], m, i);
  __syncthreads();
  if (active) y[blk * m + i] = (double)chol_pass2<T>(Lb, &tb[w][lb * m], m, i) * s;
}

template <typename T>
static hipError_t phase1_chol(const fc_precond_s& pc, const T* L, const double* r,
                              const double* q, const CgScalars* sc, hipStream_t s) {
  const fc_problem_s& pb = *pc.pb;
  if (pc.n_blocks == 0) return hipSuccess;
  const int m = pc.m;
  const int64_t per = (int64_t)m * (m + 1) / 2;
  if (m > 64) {
    const int threads = 64 * ((m + 63) / 64);
    const size_t lds = (size_t)per * sizeof(T);
    (void)hipFuncSetAttribute((const void*)k_schwarz_chol_large<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_schwarz_chol_large<T>, dim3((unsigned)pc.n_blocks), dim3(threads), lds,
                       s, L, block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, m, r, q, pc.isd, sc,
                       pc.y, pc.n_blocks);
  } else {
    const int bpw = 64 / m;
    const int64_t per_wg = 4 * (int64_t)bpw;
    const int64_t nwg = (pc.n_blocks + per_wg - 1) / per_wg;
    const size_t lds = (size_t)(per_wg * per) * sizeof(T);
    (void)hipFuncSetAttribute((const void*)k_schwarz_chol_small<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_schwarz_chol_small<T>, dim3((unsigned)nwg), dim3(256), lds, s, L,
                       block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, m, r, q, pc.isd, sc, pc.y,
                       pc.n_blocks);
  }
  return hipGetLastError();
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

// Wrapped-diagonal copy: entry (k, i) of block blk, P[blk][i][(i+k) mod m]
// for k <= m/2, at Q[blk * (m/2 + 1) m + sym_offset(k, i, m)].
// With isd (low-precision copies) the stored block is the diagonally
// scaled D^{1/2} P_B D^{1/2} (D = diag(A) on the block's unknowns, isd =
// D^{-1/2}), which removes the 1/alpha dynamic range of fictitious
// functions before rounding; the apply undoes the scaling in FP64.
template <typename T>
__global__ void k_pack_sym(const double* __restrict__ P, T* __restrict__ Q, int m,
                           int64_t n_blocks, const double* __restrict__ isd,
                           const int32_t* __restrict__ elem_nodes,
                           const int32_t* __restrict__ block_elem, int nn, int bd) {
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
    double v = P[blk * (int64_t)m * m + (int64_t)i * m + j];
    if (isd) {
      const int64_t e = block_elem[blk];
      const int64_t di = block_dof(elem_nodes, e, nn, bd, i);
      const int64_t dj = block_dof(elem_nodes, e, nn, bd, j);
      v = (di < 0 || dj < 0) ? 0.0 : v / (isd[di] * isd[dj]);
    }
    const int64_t dst = blk * per + sym_offset(k, i, m);
    if constexpr (sizeof(T) == 8) {
      Q[dst] = v;
    } else if constexpr (sizeof(T) == 4) {
      Q[dst] = (float)v;
    } else {
      // FP64 -> BF16 through FP32, round to nearest even
      uint32_t u = __float_as_uint((float)v);
      u += 0x7fffu + ((u >> 16) & 1u);
      Q[dst] = (T)(u >> 16);
    }
  }
}

int64_t sym_block_stride(int m) { return (int64_t)(m / 2 + 1) * m; }

hipError_t launch_pack_sym(const fc_precond_s& pc, void* Q, int precision, hipStream_t s) {
  const int64_t nb = pc.n_blocks;
  const int m = pc.m;
  if (nb == 0) return hipSuccess;
  dim3 g(8192), b(256);
  const int32_t* en = block_nodes(pc);
  switch (precision) {
    case 0:
      hipLaunchKernelGGL(k_pack_sym<double>, g, b, 0, s, pc.P, (double*)Q, m, nb, nullptr, en,
                         pc.block_elem, pc.nn, pc.bdim);
      break;
    case 1:
      hipLaunchKernelGGL(k_pack_sym<float>, g, b, 0, s, pc.P, (float*)Q, m, nb, pc.isd, en,
                         pc.block_elem, pc.nn, pc.bdim);
      break;
    case 2:
      hipLaunchKernelGGL(k_pack_sym<uint16_t>, g, b, 0, s, pc.P, (uint16_t*)Q, m, nb, pc.isd, en,
                         pc.block_elem, pc.nn, pc.bdim);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// rows whose unknown differs from the lattice's (counted with an atomic only
// where one occurs)
__global__ void k_check_cell_lattice(const int32_t* __restrict__ nodes,
                                     const int32_t* __restrict__ block_elem, int nn, int bd,
                                     int m, int64_t n_blocks, const PullLattice L,
                                     unsigned long long* __restrict__ bad) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_blocks * m;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / m;
    const int i = (int)(t - b * m);
    const int64_t want = lattice_cell_node(L, (int)b, i / bd) * bd + i % bd;
    if (block_elem[b] != b || block_dof(nodes, b, nn, bd, i) != want) atomicAdd(bad, 1ull);
  }
}

hipError_t schwarz_check_lattice(const fc_precond_s& pc, const PullLattice L, bool* ok,
                                 hipStream_t s) {
  *ok = false;
  if (pc.n_blocks == 0) return hipSuccess;
  unsigned long long* bad = nullptr;
  hipError_t e = hipMalloc(&bad, sizeof(*bad));
  if (e != hipSuccess) return e;
  unsigned long long hbad = 1;
  e = hipMemsetAsync(bad, 0, sizeof(*bad), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_check_cell_lattice, dim3(2048), dim3(256), 0, s, block_nodes(pc),
                       pc.block_elem, pc.nn, pc.bdim, pc.m, pc.n_blocks, L, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(bad);
  *ok = e == hipSuccess && hbad == 0;
  return e;
}

__global__ void k_inv_sqrt_diag(const double* __restrict__ d, double* __restrict__ isd, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    isd[i] = d[i] > 0.0 ? 1.0 / sqrt(d[i]) : 1.0;
}

hipError_t launch_inv_sqrt_diag(const fc_problem_s& pb, double* isd, hipStream_t s) {
  hipLaunchKernelGGL(k_inv_sqrt_diag, dim3(1024), dim3(256), 0, s, pb.diag, isd, pb.n_dofs);
  return hipGetLastError();
}

// Loading scheme of the staged product by block size (measured on MI355X):
// 16-byte runs for m = 192 (32^3-cell p = 3 elasticity, 1.5 % faster than
// per-thread rows), per-thread rows for m = 125 (4.5 % faster than runs in a
// 64-member Poisson batch).  One scheme per compiled kernel: a kernel holding
// both ran the m = 192 products 12 % slower.
inline bool staged_runs(int m) { return m > 128; }

template <typename T>
static void launch_staged(const fc_precond_s& pc, const T* Q, int64_t n_launch,
                          const double* r, const double* q, const double* isd,
                          const CgScalars* sc, const int32_t* list, const int32_t* skip,
                          hipStream_t s) {
  const dim3 g((unsigned)n_launch), b(64 * ((pc.m + 63) / 64));
  if (staged_runs(pc.m))
    hipLaunchKernelGGL((k_schwarz_sym_staged<T, true>), g, b, 0, s, Q, sym_block_stride(pc.m),
                       block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, pc.m, r, q, isd, sc, pc.y,
                       pc.n_blocks, list, skip);
  else
    hipLaunchKernelGGL((k_schwarz_sym_staged<T, false>), g, b, 0, s, Q, sym_block_stride(pc.m),
                       block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, pc.m, r, q, isd, sc, pc.y,
                       pc.n_blocks, list, skip);
}

template <typename T, bool kSym>
static hipError_t phase1(const fc_precond_s& pc, const T* P, const double* r, const double* q,
                         const CgScalars* sc, hipStream_t s) {
  const double* isd = sizeof(T) == 8 ? nullptr : pc.isd;
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
      launch_staged<T>(pc, P, pc.n_blocks, r, q, isd, sc, nullptr,
                       sizeof(T) == 4 ? pc.unsafe_flag32 : nullptr, s);
    else
      hipLaunchKernelGGL((k_schwarz_large<T, kSym>), dim3((unsigned)pc.n_blocks), dim3(threads),
                         0, s, P, stride, block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, pc.m, r,
                         q, isd, sc, pc.y, pc.n_blocks);
  } else {
    const int bpw = 64 / pc.m;
    const int64_t per_wg = 4 * (int64_t)bpw;
    const int64_t nwg = (pc.n_blocks + per_wg - 1) / per_wg;
    // the block sizes of scalar and vector problems at p = 1..3 (2-D and
    // 3-D) have their own compiled kernels
    const bool lat = pc.lat.dim > 0;
#define FC_SMALL_LAUNCH(KM)                                                                    \
  do {                                                                                         \
    if (lat && KM > 0)                                                                         \
      hipLaunchKernelGGL((k_schwarz_small<T, kSym, KM, true>), dim3((unsigned)nwg), dim3(256), \
                         0, s, P, stride, block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, pc.m, \
                         r, q, isd, sc, pc.y, pc.n_blocks, pc.lat);                            \
    else                                                                                       \
      hipLaunchKernelGGL((k_schwarz_small<T, kSym, KM, false>), dim3((unsigned)nwg),           \
                         dim3(256), 0, s, P, stride, block_nodes(pc), pc.block_elem, pc.nn,    \
                         pc.bdim, pc.m, r, q, isd, sc, pc.y, pc.n_blocks, pc.lat);             \
  } while (0)
    switch (kSym ? pc.m : 0) {
      case 8: FC_SMALL_LAUNCH(8); break;
      case 9: FC_SMALL_LAUNCH(9); break;
      case 16: FC_SMALL_LAUNCH(16); break;
      case 18: FC_SMALL_LAUNCH(18); break;
      case 24: FC_SMALL_LAUNCH(24); break;
      case 25: FC_SMALL_LAUNCH(25); break;
      case 27: FC_SMALL_LAUNCH(27); break;
      case 32: FC_SMALL_LAUNCH(32); break;
      case 36: FC_SMALL_LAUNCH(36); break;
      case 49: FC_SMALL_LAUNCH(49); break;
      case 50: FC_SMALL_LAUNCH(50); break;
      case 64: FC_SMALL_LAUNCH(64); break;
      default: FC_SMALL_LAUNCH(0); break;
    }
#undef FC_SMALL_LAUNCH
  }
  return hipGetLastError();
}

// FP64 symmetric product for the listed blocks (those whose FP32 copy is
// not used), one workgroup per block.
__global__ __launch_bounds__(256) void k_schwarz_sym_list(
    const double* __restrict__ Q, int64_t stride, const int32_t* __restrict__ list,
    const int32_t* __restrict__ elem_nodes, const int32_t* __restrict__ block_elem, int nn,
    int bd, int m, const double* __restrict__ r, const double* __restrict__ q,
    const CgScalars* __restrict__ sc, double* __restrict__ y) {
  __shared__ double rB[256];
  if (sc && sc->done) return;
  const int64_t blk = list[blockIdx.x];
  const double alpha = (sc && q) ? sc->alpha : 0.0;
  const int i = threadIdx.x;
  if (i < m) {
    const int64_t e = block_elem[blk];
    const int64_t dof = block_dof(elem_nodes, e, nn, bd, i);
    rB[i] = dof >= 0 ? gather_r(r, q, alpha, dof) : 0.0;
  }
  __syncthreads();
  if (i < m) y[blk * m + i] = sym_row<double>(Q + blk * stride, rB, m, i);
}

hipError_t launch_schwarz_phase1(const fc_precond_s& pc, int precision, const double* r,
                                 const double* q, const CgScalars* sc, hipStream_t s) {
  switch (precision) {
    case 0:
      if (pc.Q) return phase1<double, true>(pc, pc.Q, r, q, sc, s);
      return phase1<double, false>(pc, pc.P, r, q, sc, s);
    case 1: {
      if (!pc.Q32 || !pc.Q) return hipErrorInvalidValue;
      hipError_t e = phase1<float, true>(pc, pc.Q32, r, q, sc, s);
      if (e != hipSuccess || pc.n_unsafe32 == 0) return e;
      const fc_problem_s& pb = *pc.pb;
      if (pc.m > 64)
        launch_staged<double>(pc, pc.Q, pc.n_unsafe32, r, q, nullptr, sc, pc.unsafe32, nullptr, s);
      else
        hipLaunchKernelGGL(k_schwarz_sym_list, dim3((unsigned)pc.n_unsafe32),
                           dim3(64 * ((pc.m + 63) / 64)), 0, s, pc.Q, sym_block_stride(pc.m),
                           pc.unsafe32, block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, pc.m, r, q,
                           sc, pc.y);
      return hipGetLastError();
    }
    case 2:
      if (!pc.Lbf) return hipErrorInvalidValue;
      return phase1_chol<uint16_t>(pc, pc.Lbf, r, q, sc, s);
  }
  return hipErrorInvalidValue;
}

// The same where every cell is a block (lattice pull, see k_cg_pull_lat;
// scalar problems only).
__global__ __launch_bounds__(256) void k_schwarz_pull_lat(const double* __restrict__ y,
                                                          const PullLattice L, int m,
                                                          const double* __restrict__ fb,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ z) {
  const int64_t ntiles = pull_num_tiles(L);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int gx, gy, gz;
    if (!pull_node(L, tile, threadIdx.x, &gx, &gy, &gz)) continue;
    const double sv = pull_lattice_sum(y, L, m, gx, gy, gz);
    const int64_t i = gx + (int64_t)L.n1 * (gy + (int64_t)L.n1 * gz);
    z[i] = fb ? fma(fb[i], r[i], sv) : sv;
  }
}

hipError_t launch_schwarz_pull(const fc_precond_s& pc, const double* r, double* z,
                               hipStream_t s) {
  const int64_t n = pc.pb->n_dofs;
  if (n == 0) return hipSuccess;
  if (pc.lat.dim > 0) {
    if (pc.bdim != 1) return hipErrorInvalidValue;
    const dim3 g((unsigned)std::min<int64_t>(pull_num_tiles(pc.lat), 4096)), b(256);
    const double* fb = pc.n_fallback ? pc.fallback : nullptr;
    hipLaunchKernelGGL(k_schwarz_pull_lat, g, b, 0, s, pc.y, pc.lat, pc.m, fb, r, z);
    return hipGetLastError();
  }
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
