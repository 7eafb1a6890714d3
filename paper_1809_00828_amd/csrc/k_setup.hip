// Set-up of the additive Schwarz preconditioner on the device
// (Algorithm 1 of the paper, Sec. 4.3):
//   extractSubMatrix      A_B = R_B A R_B^T gathered from the BSR matrix
//   computePseudoInverse  the stabilised local inverse of Eqs. (9)-(11):
//                         eigen-decompose A_B, drop eigenvalues at or below
//                         eps * max eigenvalue, sum 1/lambda v v^T
//   diagonal scaling      1/A_ll for every unknown whose entry S_ll is zero
//
// Local inverses are computed in one of two ways, both FP64:
//  * a certified direct inverse.  The block is inverted by the symmetric
//    sweep operator in registers: one wave per block with a column per
//    lane for m <= 64, a 512-thread workgroup (a 16 x 32 grid of tiles)
//    for 64 < m <= 192.  The result is accepted only when every pivot is
//    positive and trace(P) * ||A_B||_inf * eps * 4 < 1.  Since
//    lambda_min >= 1/trace(A_B^-1) and lambda_max <= ||A_B||_inf, that
//    certificate proves no eigenvalue lies within a factor 4 of the
//    threshold, so the pseudo-inverse equals the inverse.
//  * cyclic two-sided Jacobi eigen-decomposition (parallel round-robin
//    ordering, m/2 disjoint rotations per step), then
//    P_B = V diag(1/lambda_+) V^T: for the blocks that fail the
//    certificate, and for every block of the unstabilised inverse when
//    m <= 64.  The block and its eigenvectors stay in LDS when they fit,
//    else in global memory.
#include "dev_common.h"
#include "k_setup.h"

namespace fc {

// ---------------------------------------------------------- extraction
__global__ __launch_bounds__(256) void k_block_extract(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ elem_nodes,
    const int32_t* __restrict__ block_elem, int nn, int bd, int m,
    double* __restrict__ out) {
  const int64_t blk = blockIdx.x;
  const int64_t e = block_elem[blk];
  const int32_t* en = elem_nodes + e * nn;
  double* Ab = out + blk * (int64_t)m * m;
  const int bb = bd * bd;
  for (int t = threadIdx.x; t < nn * nn; t += blockDim.x) {
    const int a = t / nn, b = t % nn;
    const int32_t na = en[a], nb = en[b];
    if (na < 0 || nb < 0) {
      // padding of a boundary vertex patch: zero rows and columns, whose
      // zero eigenvalues the threshold of Eq. 11 drops
      for (int i = 0; i < bd; ++i)
        for (int j = 0; j < bd; ++j) Ab[(int64_t)(a * bd + i) * m + (b * bd + j)] = 0.0;
      continue;
    }
    const int32_t lo = rowptr[na], hi = rowptr[na + 1];
    int32_t l = lo, h = hi - 1, found = -1;
    while (l <= h) {
      int32_t mid = (l + h) >> 1;
      int32_t c = col[mid];
      if (c == nb) {
        found = mid;
        break;
      }
      if (c < nb) l = mid + 1;
      else h = mid - 1;
    }
    const int64_t L = hi - lo;
    for (int i = 0; i < bd; ++i)
      for (int j = 0; j < bd; ++j) {
        double v = 0.0;
        if (found >= 0) v = val[(int64_t)lo * bb + (int64_t)(i * bd + j) * L + (found - lo)];
        Ab[(int64_t)(a * bd + i) * m + (b * bd + j)] = v;
      }
  }
}

// ------------------------------------------------------- Jacobi eigen
// Pair `pi` of round-robin step `step` over mp (even) players.
__device__ __forceinline__ void rr_pair(int pi, int step, int mp, int* p, int* q) {
  auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + step) % (mp - 1); };
  int a = player(pi), b = player(mp - 1 - pi);
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

constexpr int kMaxJacobiM = 192;

// In: A_B in P[blk] (row-major m x m).  Out: P_B in place.  With kLds the
// block and eigenvectors live in dynamic LDS (m <= 64), otherwise in `work`
// (2*m*m doubles per workgroup).  sel (optional) lists the blocks to do.
template <bool kLds>
__global__ __launch_bounds__(256) void k_jacobi_pinv(
    double* __restrict__ P, int m, const int32_t* __restrict__ sel,
    double* __restrict__ work, double eps, int stabilize,
    int32_t* __restrict__ dropped) {
  extern __shared__ double dyn[];
  __shared__ double cs[kMaxJacobiM / 2 + 1], sn[kMaxJacobiM / 2 + 1];
  __shared__ int pp[kMaxJacobiM / 2 + 1], qq[kMaxJacobiM / 2 + 1];
  __shared__ double invl[kMaxJacobiM];
  __shared__ double red[16];
  __shared__ int rotated;
  const int64_t blk = sel ? sel[blockIdx.x] : blockIdx.x;
  double* Ab = P + blk * (int64_t)m * m;
  const int ld = kLds ? m + 1 : m;
  double* A = kLds ? dyn : work + (int64_t)blockIdx.x * 2 * m * m;
  double* V = A + (int64_t)m * ld;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int t = tid; t < m * m; t += nt) {
    const int i = t / m, j = t % m;
    A[i * ld + j] = Ab[t];
    V[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int mp = m + (m & 1), np = mp / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < mp - 1; ++step) {
      for (int pi = tid; pi < np; pi += nt) {
        int p, q;
        rr_pair(pi, step, mp, &p, &q);
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double app = A[p * ld + p], aqq = A[q * ld + q], apq = A[p * ld + q];
          if (apq != 0.0 && fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rotated = 1;
          }
        }
        cs[pi] = c;
        sn[pi] = s;
        pp[pi] = p;
        qq[pi] = q;
      }
      __syncthreads();
      // rows p, q of J^T A
      for (int t = tid; t < np * m; t += nt) {
        const int pi = t / m, j = t % m;
        const double s = sn[pi];
        if (s == 0.0) continue;
        const double c = cs[pi];
        const int p = pp[pi], q = qq[pi];
        const double apj = A[p * ld + j], aqj = A[q * ld + j];
        A[p * ld + j] = c * apj - s * aqj;
        A[q * ld + j] = s * apj + c * aqj;
      }
      __syncthreads();
      // columns p, q of (J^T A) J and of V J
      for (int t = tid; t < np * m; t += nt) {
        const int pi = t / m, i = t % m;
        const double s = sn[pi];
        if (s == 0.0) continue;
        const double c = cs[pi];
        const int p = pp[pi], q = qq[pi];
        const double aip = A[i * ld + p], aiq = A[i * ld + q];
        A[i * ld + p] = c * aip - s * aiq;
        A[i * ld + q] = s * aip + c * aiq;
        const double vip = V[i * ld + p], viq = V[i * ld + q];
        V[i * ld + p] = c * vip - s * viq;
        V[i * ld + q] = s * vip + c * viq;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // threshold of Eq. (11) relative to the largest eigenvalue of the block
  double lmax = -1e308;
  for (int k = tid; k < m; k += nt) lmax = fmax(lmax, A[k * ld + k]);
  {
    double v = lmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (tid % 64 == 0) red[tid / 64] = v;
    __syncthreads();
    v = -1e308;
    for (int w = 0; w < nt / 64; ++w) v = fmax(v, red[w]);
    lmax = v;
    __syncthreads();
  }
  int ndrop = 0;
  for (int k = tid; k < m; k += nt) {
    const double lam = A[k * ld + k];
    bool keep = stabilize ? (lmax > 0.0 && lam > eps * lmax) : (lam != 0.0);
    invl[k] = keep ? 1.0 / lam : 0.0;
    ndrop += keep ? 0 : 1;
  }
  __syncthreads();
  {
    double nd = block_sum((double)ndrop, red);
    if (tid == 0 && dropped) dropped[blk] = (int32_t)nd;
  }
  for (int t = tid; t < m * m; t += nt) {
    const int i = t / m, j = t % m;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc = fma(V[i * ld + k] * invl[k], V[j * ld + k], acc);
    Ab[t] = acc;
  }
}

// ------------------------------------------------- certified sweep inverse
// Sweep operator on a symmetric matrix: sweeping every pivot turns A into
// -A^{-1}.  Thread (ti, tj) of a 16 x 32 grid holds the 2T x T tile at rows
// ti*2T.., columns tj*T..; pivot row k is broadcast through LDS.  512
// threads leave each wave 256 registers, so a 12 x 6 FP64 tile (m = 192)
// stays in registers (with 1024 threads, 128 registers per wave, the 6 x 6
// tiles of the same block spill).
template <int T>
__global__ __launch_bounds__(512) void k_sweep_inverse(
    double* __restrict__ P, int m, double eps, int stabilize,
    int32_t* __restrict__ need_eig) {
  __shared__ double rowbuf[2][32 * T];
  __shared__ double red[16];
  const int64_t blk = blockIdx.x;
  double* Ab = P + blk * (int64_t)m * m;
  constexpr int TR = 2 * T;   // rows per thread
  const int tid = threadIdx.x, ti = tid / 32, tj = tid % 32;
  double a[TR][T];
#pragma unroll
  for (int r = 0; r < TR; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int i = ti * TR + r, j = tj * T + c;
      a[r][c] = (i < m && j < m) ? Ab[(int64_t)i * m + j] : 0.0;
    }
  // ||A_B||_inf: row sums over the 32 threads of a tile row, then max
  double rmax = 0.0;
#pragma unroll
  for (int r = 0; r < TR; ++r) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < T; ++c) s += fabs(a[r][c]);
    s = group_sum<32>(s);
    rmax = fmax(rmax, s);
  }
  {
    double v = rmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (tid % 64 == 0) red[tid / 64] = v;
    __syncthreads();
    v = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) v = fmax(v, red[w]);
    rmax = v;
    __syncthreads();
  }
  const double anorm = rmax;
  bool bad = false;
  for (int k = 0; k < m; ++k) {
    double* buf = rowbuf[k & 1];
    if (ti == k / TR) {
      const int r = k % TR;
#pragma unroll
      for (int rr = 0; rr < TR; ++rr)
        if (rr == r) {
#pragma unroll
          for (int c = 0; c < T; ++c) buf[tj * T + c] = a[rr][c];
        }
    }
    __syncthreads();
    const double d = buf[k];
    if (stabilize ? !(d > 0.0) : (d == 0.0 || d != d)) {
      bad = true;   // uniform: every thread read the same pivot
      break;
    }
    const double rinv = 1.0 / d;
    // rank-one update with u = column k / pivot, then row k and column k
    // of the swept matrix overwrite their entries
    double u[TR], bj[T];
#pragma unroll
    for (int r = 0; r < TR; ++r) {
      const int i = ti * TR + r;
      u[r] = buf[i < m ? i : 0] * rinv;
    }
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int j = tj * T + c;
      bj[c] = buf[j < m ? j : 0];
    }
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
      for (int c = 0; c < T; ++c) a[r][c] = fma(-u[r], bj[c], a[r][c]);
    if (ti == k / TR) {
      const int rk = k % TR;
#pragma unroll
      for (int r = 0; r < TR; ++r)
        if (r == rk) {
#pragma unroll
          for (int c = 0; c < T; ++c) a[r][c] = bj[c] * rinv;
        }
    }
    if (tj == k / T) {
      const int ck = k % T;
#pragma unroll
      for (int c = 0; c < T; ++c)
        if (c == ck) {
#pragma unroll
          for (int r = 0; r < TR; ++r) a[r][c] = (ti * TR + r == k) ? -rinv : u[r];
        }
    }
  }
  if (bad) {
    if (tid == 0) need_eig[blk] = 1;
    return;
  }
  double tr = 0.0;
#pragma unroll
  for (int r = 0; r < TR; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int i = ti * TR + r, j = tj * T + c;
      if (i == j && i < m) tr -= a[r][c];
    }
  tr = block_sum(tr, red);
  const bool ok = !stabilize || (tr > 0.0 && tr * anorm * eps * 4.0 < 1.0);
  if (!ok) {
    if (tid == 0) need_eig[blk] = 1;
    return;
  }
#pragma unroll
  for (int r = 0; r < TR; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int i = ti * TR + r, j = tj * T + c;
      if (i < m && j < m) Ab[(int64_t)i * m + j] = -a[r][c];
    }
  if (tid == 0) need_eig[blk] = 0;
}

// The same certified sweep for small blocks (m <= KM <= 64), one wave per
// block, four blocks per workgroup: lane j holds column j of the block in
// registers, and the pivot row (by symmetry the pivot column) is read
// across lanes with readlane, so no LDS and no barrier is needed.  Blocks
// that fail a pivot or the certificate are flagged in need_eig and left
// unchanged (they still hold A_B) for the eigen-decomposition.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int KM>
__global__ __launch_bounds__(256) void k_sweep_small(double* __restrict__ P, int m,
                                                     int64_t n_blocks, double eps,
                                                     int32_t* __restrict__ need_eig) {
  const int64_t blk = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (blk >= n_blocks) return;   // the whole wave
  const int j = threadIdx.x % 64;
  double* Ab = P + blk * (int64_t)m * m;
  double a[KM];
#pragma unroll
  for (int i = 0; i < KM; ++i) a[i] = (i < m && j < m) ? Ab[(int64_t)i * m + j] : 0.0;
  // ||A_B||_inf: the column sums equal the row sums of the symmetric block
  double cs = 0.0;
#pragma unroll
  for (int i = 0; i < KM; ++i) cs += fabs(a[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cs = fmax(cs, __shfl_xor(cs, o, 64));
  const double anorm = cs;
  // fully unrolled (guards instead of breaks), so a[] stays in registers
  bool bad = false;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    if (k < m && !bad) {
      const double d = readlane_f64(a[k], k);
      bad = !(d > 0.0);   // uniform: every lane read the same pivot
      if (!bad) {
        const double rinv = 1.0 / d;
        const double bj = a[k];   // row k, column j
#pragma unroll
        for (int i = 0; i < KM; ++i) {
          if (i != k && i < m) {
            const double bi = readlane_f64(a[k], i);   // row k, column i = column k, row i
            a[i] = (j == k) ? bi * rinv : a[i] - (bi * bj) * rinv;
          }
        }
        a[k] = (j == k) ? -rinv : bj * rinv;
      }
    }
  }
  if (!bad) {
    // trace of A_B^-1 = minus the trace of the swept block
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i == j && i < m) tr = -a[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
    bad = !(tr > 0.0 && tr * anorm * eps * 4.0 < 1.0);
  }
  if (bad) {
    if (j == 0) need_eig[blk] = 1;
    return;
  }
  if (j < m) {
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (i < m) Ab[(int64_t)i * m + j] = -a[i];
  }
  if (j == 0) need_eig[blk] = 0;
}

// ------------------------------------------- factored low-precision copy
// P_B = L L^T (lower Cholesky factor of the FP64 local inverse; a pivot at
// or below 1e-14 * max diag(P_B) zeroes its column, which is exact for the
// null modes of a pseudo-inverse).  The stored factor is the diagonally
// scaled Lt = D^{1/2} L (D = diag(A) on the block, isd = D^{-1/2}), so
// Lt Lt^T = D^{1/2} P_B D^{1/2}, packed by subdiagonals:
//     diagonal d (i - j = d) at offset d*m - d*(d-1)/2, entry j.
// However it is rounded, Lt Lt^T stays positive semi-definite, which is
// what keeps CG with an FP32/BF16 preconditioner meaningful.
// Thread (ti, tj) of a GRID x GRID grid holds the T x T tile at rows
// ti*T.., columns tj*T..; the pivot row is broadcast through LDS.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// kCheck: factor fl32(D^{1/2} P_B D^{1/2}) instead (the FP32 rounding of
// the diagonally scaled inverse) and only report, in unsafe[blk], whether a
// pivot fell to 1e-10 of the largest diagonal entry: where it does not, the
// rounded matrix is positive definite with margin and may stand in for P_B.
template <int GRID, int T, bool kCheck>
__global__ __launch_bounds__(GRID * GRID) void k_chol_pack(
    const double* __restrict__ P, int m, const double* __restrict__ isd,
    const int32_t* __restrict__ elem_nodes, const int32_t* __restrict__ block_elem, int nn,
    int bd, uint16_t* __restrict__ Lbf, int32_t* __restrict__ unsafe) {
  __shared__ double rowbuf[2][GRID * T];
  __shared__ double red[16];
  __shared__ double sc[GRID * T];
  const int64_t blk = blockIdx.x;
  const double* Pb = P + blk * (int64_t)m * m;
  const int tid = threadIdx.x, ti = tid / GRID, tj = tid % GRID;
  const int64_t e = block_elem[blk];
  for (int i = tid; i < m; i += GRID * GRID) {
    const int64_t dof = (int64_t)elem_nodes[e * nn + i / bd] * bd + (i % bd);
    sc[i] = 1.0 / isd[dof];   // sqrt(A_ii)
  }
  __syncthreads();   // the check scales every tile entry by sc[i] sc[j]
  double a[T][T];
  double dmax = 0.0;
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int i = ti * T + r, j = tj * T + c;
      a[r][c] = (i < m && j < m) ? Pb[(int64_t)i * m + j] : 0.0;
      if (kCheck && i < m && j < m) a[r][c] = (double)(float)(a[r][c] * sc[i] * sc[j]);
      if (i == j && i < m) dmax = fmax(dmax, a[r][c]);
    }
  {
    double v = dmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (tid % 64 == 0) red[tid / 64] = v;
    __syncthreads();
    v = 0.0;
    for (int w = 0; w < (GRID * GRID + 63) / 64; ++w) v = fmax(v, red[w]);
    dmax = v;
  }
  const double tiny = (kCheck ? 1e-10 : 1e-14) * dmax;
  bool bad = false;
  for (int k = 0; k < m; ++k) {
    double* buf = rowbuf[k & 1];
    if (ti == k / T) {
      const int r = k % T;
#pragma unroll
      for (int rr = 0; rr < T; ++rr)
        if (rr == r) {
#pragma unroll
          for (int c = 0; c < T; ++c) buf[tj * T + c] = a[rr][c];
        }
    }
    __syncthreads();
    const double d = buf[k];
    const bool live = d > tiny;
    bad = bad || !live;
    const double lkk = live ? sqrt(d) : 0.0;
    const double rl = live ? 1.0 / lkk : 0.0;
    // L[i][k] below the pivot (zero elsewhere, so the rank-one update below
    // leaves every entry outside the trailing block as it is), then column
    // k of L.  Entries above the diagonal are never stored or read again.
    double li[T], lj[T];
#pragma unroll
    for (int r = 0; r < T; ++r) {
      const int i = ti * T + r;
      li[r] = (i > k && i < m) ? buf[i] * rl : 0.0;
    }
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int j = tj * T + c;
      lj[c] = (j > k && j < m) ? buf[j] * rl : 0.0;
    }
#pragma unroll
    for (int r = 0; r < T; ++r)
#pragma unroll
      for (int c = 0; c < T; ++c) a[r][c] = fma(-li[r], lj[c], a[r][c]);
    if (tj == k / T) {
      const int ck = k % T;
#pragma unroll
      for (int c = 0; c < T; ++c)
        if (c == ck) {
#pragma unroll
          for (int r = 0; r < T; ++r) a[r][c] = (ti * T + r == k) ? lkk : li[r];
        }
    }
  }
  __syncthreads();
  if constexpr (kCheck) {
    if (tid == 0) unsafe[blk] = bad ? 1 : 0;
    return;
  }
  // write the scaled lower triangle by subdiagonals
  const int64_t per = (int64_t)m * (m + 1) / 2;
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int i = ti * T + r, j = tj * T + c;
      if (i >= m || j > i) continue;
      const int dg = i - j;
      const int64_t pos = blk * per + (int64_t)dg * m - (int64_t)dg * (dg - 1) / 2 + j;
      const double v = a[r][c] * sc[i];
      Lbf[pos] = f32_to_bf16((float)v);
    }
}

hipError_t launch_chol_pack(fc_precond_s& pc, hipStream_t s, int32_t* unsafe) {
  const int m = pc.m;
  const int64_t nb = pc.n_blocks;
  if (nb == 0) return hipSuccess;
  dim3 g((unsigned)nb);
  const fc_problem_s& pb = *pc.pb;
#define FC_CHOL(GR, TT)                                                                     \
  if (unsafe)                                                                               \
    hipLaunchKernelGGL((k_chol_pack<GR, TT, true>), g, dim3(GR * GR), 0, s, pc.P, m, pc.isd, \
                       block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, nullptr, unsafe);       \
  else                                                                                      \
    hipLaunchKernelGGL((k_chol_pack<GR, TT, false>), g, dim3(GR * GR), 0, s, pc.P, m,        \
                       pc.isd, block_nodes(pc), pc.block_elem, pc.nn, pc.bdim, pc.Lbf, nullptr)
  if (m <= 8) FC_CHOL(8, 1);
  else if (m <= 16) FC_CHOL(8, 2);
  else if (m <= 32) FC_CHOL(8, 4);
  else if (m <= 64) FC_CHOL(8, 8);
  else if (m <= 96) FC_CHOL(32, 3);
  else if (m <= 128) FC_CHOL(32, 4);
  else if (m <= 160) FC_CHOL(32, 5);
  else FC_CHOL(32, 6);
#undef FC_CHOL
  return hipGetLastError();
}

// ---------------------------------------------------- diagonal / fallback
__global__ void k_diag(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                       const double* __restrict__ val, int bd, int64_t n_rows,
                       double* __restrict__ diag) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_rows) return;
  const int32_t lo = rowptr[row], hi = rowptr[row + 1];
  int32_t l = lo, h = hi - 1, found = -1;
  while (l <= h) {
    int32_t mid = (l + h) >> 1;
    int32_t c = col[mid];
    if (c == row) {
      found = mid;
      break;
    }
    if (c < row) l = mid + 1;
    else h = mid - 1;
  }
  const int64_t L = hi - lo;
  for (int c = 0; c < bd; ++c)
    diag[row * bd + c] =
        found >= 0 ? val[(int64_t)lo * bd * bd + (int64_t)(c * bd + c) * L + (found - lo)] : 0.0;
}

// Algorithm 1 diagonal scaling: S_ll == 0 -> 1/A_ll (only where A_ll > 0).
__global__ void k_fallback(const double* __restrict__ P, const int32_t* __restrict__ inv_ptr,
                           const int32_t* __restrict__ inv_idx, const double* __restrict__ diag,
                           int m, int bd, int64_t n_dofs, double* __restrict__ fb,
                           unsigned long long* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_dofs) return;
  const int64_t node = i / bd;
  const int c = (int)(i % bd);
  double s = 0.0;
  for (int32_t e = inv_ptr[node]; e < inv_ptr[node + 1]; ++e) {
    const int64_t idx = inv_idx[e];
    const int64_t blk = idx / m;
    const int slot = (int)(idx - blk * m) + c;
    s += P[blk * (int64_t)m * m + (int64_t)slot * m + slot];
  }
  const double a = diag[i];
  const bool fall = (s == 0.0) && (a > 0.0);
  fb[i] = fall ? 1.0 / a : 0.0;
  if (fall) atomicAdd(count, 1ull);
}

__global__ void k_cast_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// ---------------------------------------------------------- launchers
hipError_t launch_block_extract(const fc_problem_s& pb, const fc_precond_s& pc,
                                hipStream_t s) {
  if (pc.n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_extract, dim3((unsigned)pc.n_blocks), dim3(256), 0, s,
                     pb.A.rowptr, pb.A.col, pb.A.val, block_nodes(pc), pc.block_elem,
                     pc.nn, pc.bdim, pc.m, pc.P);
  return hipGetLastError();
}

hipError_t launch_jacobi(fc_precond_s& pc, const int32_t* sel, int64_t count,
                         double* work, int32_t* dropped, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int m = pc.m;
  // one wave per block for small blocks, four waves otherwise
  const int threads = m <= 32 ? 64 : 256;
  const size_t lds = sizeof(double) * 2 * (size_t)m * (m + 1);
  int dev = 0, limit = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    limit = 65536;
  const size_t static_lds = 6 * 1024;   // rotation tables and reductions
  if (m <= 64 && lds + static_lds <= (size_t)limit) {
    (void)hipFuncSetAttribute((const void*)k_jacobi_pinv<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_jacobi_pinv<true>, dim3((unsigned)count), dim3(threads), lds, s,
                       pc.P, m, sel, nullptr, pc.eps, pc.stabilize, dropped);
  } else {
    if (!work) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi_pinv<false>, dim3((unsigned)count), dim3(threads), 0, s,
                       pc.P, m, sel, work, pc.eps, pc.stabilize, dropped);
  }
  return hipGetLastError();
}

bool jacobi_needs_work(int m) {
  const size_t lds = sizeof(double) * 2 * (size_t)m * (m + 1);
  int dev = 0, limit = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    limit = 65536;
  return !(m <= 64 && lds + 6 * 1024 <= (size_t)limit);
}

hipError_t launch_sweep(fc_precond_s& pc, int32_t* need_eig, hipStream_t s) {
  const int m = pc.m;
  dim3 g((unsigned)pc.n_blocks), b(512);
  if (m <= 96)
    hipLaunchKernelGGL(k_sweep_inverse<3>, g, b, 0, s, pc.P, m, pc.eps, pc.stabilize, need_eig);
  else if (m <= 128)
    hipLaunchKernelGGL(k_sweep_inverse<4>, g, b, 0, s, pc.P, m, pc.eps, pc.stabilize, need_eig);
  else if (m <= 160)
    hipLaunchKernelGGL(k_sweep_inverse<5>, g, b, 0, s, pc.P, m, pc.eps, pc.stabilize, need_eig);
  else
    hipLaunchKernelGGL(k_sweep_inverse<6>, g, b, 0, s, pc.P, m, pc.eps, pc.stabilize, need_eig);
  return hipGetLastError();
}

hipError_t launch_sweep_small(fc_precond_s& pc, int32_t* need_eig, hipStream_t s) {
  const int m = pc.m;
  const dim3 g((unsigned)((pc.n_blocks + 3) / 4)), b(256);
  if (m <= 16)
    hipLaunchKernelGGL(k_sweep_small<16>, g, b, 0, s, pc.P, m, pc.n_blocks, pc.eps, need_eig);
  else if (m <= 32)
    hipLaunchKernelGGL(k_sweep_small<32>, g, b, 0, s, pc.P, m, pc.n_blocks, pc.eps, need_eig);
  else if (m <= 64)
    hipLaunchKernelGGL(k_sweep_small<64>, g, b, 0, s, pc.P, m, pc.n_blocks, pc.eps, need_eig);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_diag(const fc_problem_s& pb, hipStream_t s) {
  const int64_t n = pb.A.n_rows;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     pb.A.rowptr, pb.A.col, pb.A.val, pb.bdim, n, pb.diag);
  return hipGetLastError();
}

hipError_t launch_fallback(const fc_problem_s& pb, fc_precond_s& pc,
                           unsigned long long* d_count, hipStream_t s) {
  const int64_t n = pb.n_dofs;
  hipLaunchKernelGGL(k_fallback, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     pc.P, pc.inv_ptr, pc.inv_idx, pb.diag, pc.m, pc.bdim, n,
                     pc.fallback, d_count);
  return hipGetLastError();
}

// FP32 copy of the matrix values, same layout (k_cast_f32 above)
hipError_t launch_cast_matrix(const DeviceBsr& A, hipStream_t s) {
  const int64_t n = A.nnzb * A.bdim * A.bdim;
  if (!A.val32 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f32, dim3(4096), dim3(256), 0, s, A.val, A.val32, n);
  return hipGetLastError();
}

}  // namespace fc
