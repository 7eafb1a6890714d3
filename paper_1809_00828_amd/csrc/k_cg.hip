// Preconditioned conjugate gradients on the device (Sec. 5, with the
// Schwarz preconditioner of Eq. 6 and the stopping test of Eq. 12).
//
// Recurrences (x_0 = 0):  r_0 = b, z_0 = S r_0, p_0 = z_0, then per step
//   q = A p;  alpha = (r,z)/(p,q);  x += alpha p;  r -= alpha q;
//   z = S r;  beta = (r,z)_new/(r,z);  p = z + beta p.
// One step is seven kernels, all reading their scalars from device memory:
//   1. SpMV q = A p (k_spmv.hip)
//   2. (p, q) by workgroup partials in a separate pass over p and q, then
//      one workgroup sums them in a fixed order: alpha, step count.
//      Fusing the dot into the SpMV costs more than this extra pass: the
//      SpMV's end-of-workgroup reduction holds its four waves until the
//      slowest one finishes.
//   3. Schwarz phase 1 on the gathered r - alpha q (k_schwarz.hip)
//   4. pull z = sum_B R_B^T y_B + fallback, fused with the x and r updates
//      and per-workgroup (r,z), (z,z), (r,r) partials
//   5. one workgroup: stop test and beta
//   6. p = z + beta p
// The reductions stay atomic-free: a same-address atomic per workgroup
// serialises in L2 and costs more than the SpMV itself at this size.
// Every kernel returns at once when the stop flag is set, so a captured
// chunk of steps can be replayed without the host and the iterate stays the
// one at which the test fired.  The host checks the flag between chunks.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdlib>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "dev_common.h"
#include "k_schwarz.h"
#include "learned.h"
#include "k_setup.h"
#include "k_spmv.h"

#define FC_TRY_ST(x)               \
  do {                             \
    fc_status s_ = (x);            \
    if (s_ != FC_OK) return s_;    \
  } while (0)

namespace fc {

struct SolverWs {
  int64_t n = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *t = nullptr;
  double *d = nullptr, *ro = nullptr;   // refinement correction and outer residual
  float* p32 = nullptr;                  // fl32(p) for the mixed product
  double* partial = nullptr;
  int64_t partial_len = 0;
  CgScalars* sc = nullptr;
  CgScalars* host = nullptr;    // pinned mirror
  hipStream_t stream = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
  int key_chunk = 0, key_prec = -1;
  const void* key_b = nullptr;
  std::vector<hipEvent_t> tev;  // timing mode: 4 events per step of a chunk
  // learned mode with m > 1 kept directions (flexible CG, FCG(m))
  double* ring = nullptr;         // [2][ring_cap][n]: p_j, then A p_j
  double* ring_part = nullptr;    // [ring_cap][ring_blocks] dot partials
  struct FcgRing* fr = nullptr;
  int ring_cap = 0;
};

void solver_ws_destroy(SolverWs* w) {
  if (!w) return;
  if (w->exec) (void)hipGraphExecDestroy(w->exec);
  if (w->graph) (void)hipGraphDestroy(w->graph);
  for (auto* p : {w->r, w->z, w->p, w->q, w->t, w->d, w->ro, w->partial, w->ring, w->ring_part})
    if (p) (void)hipFree(p);
  if (w->p32) (void)hipFree(w->p32);
  if (w->fr) (void)hipFree(w->fr);
  if (w->sc) (void)hipFree(w->sc);
  if (w->host) (void)hipHostFree(w->host);
  for (auto& e : w->ev) if (e) (void)hipEventDestroy(e);
  for (auto& e : w->tev) if (e) (void)hipEventDestroy(e);
  if (w->stream) (void)hipStreamDestroy(w->stream);
  delete w;
}

// -------------------------------------------------------------- kernels
constexpr int kVecThreads = 256;

// Three dots of the starting vectors: (r,z), (z,z), (r,r); the last
// workgroup initialises the scalars.
__global__ __launch_bounds__(256) void k_cg_start(const double* __restrict__ r,
                                                  const double* __restrict__ z, int64_t n,
                                                  double* __restrict__ partial, CgScalars* sc) {
  __shared__ double lds[16];
  __shared__ int flag;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    a = fma(r[i], z[i], a);
    b = fma(z[i], z[i], b);
    c = fma(r[i], r[i], c);
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  c = block_sum(c, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[gridDim.x + blockIdx.x] = b;
    partial[2 * gridDim.x + blockIdx.x] = c;
  }
  if (!last_block(&sc->ticket, gridDim.x, &flag)) return;
  const double rz = sum_partials(partial, gridDim.x, lds);
  const double zz = sum_partials(partial + gridDim.x, gridDim.x, lds);
  const double rr = sum_partials(partial + 2 * gridDim.x, gridDim.x, lds);
  if (threadIdx.x == 0) {
    sc->rz = rz;
    sc->zz = zz;
    sc->rr = rr;
    sc->iter = 0;
    sc->zn0 = sqrt(zz);
    sc->rn0 = sqrt(rr);
    const double c0 = sc->stop == FC_STOP_PRECOND ? sc->zn0 : sc->rn0;
    sc->crit0 = c0;
    sc->crit = c0 > 0.0 ? 1.0 : 0.0;
    if (sc->history) sc->history[0] = sc->crit;
    if (!(c0 == c0) || !(rz == rz)) sc->done = 4;
    else if (c0 == 0.0) sc->done = 1;
    else sc->done = 0;
  }
}

// Step length: sum the per-workgroup (p, A p) partials of the SpMV in a
// fixed order (one workgroup), count the step and check for breakdown.
__global__ __launch_bounds__(1024) void k_cg_alpha(const double* __restrict__ partial, int np,
                                                   CgScalars* sc) {
  __shared__ double lds[16];
  if (sc->done) return;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * (int)blockDim.x < np; i += 4 * blockDim.x) {
    t0 += partial[i];
    t1 += partial[i + blockDim.x];
    t2 += partial[i + 2 * blockDim.x];
    t3 += partial[i + 3 * blockDim.x];
  }
  for (; i < np; i += blockDim.x) t0 += partial[i];
  const double pq = block_sum((t0 + t1) + (t2 + t3), lds);
  if (threadIdx.x == 0) {
    sc->pq = pq;
    sc->iter += 1;
    const double rz = sc->rz;
    if (!(pq > 0.0) || !(rz > 0.0)) {
      sc->done = (pq != pq || rz != rz) ? 4 : 3;
    } else {
      sc->alpha = rz / pq;
    }
  }
}

// (p, q) partials of a separate pass over p and q, one per workgroup; the
// one-workgroup k_cg_alpha sums them in a fixed order.  (A last-workgroup
// ticket here would serialise thousands of same-address atomics in L2.)
__global__ __launch_bounds__(256) void k_cg_pq(const double* __restrict__ p,
                                               const double* __restrict__ q, int64_t n,
                                               double* __restrict__ partial,
                                               const CgScalars* __restrict__ sc) {
  __shared__ double lds[16];
  if (sc->done) return;
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a = fma(p[i], q[i], a);
  a = block_sum(a, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = a;
}

// Pull of the Schwarz apply fused with x += alpha p, r -= alpha q and the
// reductions of the new r and z (one partial triple per workgroup; the
// grid loops over the unknowns).  kFlex adds a fourth partial, (z, q),
// for the flexible beta.
template <bool kFlex>
__global__ __launch_bounds__(256) void k_cg_pull(
    const double* __restrict__ y, const int32_t* __restrict__ inv_ptr,
    const int32_t* __restrict__ inv_idx, const double* __restrict__ fb, int bd, int64_t n,
    double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ z, double* __restrict__ partial,
    const CgScalars* __restrict__ sc) {
  __shared__ double lds[16];
  if (sc->done) return;
  const double alpha = sc->alpha;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = i / bd;
    const int cc = (int)(i - node * bd);
    double s = 0.0;
    for (int32_t e = inv_ptr[node]; e < inv_ptr[node + 1]; ++e) s += y[(int64_t)inv_idx[e] + cc];
    const double qi = q[i];
    const double ri = fma(-alpha, qi, r[i]);
    x[i] = fma(alpha, p[i], x[i]);
    r[i] = ri;
    const double zi = fma(fb[i], ri, s);
    z[i] = zi;
    a = fma(ri, zi, a);
    b = fma(zi, zi, b);
    c = fma(ri, ri, c);
    if (kFlex) d = fma(zi, qi, d);
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  c = block_sum(c, lds);
  if (kFlex) d = block_sum(d, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[gridDim.x + blockIdx.x] = b;
    partial[2 * gridDim.x + blockIdx.x] = c;
    if (kFlex) partial[3 * gridDim.x + blockIdx.x] = d;
  }
}

// The same pull where every cell is a block (scalar problems): the
// workgroups walk node tiles of the lattice and find each node's blocks
// from its lattice indices (no node-to-block map is read), summing them in
// the same ascending order, so z is bitwise the mapped pull's.  fb may be
// null (no unknown needs the diagonal scaling).  The partial sums of a
// workgroup are reduced together, with one barrier.
template <bool kFlex>
__global__ __launch_bounds__(256) void k_cg_pull_lat(
    const double* __restrict__ y, const PullLattice L, int m, const double* __restrict__ fb,
    double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ z, double* __restrict__ partial,
    const CgScalars* __restrict__ sc) {
  constexpr int kN = kFlex ? 4 : 3;
  __shared__ double lds[4][kN];
  if (sc->done) return;
  const double alpha = sc->alpha;
  const int64_t ntiles = pull_num_tiles(L);
  double v[kN] = {};
  // XCD-contiguous tile ranges: the block outputs of the cells on a tile's
  // faces, which the neighbouring tiles read too, stay in one XCD's L2
  const XcdRange xr = xcd_range(blockIdx.x, gridDim.x, ntiles);
  for (int64_t tile = xr.t0 + xr.j; tile < xr.t1; tile += xr.per) {
    int gx, gy, gz;
    if (!pull_node(L, tile, threadIdx.x, &gx, &gy, &gz)) continue;
    const double sv = pull_lattice_sum(y, L, m, gx, gy, gz);
    const int64_t i = gx + (int64_t)L.n1 * (gy + (int64_t)L.n1 * gz);
    const double qi = q[i];
    const double ri = fma(-alpha, qi, r[i]);
    x[i] = fma(alpha, p[i], x[i]);
    r[i] = ri;
    const double zi = fb ? fma(fb[i], ri, sv) : sv;
    z[i] = zi;
    v[0] = fma(ri, zi, v[0]);
    v[1] = fma(zi, zi, v[1]);
    v[2] = fma(ri, ri, v[2]);
    if constexpr (kFlex) v[3] = fma(zi, qi, v[3]);
  }
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    v[k] = group_sum<kWave>(v[k]);
    if (threadIdx.x % kWave == 0) lds[w][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < kN) {
    const int k = threadIdx.x;
    partial[k * gridDim.x + blockIdx.x] = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
  }
}

// Stop test (Eq. 12 or the plain residual) and beta from the pull's
// partials, summed in a fixed order by one workgroup.
__global__ __launch_bounds__(1024) void k_cg_beta(const double* __restrict__ partial, int np,
                                                  CgScalars* sc) {
  __shared__ double lds[16];
  if (sc->done) return;
  double ta = 0.0, tb = 0.0, tc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    ta += partial[i];
    tb += partial[np + i];
    tc += partial[2 * np + i];
  }
  const double rz = block_sum(ta, lds);
  const double zz = block_sum(tb, lds);
  const double rr = block_sum(tc, lds);
  if (threadIdx.x == 0) {
    const double crit = (sc->stop == FC_STOP_PRECOND ? sqrt(zz) : sqrt(rr)) / sc->crit0;
    sc->zz = zz;
    sc->rr = rr;
    sc->crit = crit;
    if (sc->history) sc->history[sc->iter] = crit;
    if (!(crit == crit) || !(rz == rz) || isinf(rz)) {
      sc->done = 4;
    } else if (crit <= sc->tol) {
      sc->done = 1;
    } else if (sc->iter >= sc->maxit) {
      sc->done = 2;
    }
    sc->beta = rz / sc->rz;
    sc->rz = rz;
  }
}

// Flexible variant (FCG(1)) for the learned correction z = S r + gamma w:
// (r, z) and (z, q) are the pull's Schwarz parts plus the correction's
// gamma (y . P_c^T r) and gamma (w . q); beta = -(z, q) / (p, q) keeps p
// A-orthogonal to the previous direction.  (z, z) keeps the Schwarz part.
__global__ __launch_bounds__(1024) void k_cg_beta_flex(const double* __restrict__ partial, int np,
                                                       CgScalars* sc,
                                                       const LearnScalars* __restrict__ ls) {
  __shared__ double lds[16];
  if (sc->done) return;
  double ta = 0.0, tb = 0.0, tc = 0.0, td = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    ta += partial[i];
    tb += partial[np + i];
    tc += partial[2 * np + i];
    td += partial[3 * np + i];
  }
  double rz = block_sum(ta, lds);
  const double zz = block_sum(tb, lds);
  const double rr = block_sum(tc, lds);
  double zq = block_sum(td, lds);
  if (threadIdx.x == 0) {
    const double g = ls->gamma;
    if (g != 0.0) {
      rz += g * ls->yrc;
      zq += g * ls->wq;
    }
    const double crit = sqrt(rr) / sc->crit0;
    sc->zz = zz;
    sc->rr = rr;
    sc->crit = crit;
    if (sc->history) sc->history[sc->iter] = crit;
    if (!(crit == crit) || !(rz == rz) || isinf(rz) || !(zq == zq)) {
      sc->done = 4;
    } else if (crit <= sc->tol) {
      sc->done = 1;
    } else if (sc->iter >= sc->maxit) {
      sc->done = 2;
    }
    sc->beta = -zq / sc->pq;
    sc->rz = rz;
  }
}

__global__ __launch_bounds__(256) void k_cg_p(const double* __restrict__ z, double* __restrict__ p,
                                              int64_t n, const CgScalars* sc) {
  if (sc->done) return;
  const double beta = sc->beta;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = fma(beta, p[i], z[i]);
}

// ---- flexible CG keeping m > 1 directions (learned mode)
// The direction of every step (p, A p, (p, A p)) goes to slot count mod m
// of a ring; the next direction is z made A-orthogonal to every kept one,
// p = z - sum_j (z, A p_j) / (p_j, A p_j) p_j (slots in index order).
constexpr int kMaxFcg = 64;
constexpr int kRingElems = 8;   // unknowns per thread of the dot pass
struct FcgRing {
  int64_t count;                // directions taken so far
  double pq[kMaxFcg];           // (p_j, A p_j) per slot
  double beta[kMaxFcg];         // -(z, A p_j) / (p_j, A p_j) per slot
};

inline unsigned ring_blocks(int64_t n) {
  return (unsigned)((n + 256 * kRingElems - 1) / (256 * kRingElems));
}

__global__ void k_fcg_reset(FcgRing* fr) { fr->count = 0; }

// Store the step's p and q = A p in slot count mod m and form, per
// workgroup (one contiguous chunk of unknowns), the partial (z, A p_j) of
// every kept slot j: wave sums by shuffles, one barrier for all slots.
__global__ __launch_bounds__(256) void k_fcg_keep_dots(
    const double* __restrict__ p, const double* __restrict__ q, const double* __restrict__ z,
    int64_t n, int m, double* __restrict__ ring, double* __restrict__ part, FcgRing* fr,
    const CgScalars* __restrict__ sc) {
  __shared__ double red[kMaxFcg][4];
  if (sc->done) return;
  const int64_t cnt0 = fr->count;
  const int slot = (int)(cnt0 % m);
  const int cnt = (int)(cnt0 + 1 < m ? cnt0 + 1 : m);
  double* P = ring + (int64_t)slot * n;
  const double* Q = ring + (int64_t)m * n;
  double* Qs = ring + ((int64_t)m + slot) * n;
  const int64_t base = (int64_t)blockIdx.x * (256 * kRingElems) + threadIdx.x;
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  double zv[kRingElems], qv[kRingElems];
#pragma unroll
  for (int e = 0; e < kRingElems; ++e) {
    const int64_t i = base + (int64_t)e * 256;
    zv[e] = 0.0;
    qv[e] = 0.0;
    if (i < n) {
      zv[e] = z[i];
      qv[e] = q[i];
      P[i] = p[i];
      Qs[i] = qv[e];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) fr->pq[slot] = sc->pq;
  for (int j = 0; j < cnt; ++j) {
    const double* Qj = Q + (int64_t)j * n;
    double d = 0.0;
#pragma unroll
    for (int e = 0; e < kRingElems; ++e) {
      const int64_t i = base + (int64_t)e * 256;
      if (i < n) d = fma(zv[e], j == slot ? qv[e] : Qj[i], d);
    }
    d = group_sum<kWave>(d);
    if (l == 0) red[j][w] = d;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += blockDim.x)
    part[(int64_t)j * gridDim.x + blockIdx.x] = (red[j][0] + red[j][1]) + (red[j][2] + red[j][3]);
}

// Stop test as in k_cg_beta_flex (residual stop; (r, z) gains the
// correction's gamma (y . P_c^T r)), then beta_j for every kept slot: one
// wave per slot (16 waves take the slots in turn), each summing that
// slot's partials in a fixed order.
__global__ __launch_bounds__(1024) void k_fcg_beta(const double* __restrict__ partial, int np,
                                                   const double* __restrict__ part, int nb,
                                                   int m, FcgRing* fr, CgScalars* sc,
                                                   const LearnScalars* __restrict__ ls) {
  __shared__ double lds[16];
  __shared__ int bad;
  if (sc->done) return;
  if (threadIdx.x == 0) bad = 0;
  double ta = 0.0, tb = 0.0, tc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    ta += partial[i];
    tb += partial[np + i];
    tc += partial[2 * np + i];
  }
  double rz = block_sum(ta, lds);
  const double zz = block_sum(tb, lds);
  const double rr = block_sum(tc, lds);
  const int64_t cnt0 = fr->count;
  const int cnt = (int)(cnt0 + 1 < m ? cnt0 + 1 : m);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  for (int j = w; j < cnt; j += nw) {
    const double* pj = part + (int64_t)j * nb;
    double t0 = 0.0, t1 = 0.0;
    int i = l;
    for (; i + kWave < nb; i += 2 * kWave) {
      t0 += pj[i];
      t1 += pj[i + kWave];
    }
    if (i < nb) t0 += pj[i];
    const double d = group_sum<kWave>(t0 + t1);
    if (l == 0) {
      const double b = -d / fr->pq[j];
      fr->beta[j] = b;
      if (!(b == b) || isinf(b)) bad = 1;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    fr->count = cnt0 + 1;
    const double g = ls->gamma;
    if (g != 0.0) rz += g * ls->yrc;
    const double crit = sqrt(rr) / sc->crit0;
    sc->zz = zz;
    sc->rr = rr;
    sc->crit = crit;
    if (sc->history) sc->history[sc->iter] = crit;
    if (!(crit == crit) || !(rz == rz) || isinf(rz) || bad) {
      sc->done = 4;
    } else if (crit <= sc->tol) {
      sc->done = 1;
    } else if (sc->iter >= sc->maxit) {
      sc->done = 2;
    }
    sc->rz = rz;
  }
}

// p = z + sum_j beta_j p_j over the kept slots
__global__ __launch_bounds__(256) void k_fcg_dir(const double* __restrict__ z,
                                                 double* __restrict__ p,
                                                 const double* __restrict__ ring, int64_t n,
                                                 int m, const FcgRing* __restrict__ fr,
                                                 const CgScalars* __restrict__ sc) {
  __shared__ double beta[kMaxFcg];
  if (sc->done) return;
  const int cnt = (int)(fr->count < m ? fr->count : m);
  for (int j = threadIdx.x; j < cnt; j += blockDim.x) beta[j] = fr->beta[j];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = z[i];
    for (int j = 0; j < cnt; ++j) v = fma(beta[j], ring[(int64_t)j * n + i], v);
    p[i] = v;
  }
}

// b = fl32(a) (skipped once the stop flag is set)
__global__ void k_round_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n,
                            const CgScalars* __restrict__ sc) {
  if (sc && sc->done) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_axpy(double alpha, const double* __restrict__ a, double* __restrict__ b,
                       int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = fma(alpha, a[i], b[i]);
}

// c = a - b
__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    c[i] = a[i] - b[i];
}

__global__ void k_fill(double* __restrict__ a, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// ||b - t||^2 and ||b||^2 into sc->rr and sc->zz (final true residual).
__global__ __launch_bounds__(256) void k_resid(const double* __restrict__ b,
                                               const double* __restrict__ t, int64_t n,
                                               double* __restrict__ partial, CgScalars* sc,
                                               double* out /* [2] */) {
  __shared__ double lds[16];
  __shared__ int flag;
  double a = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = b[i] - t[i];
    a = fma(d, d, a);
    c = fma(b[i], b[i], c);
  }
  a = block_sum(a, lds);
  c = block_sum(c, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[gridDim.x + blockIdx.x] = c;
  }
  if (!last_block(&sc->ticket, gridDim.x, &flag)) return;
  const double ra = sum_partials(partial, gridDim.x, lds);
  const double rc = sum_partials(partial + gridDim.x, gridDim.x, lds);
  if (threadIdx.x == 0) {
    out[0] = ra;
    out[1] = rc;
  }
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kVecThreads - 1) / kVecThreads); }
static constexpr unsigned kRedBlocks = 1024;
// grid of the fused pull: enough workgroups to fill the chip, few partials
static inline unsigned pull_grid(int64_t n) { return std::min<unsigned>(nblk(n), 2048u); }
// grid of the pull actually launched for this preconditioner (the lattice
// pull walks node tiles, one workgroup per tile up to 16,384 workgroups,
// which at 64^3 cells, p = 2 is 6 % faster than 4,096; never more
// workgroups than partial slots)
static inline unsigned pull_grid_for(const fc_precond_s& pc, int64_t n, int64_t partial_len) {
  if (pc.lat.dim == 0) return pull_grid(n);
  static const int cap = [] {
    const char* e = std::getenv("FC_PULL_GRID");
    return e ? std::max(64, std::atoi(e)) : 16384;
  }();
  const int64_t nt = pull_num_tiles(pc.lat);
  // at most one partial set (four values) per workgroup fits in `partial`
  return (unsigned)std::min<int64_t>({nt, (int64_t)cap, (partial_len - 8) / 4});
}

// Schwarz pull fused with the CG updates and the (r,z), (z,z), (r,r)
// [, (z,q)] partials, one partial set per workgroup of the grid pg.
template <bool kFlex>
static hipError_t launch_cg_pull(const fc_precond_s& pc, unsigned pg, double* x, double* r,
                                 const double* p, const double* q, double* z, double* partial,
                                 const CgScalars* sc, hipStream_t s) {
  const int64_t n = pc.pb->n_dofs;
  if (pc.lat.dim == 0) {
    hipLaunchKernelGGL(k_cg_pull<kFlex>, dim3(pg), dim3(kVecThreads), 0, s, pc.y, pc.inv_ptr,
                       pc.inv_idx, pc.fallback, pc.bdim, n, x, r, p, q, z, partial, sc);
    return hipGetLastError();
  }
  // the lattice is set for scalar problems only
  if (pc.bdim != 1) return hipErrorInvalidValue;
  const double* fb = pc.n_fallback ? pc.fallback : nullptr;
  hipLaunchKernelGGL(k_cg_pull_lat<kFlex>, dim3(pg), dim3(256), 0, s, pc.y, pc.lat, pc.m, fb, x,
                     r, p, q, z, partial, sc);
  return hipGetLastError();
}

// grid of a two-vector dot: a few elements per lane keep enough loads in
// flight (1024 workgroups left ten dependent iterations per lane at 2.7M)
static inline unsigned dot_grid(int64_t n) { return std::min<unsigned>(nblk(n), 4096u); }

// ----------------------------------------------------------- host side
static fc_status ensure_ws(fc_precond_s& pc, SolverWs** out) {
  fc_problem_s& pb = *pc.pb;
  SolverWs* w = pc.ws;
  const int64_t n = pb.n_dofs;
  if (!w) {
    w = new SolverWs();
    pc.ws = w;
    w->n = n;
    FC_HIP(hipMalloc(&w->r, n * sizeof(double)));
    FC_HIP(hipMalloc(&w->z, n * sizeof(double)));
    FC_HIP(hipMalloc(&w->p, n * sizeof(double)));
    FC_HIP(hipMalloc(&w->q, n * sizeof(double)));
    FC_HIP(hipMalloc(&w->t, n * sizeof(double)));
    int64_t np = std::max<int64_t>({(int64_t)spmv_num_blocks(pb.A), (int64_t)nblk(n),
                                    (int64_t)kRedBlocks});
    w->partial_len = 4 * np + 8;
    FC_HIP(hipMalloc(&w->partial, w->partial_len * sizeof(double)));
    FC_HIP(hipMalloc(&w->sc, sizeof(CgScalars)));
    FC_HIP(hipMemset(w->sc, 0, sizeof(CgScalars)));
    FC_HIP(hipHostMalloc(&w->host, sizeof(CgScalars), hipHostMallocDefault));
    FC_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    for (auto& e : w->ev) FC_HIP(hipEventCreate(&e));
  }
  *out = w;
  return FC_OK;
}

// Ring of m kept directions for the learned mode's FCG(m); a larger ring
// replaces the old one and drops the captured chunk that used it.
static fc_status ensure_ring(SolverWs& w, int m) {
  if (m <= 1 || w.ring_cap >= m) return FC_OK;
  if (w.exec) {
    FC_HIP(hipGraphExecDestroy(w.exec));
    w.exec = nullptr;
  }
  if (w.graph) {
    FC_HIP(hipGraphDestroy(w.graph));
    w.graph = nullptr;
  }
  w.key_prec = -1;
  if (w.ring) FC_HIP(hipFree(w.ring));
  if (w.ring_part) FC_HIP(hipFree(w.ring_part));
  w.ring = nullptr;
  w.ring_part = nullptr;
  w.ring_cap = 0;
  FC_HIP(hipMalloc(&w.ring, (size_t)2 * m * w.n * sizeof(double)));
  FC_HIP(hipMalloc(&w.ring_part, (size_t)m * ring_blocks(w.n) * sizeof(double)));
  if (!w.fr) FC_HIP(hipMalloc(&w.fr, sizeof(FcgRing)));
  w.ring_cap = m;
  return FC_OK;
}

// FC_CG_SPLIT_DOT=0 fuses (p, A p) into the SpMV (one partial per SpMV
// workgroup); the default computes it in a separate pass over p and q.
static bool split_dot() {
  static const bool v = [] {
    const char* e = std::getenv("FC_CG_SPLIT_DOT");
    return !(e && e[0] == '0');
  }();
  return v;
}

// Enqueue `chunk` PCG steps on stream s (with timing events when tev).
// precA: 0 = FP64 matrix, 1 = row-mixed FP64/FP32 matrix; precS: 0/1/2 =
// FP64/FP32/BF16 local inverses.
static hipError_t enqueue_steps(fc_precond_s& pc, SolverWs& w, double* x, int chunk, int precA,
                                int precS, hipStream_t s, hipEvent_t* tev = nullptr,
                                CoarseCtx* learn = nullptr, int every = 1, int fcg_m = 1) {
  fc_problem_s& pb = *pc.pb;
  const int64_t n = pb.n_dofs;
  for (int it = 0; it < chunk; ++it) {
    hipError_t e;
    hipEvent_t* tev_it = (tev && it % every == 0) ? tev : nullptr;
    if (tev_it && (e = hipEventRecord(tev[4 * it + 0], s)) != hipSuccess) return e;
    if (precA == 1) {
      // row-mixed matrix: rows touching cut or fictitious cells in FP64,
      // the others from the FP32 copy, which gather p rounded to FP32 (half
      // the gathered bytes; those products round p to FP32 anyway)
      hipLaunchKernelGGL(k_round_f32, dim3(pull_grid(n)), dim3(kVecThreads), 0, s, w.p, w.p32,
                         n, w.sc);
      e = launch_spmv_mixed(pb.A, w.p, w.p32, w.q, w.sc, s);
      if (e != hipSuccess) return e;
      if (tev_it && (e = hipEventRecord(tev[4 * it + 1], s)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_cg_pq, dim3(dot_grid(n)), dim3(256), 0, s, w.p, w.q, n, w.partial,
                         w.sc);
      hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, s, w.partial, (int)dot_grid(n),
                         w.sc);
    } else if (split_dot()) {
      // SpMV without its fused dot, then (p, q) and alpha in one reduction
      e = launch_spmv_pq(pb.A, w.p, w.q, w.sc, nullptr, s);
      if (e != hipSuccess) return e;
      if (tev_it && (e = hipEventRecord(tev[4 * it + 1], s)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_cg_pq, dim3(dot_grid(n)), dim3(256), 0, s, w.p, w.q, n, w.partial,
                         w.sc);
      hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, s, w.partial, (int)dot_grid(n),
                         w.sc);
    } else {
      e = launch_spmv_pq(pb.A, w.p, w.q, w.sc, w.partial, s);
      if (e != hipSuccess) return e;
      if (tev_it && (e = hipEventRecord(tev[4 * it + 1], s)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, s, w.partial,
                         spmv_num_blocks(pb.A), w.sc);
    }
    if (tev_it && (e = hipEventRecord(tev[4 * it + 2], s)) != hipSuccess) return e;
    e = launch_schwarz_phase1(pc, precS, w.r, w.q, w.sc, s);
    if (e != hipSuccess) return e;
    if (tev_it && (e = hipEventRecord(tev[4 * it + 3], s)) != hipSuccess) return e;
    const unsigned pg = pull_grid_for(pc, n, w.partial_len);
    const bool ring = learn && fcg_m > 1;
    if (ring) {
      // FCG(m): Schwarz pull, correction, then the new direction made
      // A-orthogonal to the m kept ones
      if ((e = launch_cg_pull<false>(pc, pg, x, w.r, w.p, w.q, w.z, w.partial, w.sc, s)) !=
          hipSuccess)
        return e;
      if ((e = coarse_correct(*learn, w.r, w.z, nullptr, w.sc, s)) != hipSuccess) return e;
      const unsigned rb = ring_blocks(n);
      hipLaunchKernelGGL(k_fcg_keep_dots, dim3(rb), dim3(256), 0, s, w.p, w.q, w.z, n, fcg_m,
                         w.ring, w.ring_part, w.fr, w.sc);
      hipLaunchKernelGGL(k_fcg_beta, dim3(1), dim3(1024), 0, s, w.partial, (int)pg, w.ring_part,
                         (int)rb, fcg_m, w.fr, w.sc, learn->ls);
      hipLaunchKernelGGL(k_fcg_dir, dim3(pg), dim3(kVecThreads), 0, s, w.z, w.p, w.ring, n, fcg_m,
                         w.fr, w.sc);
    } else if (learn) {
      if ((e = launch_cg_pull<true>(pc, pg, x, w.r, w.p, w.q, w.z, w.partial, w.sc, s)) !=
          hipSuccess)
        return e;
      if ((e = coarse_correct(*learn, w.r, w.z, w.q, w.sc, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_cg_beta_flex, dim3(1), dim3(1024), 0, s, w.partial, (int)pg, w.sc,
                         learn->ls);
    } else {
      if ((e = launch_cg_pull<false>(pc, pg, x, w.r, w.p, w.q, w.z, w.partial, w.sc, s)) !=
          hipSuccess)
        return e;
      hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(1024), 0, s, w.partial, (int)pg, w.sc);
    }
    if (!ring)
      hipLaunchKernelGGL(k_cg_p, dim3(nblk(n)), dim3(kVecThreads), 0, s, w.z, w.p, n, w.sc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct CoreArgs {
  const double* b;
  double* x;
  double tol;
  int64_t maxit;
  int stop, precA, precS, timing, chunk;
  double* history;
  CoarseCtx* learn = nullptr;   // learned correction (flexible CG) when set
  int fcg_m = 1;                // directions kept by the flexible CG
};

struct CoreResult {
  int done = 0;
  int64_t iters = 0;
  double crit = 0, zz = 0, zn0 = 0;
  double t_spmv = 0, t_schw = 0;
  int64_t n_timed = 0;
};

// Events bracketing the SpMV and the block products of the steps of a
// chunk (timing mode).
static fc_status ensure_events(SolverWs& w, int chunk) {
  if ((int)w.tev.size() >= 4 * chunk) return FC_OK;
  const size_t old = w.tev.size();
  w.tev.resize(4 * chunk, nullptr);
  for (size_t i = old; i < w.tev.size(); ++i) FC_HIP(hipEventCreate(&w.tev[i]));
  return FC_OK;
}

// (Re)capture the chunk of steps into a graph when the buffers, precisions
// or length change.
// Capturing is host work: callers that time the solve on the device call
// this before their first event so the timed region does not include it.
static fc_status ensure_graph(fc_precond_s& pc, SolverWs& w, const CoreArgs& a, hipStream_t s) {
  const int chunk = a.chunk > 0 ? a.chunk : 16;
  const int prec = a.precA * 4 + a.precS + (a.learn ? 16 + 32 * a.fcg_m : 0);
  if (w.exec && w.key[0] == a.x && w.key_chunk == chunk && w.key_prec == prec) return FC_OK;
  if (w.exec) {
    FC_HIP(hipGraphExecDestroy(w.exec));
    w.exec = nullptr;
  }
  if (w.graph) {
    FC_HIP(hipGraphDestroy(w.graph));
    w.graph = nullptr;
  }
  w.key_prec = -1;
  FC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_steps(pc, w, a.x, chunk, a.precA, a.precS, s, nullptr, a.learn, 1,
                               a.fcg_m);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    FC_HIP(e != hipSuccess ? e : e2);
  }
  w.graph = g;
  FC_HIP(hipGraphInstantiate(&w.exec, g, nullptr, nullptr, 0));
  w.key[0] = a.x;
  w.key_chunk = chunk;
  w.key_prec = prec;
  return FC_OK;
}

// One PCG run from x = 0 on the solver stream s.
static fc_status pcg_core(fc_precond_s& pc, SolverWs& w, const CoreArgs& a, CoreResult* res,
                          hipStream_t s) {
  fc_problem_s& pb = *pc.pb;
  const int64_t n = pb.n_dofs;
  CgScalars init{};
  init.tol = a.tol;
  init.maxit = a.maxit;
  init.stop = a.stop;
  init.history = a.history;
  FC_HIP(hipMemcpyAsync(w.sc, &init, sizeof(CgScalars), hipMemcpyHostToDevice, s));
  // x = 0, r = b, z = S r, p = z
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, a.x, 0.0, n);
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, a.b, w.r, n);
  FC_HIP(hipGetLastError());
  FC_HIP(launch_schwarz_phase1(pc, a.precS, w.r, nullptr, nullptr, s));
  FC_HIP(launch_schwarz_pull(pc, w.r, w.z, s));
  if (a.learn) FC_HIP(coarse_correct(*a.learn, w.r, w.z, nullptr, w.sc, s));
  if (a.learn && a.fcg_m > 1) hipLaunchKernelGGL(k_fcg_reset, dim3(1), dim3(1), 0, s, w.fr);
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, w.z, w.p, n);
  hipLaunchKernelGGL(k_cg_start, dim3(kRedBlocks), dim3(256), 0, s, w.r, w.z, n, w.partial,
                     w.sc);
  FC_HIP(hipGetLastError());
  const int chunk = a.chunk > 0 ? a.chunk : 16;
  const int64_t max_chunks = (a.maxit + chunk - 1) / chunk + 1;
  int64_t launched = 0;
  if (a.timing) {
    // direct launches (events recorded by a captured graph carry no
    // timestamps here); every a.timing-th step is bracketed by events
    FC_TRY_ST(ensure_events(w, chunk));
    const int every = std::max(1, a.timing);
    int64_t iter_before = 0;
    for (;;) {
      FC_HIP(enqueue_steps(pc, w, a.x, chunk, a.precA, a.precS, s, w.tev.data(), a.learn, every,
                           a.fcg_m));
      ++launched;
      FC_HIP(hipMemcpyAsync(w.host, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
      FC_HIP(hipStreamSynchronize(s));
      const int64_t ran = std::min<int64_t>(chunk, w.host->iter - iter_before);
      iter_before = w.host->iter;
      for (int64_t it = 0; it < ran; ++it) {
        if (it % every) continue;
        float t0 = 0.f, t1 = 0.f;
        FC_HIP(hipEventElapsedTime(&t0, w.tev[4 * it + 0], w.tev[4 * it + 1]));
        FC_HIP(hipEventElapsedTime(&t1, w.tev[4 * it + 2], w.tev[4 * it + 3]));
        res->t_spmv += t0;
        res->t_schw += t1;
        res->n_timed += 1;
      }
      if (w.host->done != 0 || launched > max_chunks) break;
    }
  } else {
    FC_TRY_ST(ensure_graph(pc, w, a, s));
    for (;;) {
      FC_HIP(hipGraphLaunch(w.exec, s));
      ++launched;
      FC_HIP(hipMemcpyAsync(w.host, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
      FC_HIP(hipStreamSynchronize(s));
      if (w.host->done != 0 || launched > max_chunks) break;
    }
  }
  const CgScalars& h = *w.host;
  res->done = h.done;
  res->iters = h.iter;
  res->crit = h.crit;
  res->zz = h.zz;
  res->zn0 = h.zn0;
  return FC_OK;
}

// ||b - A x|| / ||b|| with the FP64 matrix; t receives A x.
static fc_status true_residual(fc_precond_s& pc, SolverWs& w, const double* b, const double* x,
                               double* t, hipStream_t s, double* rel, double* out_r = nullptr) {
  fc_problem_s& pb = *pc.pb;
  const int64_t n = pb.n_dofs;
  FC_HIP(launch_spmv(pb.A, x, t, s));
  if (out_r) hipLaunchKernelGGL(k_sub, dim3(1024), dim3(256), 0, s, b, t, out_r, n);
  double* out2 = w.partial + w.partial_len - 2;
  hipLaunchKernelGGL(k_resid, dim3(kRedBlocks), dim3(256), 0, s, b, t, n, w.partial, w.sc, out2);
  FC_HIP(hipGetLastError());
  FC_HIP(hipMemcpyAsync(w.host, out2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  FC_HIP(hipStreamSynchronize(s));
  const double* v = reinterpret_cast<const double*>(w.host);
  *rel = v[1] > 0 ? std::sqrt(v[0] / v[1]) : 0.0;
  return FC_OK;
}

static fc_status status_of(int done) {
  switch (done) {
    case 1: return FC_OK;
    case 2: return FC_E_NOTCONV;
    case 3: return FC_E_BREAKDOWN;
    case 4: return FC_E_NAN;
  }
  return FC_E_NOTCONV;
}

// The refinement's inner matrix: an FP32 copy of A, read only for the block
// rows whose functions touch no cell with eta_T < 1; the rows of functions
// on cut or fictitious cells keep FP64, so the low-energy modes of the cut
// cells (energies down to alpha, below the FP32 unit roundoff) keep their
// exact entries.  Problems without cell data read every row from FP32.
static fc_status ensure_mixed_matrix(fc_problem_s& pb, hipStream_t s) {
  DeviceBsr& A = pb.A;
  if (A.val32) return FC_OK;
  const int64_t nr = A.n_rows;
  std::vector<uint8_t> hi((size_t)nr, 0);
  const int64_t nn = pb.nn;
  if (!pb.eta.empty() && (int64_t)pb.elem_nodes_host.size() == pb.n_el * nn)
    for (int64_t e = 0; e < pb.n_el; ++e)
      if (pb.eta[e] < 1.0)
        for (int64_t a = 0; a < nn; ++a) hi[pb.elem_nodes_host[e * nn + a]] = 1;
  std::vector<int32_t> rh, rl;
  for (int64_t r = 0; r < nr; ++r) (hi[r] ? rh : rl).push_back((int32_t)r);
  auto up = [&](const std::vector<int32_t>& v, int32_t** d) -> fc_status {
    if (v.empty()) return FC_OK;
    FC_HIP(hipMalloc(d, v.size() * sizeof(int32_t)));
    FC_HIP(hipMemcpyAsync(*d, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    return FC_OK;
  };
  FC_TRY_ST(up(rh, &A.rows_hi));
  FC_TRY_ST(up(rl, &A.rows_lo));
  A.n_hi = (int64_t)rh.size();
  A.n_lo = (int64_t)rl.size();
  FC_HIP(hipMalloc(&A.val32, A.nnzb * A.bdim * A.bdim * sizeof(float)));
  FC_HIP(launch_cast_matrix(A, s));
  FC_HIP(hipStreamSynchronize(s));   // the host lists must outlive the copies
  return FC_OK;
}

fc_status pcg_solve(fc_precond_s& pc, const double* b, double* x, const fc_solve_opts& o,
                    fc_solve_info* info, hipStream_t user) {
  fc_problem_s& pb = *pc.pb;
  const int64_t n = pb.n_dofs;
  SolverWs* wp = nullptr;
  fc_status st = ensure_ws(pc, &wp);
  if (st != FC_OK) return st;
  SolverWs& w = *wp;
  hipStream_t s = w.stream;
  FC_HIP(hipEventRecord(w.ev[0], user));
  FC_HIP(hipStreamWaitEvent(s, w.ev[0], 0));

  fc_status result = FC_OK;
  int64_t iters = 0, outer = 1;
  double rel_true = 0.0, rel_prec = 0.0;
  CoreResult acc;
  int64_t fallbacks = 0;
  const bool low_s = o.mode == FC_MODE_S_F32 || o.mode == FC_MODE_S_BF16 ||
                     o.mode == FC_MODE_IR_F32 || o.mode == FC_MODE_IR_BF16;
  const int precS = !low_s ? 0
                    : (o.mode == FC_MODE_S_F32 || o.mode == FC_MODE_IR_F32) ? 1 : 2;
  if ((precS == 1 && !pc.Q32) || (precS == 2 && !pc.Lbf)) {
    set_error("fc_pcg_solve: the preconditioner holds no copy in the requested precision");
    return FC_E_ARG;
  }
  CoarseCtx* learn = nullptr;
  if (o.mode == FC_MODE_LEARNED) {
    if (!pc.coarse || !pc.coarse->model) {
      set_error("fc_pcg_solve: FC_MODE_LEARNED needs a network attached with fc_learned_attach");
      return FC_E_ARG;
    }
    // a network that validation found not to pay falls back to plain PCG
    if (pc.coarse->enabled) learn = pc.coarse;
    else fallbacks = 1;
  }
  const int fcg_m = o.fcg_m > 1 ? o.fcg_m : 1;
  if (fcg_m > kMaxFcg) {
    set_error("fc_pcg_solve: fcg_m above 64");
    return FC_E_ARG;
  }
  if (learn) FC_TRY_ST(ensure_ring(w, fcg_m));
  if (o.mode == FC_MODE_F64 || o.mode == FC_MODE_S_F32 || o.mode == FC_MODE_S_BF16 ||
      o.mode == FC_MODE_LEARNED) {
    // one PCG run with the FP64 matrix (and a low-precision S if asked, or
    // flexible CG with the learned correction)
    const int stop = o.mode == FC_MODE_LEARNED ? (int)FC_STOP_RESIDUAL : o.stop;
    CoreArgs a{b, x, o.tol, o.maxit, stop, 0, precS, o.timing, o.check_every, o.history_dev, learn,
               fcg_m};
    if (!o.timing) FC_TRY_ST(ensure_graph(pc, w, a, s));
    FC_HIP(hipEventRecord(w.ev[1], s));
    FC_TRY_ST(pcg_core(pc, w, a, &acc, s));
    iters = acc.iters;
    rel_prec = acc.zn0 > 0 ? std::sqrt(acc.zz) / acc.zn0 : 0.0;
    FC_HIP(hipEventRecord(w.ev[2], s));
    FC_TRY_ST(true_residual(pc, w, b, x, w.t, s, &rel_true));
    result = status_of(acc.done);
  } else {
    // iterative refinement: FP64 residual outside, low-precision PCG inside.
    // A correction that does not reduce the FP64 residual is undone and the
    // inner solves continue with the FP64 matrix (FP32 rounding can make
    // the stored matrix indefinite on the low-energy fictitious modes).
    int precA = 1;
    FC_TRY_ST(ensure_mixed_matrix(pb, s));
    if (!w.p32) FC_HIP(hipMalloc(&w.p32, n * sizeof(float)));
    if (!w.d) FC_HIP(hipMalloc(&w.d, n * sizeof(double)));
    if (!w.ro) FC_HIP(hipMalloc(&w.ro, n * sizeof(double)));
    FC_HIP(hipEventRecord(w.ev[1], s));
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, x, 0.0, n);
    hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, b, w.ro, n);
    FC_HIP(hipGetLastError());
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-4;
    result = FC_E_NOTCONV;
    outer = 0;
    double rel_prev = 1.0;
    for (;;) {
      ++outer;
      CoreArgs a{w.ro, w.d, inner_tol, std::max<int64_t>(1, o.maxit - iters), FC_STOP_RESIDUAL,
                 precA, precS, o.timing, o.check_every, nullptr};
      CoreResult cr;
      FC_TRY_ST(pcg_core(pc, w, a, &cr, s));
      iters += cr.iters;
      acc.t_spmv += cr.t_spmv;
      acc.t_schw += cr.t_schw;
      acc.n_timed += cr.n_timed;
      hipLaunchKernelGGL(k_axpy, dim3(1024), dim3(256), 0, s, 1.0, w.d, x, n);
      FC_HIP(hipGetLastError());
      FC_TRY_ST(true_residual(pc, w, b, x, w.t, s, &rel_true, w.ro));
      if (!(rel_true < 0.9 * rel_prev)) {
        // undo the correction and restore the residual of the previous x
        hipLaunchKernelGGL(k_axpy, dim3(1024), dim3(256), 0, s, -1.0, w.d, x, n);
        FC_HIP(hipGetLastError());
        FC_TRY_ST(true_residual(pc, w, b, x, w.t, s, &rel_true, w.ro));
        if (precA == 0) break;    // no progress even with the FP64 matrix
        precA = 0;
        ++fallbacks;
      } else {
        rel_prev = rel_true;
      }
      if (rel_true <= o.tol) {
        result = FC_OK;
        break;
      }
      if (iters >= o.maxit || outer >= 1000) break;
    }
    FC_HIP(hipEventRecord(w.ev[2], s));
  }
  FC_HIP(hipEventRecord(w.ev[3], s));
  FC_HIP(hipStreamSynchronize(s));
  FC_HIP(hipStreamWaitEvent(user, w.ev[3], 0));
  float ms = 0.f;
  FC_HIP(hipEventElapsedTime(&ms, w.ev[1], w.ev[2]));
  if (info) {
    info->iters = iters;
    info->outer_iters = outer;
    info->rel_res_true = rel_true;
    info->rel_res_prec = rel_prec;
    info->status = result;
    info->ms_solve = ms;
    info->ms_spmv = acc.t_spmv;
    info->ms_schwarz = acc.t_schw;
    info->n_timed = acc.n_timed;
    info->fallbacks = fallbacks;
  }
  return result;
}

// ------------------------------------------- solve without allocation
// Device scratch of fc_pcg_solve_noalloc: the CG vectors r, z, p, q and the
// residual product t (kNoAllocMaxDofs doubles each), the dot partials and
// the CG scalars.  One copy per GPU, held until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device.
constexpr int64_t kNoAllocMaxDofs = int64_t(1) << 19;
constexpr int64_t kNoAllocPartials = 4 * 4096 + 8;
constexpr int64_t kNoAllocScalars = (sizeof(CgScalars) + sizeof(double) - 1) / sizeof(double);
constexpr int64_t kNoAllocDoubles = 5 * kNoAllocMaxDofs + kNoAllocPartials + kNoAllocScalars;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch (looked up once per device).
static fc_status scratch_for(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("fc_pcg_solve_noalloc: device index above the supported maximum");
    return FC_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("fc_pcg_solve_noalloc: hipGetSymbolAddress: ") +
                hipGetErrorString(e));
      return FC_E_DEVICE;
    }
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return FC_OK;
}

// The scalars start from a kernel, not a copy from host memory, so the
// ticket of the last-workgroup reductions starts at zero on every call.
__global__ void k_sc_init(CgScalars* sc, double tol, int64_t maxit, int32_t stop,
                          double* history) {
  CgScalars v{};
  v.tol = tol;
  v.maxit = maxit;
  v.stop = stop;
  v.history = history;
  *sc = v;
}

fc_status pcg_solve_noalloc(fc_precond_s& pc, const double* b, double* x, const fc_solve_opts& o,
                            fc_solve_info* info, hipStream_t s) {
  fc_problem_s& pb = *pc.pb;
  const int64_t n = pb.n_dofs;
  if (n > kNoAllocMaxDofs) {
    set_error("fc_pcg_solve_noalloc: " + std::to_string(n) +
              " unknowns exceed the scratch maximum of " + std::to_string(kNoAllocMaxDofs));
    return FC_E_UNSUPPORTED;
  }
  if (o.mode != FC_MODE_F64 || o.timing != 0) {
    set_error("fc_pcg_solve_noalloc: only FP64 PCG without timing mode");
    return FC_E_UNSUPPORTED;
  }
  int dev = -1;
  FC_HIP(hipGetDevice(&dev));
  if (dev != pb.device) {
    set_error("fc_pcg_solve_noalloc: the current device is not the problem's");
    return FC_E_ARG;
  }
  // the SpMV with its fused dot (FC_CG_SPLIT_DOT=0) leaves one partial per
  // workgroup, which must fit the scratch's partial sums
  if (!split_dot() && (int64_t)spmv_num_blocks(pb.A) > (kNoAllocPartials - 8) / 4) {
    set_error("fc_pcg_solve_noalloc: too many SpMV partials for the fused dot");
    return FC_E_UNSUPPORTED;
  }
  double* base = nullptr;
  FC_TRY_ST(scratch_for(dev, &base));
  // a workspace view of the scratch: only the members the FP64 steps use
  SolverWs w;
  w.n = n;
  w.r = base;
  w.z = base + kNoAllocMaxDofs;
  w.p = base + 2 * kNoAllocMaxDofs;
  w.q = base + 3 * kNoAllocMaxDofs;
  w.t = base + 4 * kNoAllocMaxDofs;
  w.partial = base + 5 * kNoAllocMaxDofs;
  w.partial_len = kNoAllocPartials;
  w.sc = reinterpret_cast<CgScalars*>(w.partial + kNoAllocPartials);
  hipLaunchKernelGGL(k_sc_init, dim3(1), dim3(1), 0, s, w.sc, o.tol, o.maxit, o.stop,
                     o.history_dev);
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, x, 0.0, n);
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, b, w.r, n);
  FC_HIP(hipGetLastError());
  FC_HIP(launch_schwarz_phase1(pc, 0, w.r, nullptr, nullptr, s));
  FC_HIP(launch_schwarz_pull(pc, w.r, w.z, s));
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, w.z, w.p, n);
  hipLaunchKernelGGL(k_cg_start, dim3(kRedBlocks), dim3(256), 0, s, w.r, w.z, n, w.partial,
                     w.sc);
  FC_HIP(hipGetLastError());
  const int chunk = o.check_every > 0 ? o.check_every : 16;
  const int64_t max_chunks = (o.maxit + chunk - 1) / chunk + 1;
  CgScalars h{};
  for (int64_t launched = 0;;) {
    FC_HIP(enqueue_steps(pc, w, x, chunk, 0, 0, s));
    ++launched;
    FC_HIP(hipMemcpyAsync(&h, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    if (h.done != 0 || launched > max_chunks) break;
  }
  // ||b - A x|| / ||b|| with the FP64 matrix
  FC_HIP(launch_spmv(pb.A, x, w.t, s));
  double* out2 = w.partial + w.partial_len - 2;
  hipLaunchKernelGGL(k_resid, dim3(kRedBlocks), dim3(256), 0, s, b, w.t, n, w.partial, w.sc,
                     out2);
  FC_HIP(hipGetLastError());
  double v[2] = {0.0, 0.0};
  FC_HIP(hipMemcpyAsync(v, out2, sizeof(v), hipMemcpyDeviceToHost, s));
  FC_HIP(hipStreamSynchronize(s));
  const fc_status result = status_of(h.done);
  if (info) {
    *info = fc_solve_info{};
    info->iters = h.iter;
    info->outer_iters = 1;
    info->rel_res_true = v[1] > 0 ? std::sqrt(v[0] / v[1]) : 0.0;
    info->rel_res_prec = h.zn0 > 0 ? std::sqrt(h.zz) / h.zn0 : 0.0;
    info->status = result;
  }
  return result;
}

void solver_invalidate_graph(fc_precond_s& pc) {
  SolverWs* w = pc.ws;
  if (!w) return;
  if (w->exec) (void)hipGraphExecDestroy(w->exec);
  if (w->graph) (void)hipGraphDestroy(w->graph);
  w->exec = nullptr;
  w->graph = nullptr;
  w->key[0] = nullptr;
  w->key_prec = -1;
}

}  // namespace fc

using namespace fc;

extern "C" fc_status fc_learned_snapshots(fc_precond pc, const double* b, const double* xs,
                                          int32_t n_snap, const int32_t* iters, int32_t kind,
                                          double tol, float* xin, float* t, int32_t* n_taken,
                                          void* stream) {
  if (!pc || !b || !xs || n_snap < 1 || !iters || !xin || !t || kind < 0 || kind > 2) {
    set_error("fc_learned_snapshots: invalid arguments");
    return FC_E_ARG;
  }
  for (int j = 0; j < n_snap; ++j)
    if (iters[j] < 0 || (j > 0 && iters[j] <= iters[j - 1])) {
      set_error("fc_learned_snapshots: iterations must be ascending and non-negative");
      return FC_E_ARG;
    }
  if (n_taken) *n_taken = 0;
  hipStream_t user = (hipStream_t)stream;
  FC_TRY_ST(coarse_ensure(*pc, user));
  CoarseCtx& c = *pc->coarse;
  SolverWs* wp = nullptr;
  FC_TRY_ST(ensure_ws(*pc, &wp));
  SolverWs& w = *wp;
  fc_problem_s& pb = *pc->pb;
  const int64_t n = pb.n_dofs;
  if (!w.d) FC_HIP(hipMalloc(&w.d, n * sizeof(double)));
  double* x = w.d;
  hipStream_t s = w.stream;
  FC_HIP(hipEventRecord(w.ev[0], user));
  FC_HIP(hipStreamWaitEvent(s, w.ev[0], 0));
  CgScalars init{};
  init.tol = tol;
  init.maxit = (int64_t)iters[n_snap - 1] + 1;
  init.stop = FC_STOP_RESIDUAL;
  FC_HIP(hipMemcpyAsync(w.sc, &init, sizeof(CgScalars), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, x, 0.0, n);
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, b, w.r, n);
  FC_HIP(hipGetLastError());
  FC_HIP(launch_schwarz_phase1(*pc, 0, w.r, nullptr, nullptr, s));
  FC_HIP(launch_schwarz_pull(*pc, w.r, w.z, s));
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, w.z, w.p, n);
  hipLaunchKernelGGL(k_cg_start, dim3(kRedBlocks), dim3(256), 0, s, w.r, w.z, n, w.partial,
                     w.sc);
  FC_HIP(hipGetLastError());
  const int64_t nv = c.nvox;
  int j = 0;
  int64_t it = 0;
  auto take = [&]() -> fc_status {
    float* xo = xin + (int64_t)j * 2 * nv;
    float* to = t + (int64_t)j * nv;
    ++j;
    if (kind == 2) return coarse_snapshot_projection(c, w.r, xo, to, 1e-8, 20000, s);
    FC_HIP(coarse_snapshot(c, w.r, xs, x, kind == 0 ? w.z : nullptr, xo, to, s));
    return FC_OK;
  };
  if (iters[0] == 0) FC_TRY_ST(take());
  while (j < n_snap) {
    FC_HIP(enqueue_steps(*pc, w, x, 1, 0, 0, s));
    ++it;
    FC_HIP(hipMemcpyAsync(w.host, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    if (w.host->iter != it) break;   // stopped before this step (flag set earlier)
    if (iters[j] == it) FC_TRY_ST(take());
    if (w.host->done != 0) break;
  }
  FC_HIP(hipEventRecord(w.ev[3], s));
  FC_HIP(hipStreamWaitEvent(user, w.ev[3], 0));
  FC_HIP(hipStreamSynchronize(s));
  if (n_taken) *n_taken = j;
  return FC_OK;
}

extern "C" fc_status fc_learned_validate(fc_precond pc, const double* b, double tol,
                                         int32_t fcg_m, int32_t* use_network,
                                         fc_solve_info* plain, fc_solve_info* learned,
                                         void* stream) {
  if (!pc || !b || !pc->coarse || !pc->coarse->model || !(tol > 0.0)) {
    set_error("fc_learned_validate: needs a preconditioner with an attached network, b, tol > 0");
    return FC_E_ARG;
  }
  hipStream_t user = (hipStream_t)stream;
  const int64_t n = pc->pb->n_dofs;
  double* x = nullptr;
  FC_HIP(hipMalloc(&x, n * sizeof(double)));
  fc_solve_opts o{tol, 300000, FC_STOP_RESIDUAL, FC_MODE_F64, 16, 1e-4, nullptr, 0};
  fc_solve_info ip{}, il{};
  pc->coarse->enabled = 1;
  const fc_status s1 = pcg_solve(*pc, b, x, o, &ip, user);
  o.mode = FC_MODE_LEARNED;
  o.fcg_m = fcg_m;
  const fc_status s2 = pcg_solve(*pc, b, x, o, &il, user);
  (void)hipStreamSynchronize(user);
  (void)hipFree(x);
  if (s1 != FC_OK && s1 != FC_E_NOTCONV && s1 != FC_E_BREAKDOWN && s1 != FC_E_NAN) return s1;
  if (s2 != FC_OK && s2 != FC_E_NOTCONV && s2 != FC_E_BREAKDOWN && s2 != FC_E_NAN) return s2;
  // keep the network only where it reaches tol and beats plain PCG in time
  const bool keep = s2 == FC_OK && (s1 != FC_OK || il.ms_solve < ip.ms_solve);
  pc->coarse->enabled = keep ? 1 : 0;
  if (use_network) *use_network = keep ? 1 : 0;
  if (plain) *plain = ip;
  if (learned) *learned = il;
  return FC_OK;
}

