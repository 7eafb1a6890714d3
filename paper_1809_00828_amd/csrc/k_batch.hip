// Batched Schwarz-PCG: many independent finite cell problems of uneven size
// iterate together.  Every PCG step of the whole batch is a fixed sequence
// of launches over segmented work lists (problem, tile), one launch per
// shape class, so the launch count does not grow with the number of
// problems; each problem keeps its own CG scalars and stop flag, and the
// work items of a converged problem return at once.  A chunk of steps is
// captured into one hipGraph and replayed until every problem has stopped.
//
// Shape classes and their launch variants are fixed at batch creation by a
// small autotuner: for every SpMV class (block dimension, mean row length)
// it times the group widths 8/16/32/64 on that class's own work items, and
// for every Schwarz class (block size m) it times the available block-
// product variants, keeping the fastest.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "dev_common.h"
#include "k_schwarz.h"
#include "k_spmv.h"
#include "schwarz_dev.h"

namespace fc {

struct BProb {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;       // row-SoA BSR
  int64_t n_rows;
  const int32_t* elem_nodes;
  const int32_t* block_elem;
  const double* Q;         // wrapped-diagonal symmetric local inverses
  const double* P;         // dense local inverses
  const int32_t* inv_ptr;
  const int32_t* inv_idx;
  const double* fallback;
  double* y;
  const double* b;
  double* x;
  int64_t n_blocks, n_dofs, voff;
  int32_t nn, m, bdim, pad;
  int32_t spmv_item0, spmv_items, pull_item0, pull_items;
};

// One tile of one problem.  slot is the item's fixed position in the
// partial-sum array, so a compacted list of the still-running problems'
// items writes where the per-problem reductions read.
struct WorkItem {
  int32_t prob, tile, slot;
};

// ------------------------------------------------------------ kernels
template <int B, int G>
__global__ __launch_bounds__(256) void kb_spmv(const BProb* __restrict__ probs,
                                               const WorkItem* __restrict__ items,
                                               const CgScalars* __restrict__ sc,
                                               const double* __restrict__ pvec,
                                               double* __restrict__ qvec) {
  constexpr int BB = B * B;
  constexpr int RPW = 256 / G;
  constexpr int U = B == 1 ? 8 : 2;   // blocks per lane per pass
  const WorkItem it = items[blockIdx.x];
  const BProb& P = probs[it.prob];
  if (sc[it.prob].done) return;
  const int64_t row = (int64_t)it.tile * RPW + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const double* x = pvec + P.voff;
  if (row >= P.n_rows) return;
  const int64_t base = P.rowptr[row];
  const int L = P.rowptr[row + 1] - (int32_t)base;
  const double* v = P.val + base * BB;
  double acc[B];
#pragma unroll
  for (int i = 0; i < B; ++i) acc[i] = 0.0;
  for (int k = lane; k < L; k += U * G) {
    int c[U];
    double a[U][BB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ku = k + u * G;
      const bool on = ku < L;
      // scalar rows read through the caches (5 % faster on a 64-member
      // batch), 3x3 blocks non-temporally
      if constexpr (B == 1)
        c[u] = on ? P.col[base + ku] : -1;
      else
        c[u] = on ? __builtin_nontemporal_load(P.col + base + ku) : -1;
#pragma unroll
      for (int e = 0; e < BB; ++e)
        if constexpr (B == 1)
          a[u][e] = on ? v[(int64_t)e * L + ku] : 0.0;
        else
          a[u][e] = on ? __builtin_nontemporal_load(v + (int64_t)e * L + ku) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < B; ++i)
#pragma unroll
        for (int j = 0; j < B; ++j)
          acc[i] = fma(a[u][i * B + j], c[u] >= 0 ? x[(int64_t)c[u] * B + j] : 0.0, acc[i]);
  }
#pragma unroll
  for (int i = 0; i < B; ++i) acc[i] = group_sum<G>(acc[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < B; ++i) qvec[P.voff + row * B + i] = acc[i];
  }
}

// (p, q) per pull tile into partial[3 n_items + slot]: the step length's
// dot runs as its own pass rather than at the end of every SpMV workgroup
// (which would hold a workgroup's waves until the slowest row finishes).
__global__ __launch_bounds__(256) void kb_pq(const BProb* __restrict__ probs,
                                             const WorkItem* __restrict__ items, int n_items,
                                             const CgScalars* __restrict__ sc,
                                             const double* __restrict__ pvec,
                                             const double* __restrict__ qvec,
                                             double* __restrict__ partial) {
  __shared__ double lds[16];
  const WorkItem it = items[blockIdx.x];
  const BProb& P = probs[it.prob];
  if (sc[it.prob].done) return;
  const int64_t i = (int64_t)it.tile * 256 + threadIdx.x;
  double a = 0.0;
  if (i < P.n_dofs) a = pvec[P.voff + i] * qvec[P.voff + i];
  a = block_sum(a, lds);
  if (threadIdx.x == 0) partial[3 * (int64_t)n_items + it.slot] = a;
}

// alpha per problem from its (p, q) partials (one workgroup per problem).
__global__ __launch_bounds__(256) void kb_alpha(const BProb* __restrict__ probs, CgScalars* sc,
                                                const double* __restrict__ partial, int n_items,
                                                const int32_t* __restrict__ active) {
  __shared__ double lds[16];
  const int k = active ? active[blockIdx.x] : (int)blockIdx.x;
  CgScalars& S = sc[k];
  if (S.done) return;
  const BProb& P = probs[k];
  const double* pp = partial + 3 * (int64_t)n_items + P.pull_item0;
  double t = 0.0;
  for (int i = threadIdx.x; i < P.pull_items; i += blockDim.x) t += pp[i];
  const double pq = block_sum(t, lds);
  if (threadIdx.x == 0) {
    S.pq = pq;
    S.iter += 1;
    if (!(pq > 0.0) || !(S.rz > 0.0))
      S.done = (pq != pq || S.rz != S.rz) ? 4 : 3;
    else
      S.alpha = S.rz / pq;
  }
}

// Schwarz phase 1 for a class of blocks of size m <= 64 (BPW blocks per
// wave) or m > 64 (one block per workgroup of 64*ceil(m/64) threads).
// Gathers r - alpha q (q may be null for the start).
template <bool kSmall>
__global__ __launch_bounds__(256) void kb_schwarz(const BProb* __restrict__ probs,
                                                  const WorkItem* __restrict__ items,
                                                  const CgScalars* __restrict__ sc,
                                                  const double* __restrict__ rvec,
                                                  const double* __restrict__ qvec, int m, int bpw) {
  __shared__ double rB[256];
  const WorkItem it = items[blockIdx.x];
  const CgScalars& S = sc[it.prob];
  if (S.done) return;
  const BProb& P = probs[it.prob];
  const double alpha = qvec ? S.alpha : 0.0;
  const double* r = rvec + P.voff;
  const double* q = qvec ? qvec + P.voff : nullptr;
  const int64_t stride = sym_block_stride_dev(m);
  if constexpr (kSmall) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lb = l / m, i = l % m;
    const int64_t blk = ((int64_t)it.tile * 4 + w) * bpw + lb;
    const bool active = lb < bpw && blk < P.n_blocks;
    if (active) {
      const int64_t e = P.block_elem[blk];
      const int64_t dof = (int64_t)P.elem_nodes[e * P.nn + i / P.bdim] * P.bdim + (i % P.bdim);
      rB[threadIdx.x] = gather_r(r, q, alpha, dof);
    }
    __syncthreads();
    if (!active) return;
    P.y[blk * m + i] = sym_row<double>(P.Q + blk * stride, &rB[w * 64 + lb * m], m, i);
  } else {
    // one block per workgroup, its stored rows staged through LDS
    __shared__ __align__(16) double tile[StageRows<double>::value * 256];
    const int64_t blk = it.tile;
    const int i = threadIdx.x;
    if (i < m) {
      const int64_t e = P.block_elem[blk];
      const int64_t dof = (int64_t)P.elem_nodes[e * P.nn + i / P.bdim] * P.bdim + (i % P.bdim);
      rB[i] = gather_r(r, q, alpha, dof);
    }
    // every thread's own entry of each stored row: for the batch's block
    // sizes (m = 125 at p = 4 in 3-D) 4.5 % faster than 16-byte runs
    const double v = sym_block_staged_rows<double>(P.Q + blk * stride, rB, m, i, tile);
    if (i < m) P.y[blk * m + i] = v;
  }
}

// Dense variant of the same product (autotuner candidate).
template <bool kSmall>
__global__ __launch_bounds__(256) void kb_schwarz_dense(const BProb* __restrict__ probs,
                                                        const WorkItem* __restrict__ items,
                                                        const CgScalars* __restrict__ sc,
                                                        const double* __restrict__ rvec,
                                                        const double* __restrict__ qvec, int m,
                                                        int bpw) {
  __shared__ double rB[256];
  const WorkItem it = items[blockIdx.x];
  const CgScalars& S = sc[it.prob];
  if (S.done) return;
  const BProb& P = probs[it.prob];
  const double alpha = qvec ? S.alpha : 0.0;
  const double* r = rvec + P.voff;
  const double* q = qvec ? qvec + P.voff : nullptr;
  const int64_t stride = (int64_t)m * m;
  if constexpr (kSmall) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lb = l / m, i = l % m;
    const int64_t blk = ((int64_t)it.tile * 4 + w) * bpw + lb;
    const bool active = lb < bpw && blk < P.n_blocks;
    if (active) {
      const int64_t e = P.block_elem[blk];
      const int64_t dof = (int64_t)P.elem_nodes[e * P.nn + i / P.bdim] * P.bdim + (i % P.bdim);
      rB[threadIdx.x] = gather_r(r, q, alpha, dof);
    }
    __syncthreads();
    if (!active) return;
    P.y[blk * m + i] = dense_row<double>(P.P + blk * stride, &rB[w * 64 + lb * m], m, i);
  } else {
    const int64_t blk = it.tile;
    const int i = threadIdx.x;
    if (i < m) {
      const int64_t e = P.block_elem[blk];
      const int64_t dof = (int64_t)P.elem_nodes[e * P.nn + i / P.bdim] * P.bdim + (i % P.bdim);
      rB[i] = gather_r(r, q, alpha, dof);
    }
    __syncthreads();
    if (i >= m) return;
    P.y[blk * m + i] = dense_row<double>(P.P + blk * stride, rB, m, i);
  }
}

// Pull + x, r updates + partial dots (mode 1), or the start (mode 0: z = S r
// only, dots of r and z).
template <int kMode>
__global__ __launch_bounds__(256) void kb_pull(const BProb* __restrict__ probs,
                                               const WorkItem* __restrict__ items, int n_items,
                                               const CgScalars* __restrict__ sc,
                                               double* __restrict__ rvec,
                                               const double* __restrict__ pvec,
                                               const double* __restrict__ qvec,
                                               double* __restrict__ zvec,
                                               double* __restrict__ partial) {
  __shared__ double lds[16];
  const WorkItem it = items[blockIdx.x];
  const BProb& P = probs[it.prob];
  double a = 0.0, b = 0.0, c = 0.0;
  if (!sc[it.prob].done) {
    const int64_t i = (int64_t)it.tile * 256 + threadIdx.x;
    if (i < P.n_dofs) {
      const int bd = P.bdim;
      const int64_t node = i / bd;
      const int cc = (int)(i - node * bd);
      double s = 0.0;
      for (int32_t e = P.inv_ptr[node]; e < P.inv_ptr[node + 1]; ++e)
        s += P.y[(int64_t)P.inv_idx[e] + cc];
      const int64_t g = P.voff + i;
      double ri = rvec[g];
      if constexpr (kMode == 1) {
        const double alpha = sc[it.prob].alpha;
        ri = fma(-alpha, qvec[g], ri);
        P.x[i] = fma(alpha, pvec[g], P.x[i]);
        rvec[g] = ri;
      }
      const double zi = fma(P.fallback[i], ri, s);
      zvec[g] = zi;
      a = ri * zi;
      b = zi * zi;
      c = ri * ri;
    }
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  c = block_sum(c, lds);
  if (threadIdx.x == 0) {
    partial[it.slot] = a;
    partial[n_items + it.slot] = b;
    partial[2 * n_items + it.slot] = c;
  }
}

// Per-problem stop test and beta (mode 1) or start (mode 0).
template <int kMode>
__global__ __launch_bounds__(256) void kb_beta(const BProb* __restrict__ probs, CgScalars* sc,
                                               const double* __restrict__ partial, int n_items,
                                               const int32_t* __restrict__ active) {
  __shared__ double lds[16];
  const int k = active ? active[blockIdx.x] : (int)blockIdx.x;
  CgScalars& S = sc[k];
  if (kMode == 1 && S.done) return;
  const BProb& P = probs[k];
  double ta = 0.0, tb = 0.0, tc = 0.0;
  for (int i = threadIdx.x; i < P.pull_items; i += blockDim.x) {
    ta += partial[P.pull_item0 + i];
    tb += partial[n_items + P.pull_item0 + i];
    tc += partial[2 * n_items + P.pull_item0 + i];
  }
  const double rz = block_sum(ta, lds);
  const double zz = block_sum(tb, lds);
  const double rr = block_sum(tc, lds);
  if (threadIdx.x != 0) return;
  if constexpr (kMode == 0) {
    S.rz = rz;
    S.zz = zz;
    S.rr = rr;
    S.iter = 0;
    S.zn0 = sqrt(zz);
    S.rn0 = sqrt(rr);
    S.crit0 = S.stop == FC_STOP_PRECOND ? S.zn0 : S.rn0;
    S.crit = S.crit0 > 0 ? 1.0 : 0.0;
    S.done = !(S.crit0 == S.crit0) ? 4 : (S.crit0 == 0.0 ? 1 : 0);
  } else {
    const double crit = (S.stop == FC_STOP_PRECOND ? sqrt(zz) : sqrt(rr)) / S.crit0;
    S.zz = zz;
    S.rr = rr;
    S.crit = crit;
    if (!(crit == crit) || !(rz == rz) || isinf(rz))
      S.done = 4;
    else if (crit <= S.tol)
      S.done = 1;
    else if (S.iter >= S.maxit)
      S.done = 2;
    S.beta = rz / S.rz;
    S.rz = rz;
  }
}

// mode 0: r = b, x = 0;  mode 1: p = z + beta p;  mode 2: p = z
template <int kMode>
__global__ __launch_bounds__(256) void kb_vec(const BProb* __restrict__ probs,
                                              const WorkItem* __restrict__ items,
                                              const CgScalars* __restrict__ sc,
                                              double* __restrict__ rvec,
                                              double* __restrict__ pvec,
                                              const double* __restrict__ zvec) {
  const WorkItem it = items[blockIdx.x];
  const BProb& P = probs[it.prob];
  if (kMode == 1 && sc[it.prob].done) return;
  const int64_t i = (int64_t)it.tile * 256 + threadIdx.x;
  if (i >= P.n_dofs) return;
  const int64_t g = P.voff + i;
  if constexpr (kMode == 0) {
    rvec[g] = P.b[i];
    P.x[i] = 0.0;
  } else if constexpr (kMode == 1) {
    pvec[g] = fma(sc[it.prob].beta, pvec[g], zvec[g]);
  } else {
    pvec[g] = zvec[g];
  }
}

// ---------------------------------------------------------- host side
// items: every tile of every problem of the class; act / d_act: the tiles
// of the problems still running, which the captured iteration launches.
struct SpmvClass {
  int B, G;
  std::vector<WorkItem> items;
  WorkItem* d_items = nullptr;
  int item_base = 0;
  int n_act = 0;
  WorkItem* d_act = nullptr;
};

struct SchwarzClass {
  int m, bpw, variant;   // variant: 0 symmetric, 1 dense
  bool small;
  std::vector<WorkItem> items;
  WorkItem* d_items = nullptr;
  int n_act = 0;
  WorkItem* d_act = nullptr;
};

}  // namespace fc

struct fc_batch_s {
  int32_t nprob = 0;
  int64_t total_dofs = 0;
  std::vector<fc_precond> pcs;
  std::vector<fc::BProb> host;
  fc::BProb* d_probs = nullptr;
  std::vector<fc::SpmvClass> spmv;
  std::vector<fc::SchwarzClass> schw;
  std::vector<fc::WorkItem> pull_items;
  fc::WorkItem* d_pull = nullptr;
  int n_act_pull = 0;                 // compacted pull items (see SpmvClass)
  fc::WorkItem* d_act_pull = nullptr;
  int n_act_probs = 0;                // problems still running
  int32_t* d_act_probs = nullptr;
  int64_t act_dofs = 0;               // unknowns of the problems in the lists
  int spmv_total = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *partial = nullptr;
  fc::CgScalars* sc = nullptr;
  fc::CgScalars* host_sc = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<const double*> key_b;
  std::vector<double*> key_x;
  int key_chunk = 0;
  std::string report;
};

namespace fc {

static void destroy_batch(fc_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& c : b->spmv)
    for (void* p : {(void*)c.d_items, (void*)c.d_act}) if (p) (void)hipFree(p);
  for (auto& c : b->schw)
    for (void* p : {(void*)c.d_items, (void*)c.d_act}) if (p) (void)hipFree(p);
  for (void* p : {(void*)b->d_probs, (void*)b->d_pull, (void*)b->d_act_pull,
                  (void*)b->d_act_probs, (void*)b->r, (void*)b->z, (void*)b->p, (void*)b->q,
                  (void*)b->partial, (void*)b->sc})
    if (p) (void)hipFree(p);
  if (b->host_sc) (void)hipHostFree(b->host_sc);
  for (auto& e : b->ev) if (e) (void)hipEventDestroy(e);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

template <int B>
static void launch_bspmv_G(int G, dim3 g, hipStream_t s, const BProb* probs, const WorkItem* it,
                           const CgScalars* sc, const double* p, double* q) {
  switch (G) {
    case 8: hipLaunchKernelGGL((kb_spmv<B, 8>), g, dim3(256), 0, s, probs, it, sc, p, q); break;
    case 16: hipLaunchKernelGGL((kb_spmv<B, 16>), g, dim3(256), 0, s, probs, it, sc, p, q); break;
    case 32: hipLaunchKernelGGL((kb_spmv<B, 32>), g, dim3(256), 0, s, probs, it, sc, p, q); break;
    default: hipLaunchKernelGGL((kb_spmv<B, 64>), g, dim3(256), 0, s, probs, it, sc, p, q); break;
  }
}

static hipError_t launch_spmv_class(fc_batch_s& bt, const SpmvClass& c, const WorkItem* items,
                                    int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 g((unsigned)n);
  switch (c.B) {
    case 1: launch_bspmv_G<1>(c.G, g, s, bt.d_probs, items, bt.sc, bt.p, bt.q); break;
    case 2: launch_bspmv_G<2>(c.G, g, s, bt.d_probs, items, bt.sc, bt.p, bt.q); break;
    case 3: launch_bspmv_G<3>(c.G, g, s, bt.d_probs, items, bt.sc, bt.p, bt.q); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_schwarz_class(fc_batch_s& bt, const SchwarzClass& c, const WorkItem* items,
                                       int n, const double* q, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int threads = c.small ? 256 : 64 * ((c.m + 63) / 64);
  dim3 g((unsigned)n), b((unsigned)threads);
  if (c.variant == 0) {
    if (c.small)
      hipLaunchKernelGGL(kb_schwarz<true>, g, b, 0, s, bt.d_probs, items, bt.sc, bt.r, q, c.m, c.bpw);
    else
      hipLaunchKernelGGL(kb_schwarz<false>, g, b, 0, s, bt.d_probs, items, bt.sc, bt.r, q, c.m, c.bpw);
  } else {
    if (c.small)
      hipLaunchKernelGGL(kb_schwarz_dense<true>, g, b, 0, s, bt.d_probs, items, bt.sc, bt.r, q, c.m, c.bpw);
    else
      hipLaunchKernelGGL(kb_schwarz_dense<false>, g, b, 0, s, bt.d_probs, items, bt.sc, bt.r, q, c.m, c.bpw);
  }
  return hipGetLastError();
}

// The steps launch the compacted lists: tiles and problems still running.
static hipError_t enqueue_batch_steps(fc_batch_s& bt, int chunk, hipStream_t s) {
  const int np = (int)bt.pull_items.size();
  const int na = bt.n_act_pull;
  if (bt.n_act_probs == 0) return hipSuccess;
  for (int it = 0; it < chunk; ++it) {
    for (auto& c : bt.spmv) {
      hipError_t e = launch_spmv_class(bt, c, c.d_act, c.n_act, s);
      if (e != hipSuccess) return e;
    }
    if (na > 0) {
      hipLaunchKernelGGL(kb_pq, dim3(na), dim3(256), 0, s, bt.d_probs, bt.d_act_pull, np, bt.sc,
                         bt.p, bt.q, bt.partial);
    }
    hipLaunchKernelGGL(kb_alpha, dim3(bt.n_act_probs), dim3(256), 0, s, bt.d_probs, bt.sc,
                       bt.partial, np, bt.d_act_probs);
    for (auto& c : bt.schw) {
      hipError_t e = launch_schwarz_class(bt, c, c.d_act, c.n_act, bt.q, s);
      if (e != hipSuccess) return e;
    }
    if (na > 0) {
      hipLaunchKernelGGL(kb_pull<1>, dim3(na), dim3(256), 0, s, bt.d_probs, bt.d_act_pull, np,
                         bt.sc, bt.r, bt.p, bt.q, bt.z, bt.partial);
    }
    hipLaunchKernelGGL(kb_beta<1>, dim3(bt.n_act_probs), dim3(256), 0, s, bt.d_probs, bt.sc,
                       bt.partial, np, bt.d_act_probs);
    if (na > 0) {
      hipLaunchKernelGGL(kb_vec<1>, dim3(na), dim3(256), 0, s, bt.d_probs, bt.d_act_pull, bt.sc,
                         bt.r, bt.p, bt.z);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Time `reps` launches of fn on stream s (ms per launch).
template <class F>
static float time_launches(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, F&& fn) {
  fn();
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < reps; ++i) fn();
  (void)hipEventRecord(e1, s);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  return ms / reps;
}

}  // namespace fc

using namespace fc;

#define FC_TRY_B(x)                 \
  do {                              \
    fc_status s_ = (x);             \
    if (s_ != FC_OK) return s_;     \
  } while (0)

extern "C" fc_status fc_batch_create(int32_t nprob, const fc_problem* problems,
                                     const fc_precond* preconds, int32_t autotune, void* stream,
                                     fc_batch* out) {
  if (nprob <= 0 || !problems || !preconds || !out) {
    set_error("fc_batch_create: invalid arguments");
    return FC_E_ARG;
  }
  *out = nullptr;
  std::unique_ptr<fc_batch_s, void (*)(fc_batch_s*)> bt(new fc_batch_s(), destroy_batch);
  fc_batch_s& B = *bt;
  B.nprob = nprob;
  hipStream_t user = (hipStream_t)stream;
  FC_HIP(hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking));
  for (auto& e : B.ev) FC_HIP(hipEventCreate(&e));
  hipStream_t s = B.stream;
  B.host.resize(nprob);
  B.pcs.assign(preconds, preconds + nprob);
  int64_t voff = 0;
  // shape classes
  std::map<std::pair<int, int>, int> spmv_key;   // (B, row-length bucket) -> class
  std::map<int, int> schw_key;                   // m -> class
  for (int k = 0; k < nprob; ++k) {
    fc_problem pb = problems[k];
    fc_precond pc = preconds[k];
    if (!pb || !pc || pc->pb != pb) {
      set_error("fc_batch_create: problem/preconditioner mismatch");
      return FC_E_ARG;
    }
    if (!pc->Q) {
      set_error("fc_batch_create: preconditioner without symmetric copy");
      return FC_E_ARG;
    }
    if (pc->bnodes) {
      set_error("fc_batch_create: vertex-patch preconditioners are not batched");
      return FC_E_UNSUPPORTED;
    }
    BProb& P = B.host[k];
    std::memset(&P, 0, sizeof(P));
    P.rowptr = pb->A.rowptr;
    P.col = pb->A.col;
    P.val = pb->A.val;
    P.n_rows = pb->A.n_rows;
    P.elem_nodes = pb->elem_nodes;
    P.block_elem = pc->block_elem;
    P.Q = pc->Q;
    P.P = pc->P;
    P.inv_ptr = pc->inv_ptr;
    P.inv_idx = pc->inv_idx;
    P.fallback = pc->fallback;
    P.y = pc->y;
    P.n_blocks = pc->n_blocks;
    P.n_dofs = pb->n_dofs;
    P.voff = voff;
    P.nn = pc->nn;
    P.m = pc->m;
    P.bdim = pb->bdim;
    voff += pb->n_dofs;
    const double mean = pb->A.n_rows ? double(pb->A.nnzb) / double(pb->A.n_rows) : 1.0;
    const int bucket = mean < 12 ? 0 : mean < 24 ? 1 : mean < 48 ? 2 : mean < 96 ? 3 : 4;
    auto sk = std::make_pair(pb->bdim, bucket);
    if (!spmv_key.count(sk)) {
      spmv_key[sk] = (int)B.spmv.size();
      SpmvClass c;
      c.B = pb->bdim;
      c.G = bucket == 0 ? 8 : bucket == 1 ? 16 : bucket == 2 ? 32 : 64;
      B.spmv.push_back(c);
    }
    if (!schw_key.count(P.m)) {
      schw_key[P.m] = (int)B.schw.size();
      SchwarzClass c;
      c.m = P.m;
      c.small = P.m <= 64;
      c.bpw = c.small ? 64 / P.m : 1;
      c.variant = 0;
      B.schw.push_back(c);
    }
  }
  B.total_dofs = voff;
  // items (SpMV tiles depend on G, rebuilt after tuning)
  auto build_spmv_items = [&](SpmvClass& c, int cls) {
    c.items.clear();
    for (int k = 0; k < nprob; ++k) {
      fc_problem pb = problems[k];
      const double mean = pb->A.n_rows ? double(pb->A.nnzb) / double(pb->A.n_rows) : 1.0;
      const int bucket = mean < 12 ? 0 : mean < 24 ? 1 : mean < 48 ? 2 : mean < 96 ? 3 : 4;
      if (spmv_key[std::make_pair(pb->bdim, bucket)] != cls) continue;
      const int rpw = 256 / c.G;
      const int64_t nt = (pb->A.n_rows + rpw - 1) / rpw;
      for (int64_t t = 0; t < nt; ++t)
        c.items.push_back({k, (int32_t)t, (int32_t)c.items.size()});
    }
  };
  for (size_t c = 0; c < B.spmv.size(); ++c) build_spmv_items(B.spmv[c], (int)c);
  for (auto& c : B.schw) {
    for (int k = 0; k < nprob; ++k) {
      if (B.host[k].m != c.m) continue;
      const int64_t per = c.small ? 4 * (int64_t)c.bpw : 1;
      const int64_t nt = (B.host[k].n_blocks + per - 1) / per;
      for (int64_t t = 0; t < nt; ++t)
        c.items.push_back({k, (int32_t)t, (int32_t)c.items.size()});
    }
  }
  for (int k = 0; k < nprob; ++k) {
    const int64_t nt = (B.host[k].n_dofs + 255) / 256;
    B.host[k].pull_item0 = (int32_t)B.pull_items.size();
    B.host[k].pull_items = (int32_t)nt;
    for (int64_t t = 0; t < nt; ++t)
      B.pull_items.push_back({k, (int32_t)t, (int32_t)B.pull_items.size()});
  }
  auto upload_items = [&](std::vector<WorkItem>& v, WorkItem** d) -> fc_status {
    if (*d) {
      FC_HIP(hipFree(*d));
      *d = nullptr;
    }
    if (v.empty()) return FC_OK;
    FC_HIP(hipMalloc(d, v.size() * sizeof(WorkItem)));
    FC_HIP(hipMemcpy(*d, v.data(), v.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    return FC_OK;
  };
  auto finalize_spmv_ranges = [&]() {
    int base = 0;
    for (auto& c : B.spmv) {
      c.item_base = base;
      for (size_t i = 0; i < c.items.size(); ++i) {
        c.items[i].slot = base + (int32_t)i;
        BProb& P = B.host[c.items[i].prob];
        if (i == 0 || c.items[i - 1].prob != c.items[i].prob) {
          P.spmv_item0 = base + (int)i;
          P.spmv_items = 0;
        }
        P.spmv_items++;
      }
      base += (int)c.items.size();
    }
    B.spmv_total = base;
  };
  finalize_spmv_ranges();
  for (auto& c : B.spmv) FC_TRY_B(upload_items(c.items, &c.d_items));
  for (auto& c : B.schw) FC_TRY_B(upload_items(c.items, &c.d_items));
  FC_TRY_B(upload_items(B.pull_items, &B.d_pull));
  const int64_t n = B.total_dofs;
  FC_HIP(hipMalloc(&B.r, n * sizeof(double)));
  FC_HIP(hipMalloc(&B.z, n * sizeof(double)));
  FC_HIP(hipMalloc(&B.p, n * sizeof(double)));
  FC_HIP(hipMalloc(&B.q, n * sizeof(double)));
  // partials: SpMV items for every candidate width (<= 8 rows per item
  // minimum) and 3 per pull item
  int64_t max_spmv = 0;
  for (int k = 0; k < nprob; ++k) max_spmv += (B.host[k].n_rows + 3) / 4 + 1;
  const int64_t plen = std::max<int64_t>(max_spmv, 4 * (int64_t)B.pull_items.size()) + 8;
  FC_HIP(hipMalloc(&B.partial, plen * sizeof(double)));
  FC_HIP(hipMalloc(&B.sc, nprob * sizeof(CgScalars)));
  FC_HIP(hipMemset(B.sc, 0, nprob * sizeof(CgScalars)));
  FC_HIP(hipHostMalloc(&B.host_sc, nprob * sizeof(CgScalars), hipHostMallocDefault));
  FC_HIP(hipMalloc(&B.d_probs, nprob * sizeof(BProb)));
  FC_HIP(hipMemcpy(B.d_probs, B.host.data(), nprob * sizeof(BProb), hipMemcpyHostToDevice));
  FC_HIP(hipEventRecord(B.ev[0], user));
  FC_HIP(hipStreamWaitEvent(s, B.ev[0], 0));

  std::ostringstream rep;
  if (autotune) {
    // all problems active (done = 0) on random-free data: p = q = r = 0 is
    // enough to time memory traffic of the real matrices and blocks
    FC_HIP(hipMemsetAsync(B.p, 0, n * sizeof(double), s));
    FC_HIP(hipMemsetAsync(B.r, 0, n * sizeof(double), s));
    for (size_t ci = 0; ci < B.spmv.size(); ++ci) {
      SpmvClass& c = B.spmv[ci];
      float best = 1e30f;
      int bestG = c.G;
      for (int G : {8, 16, 32, 64}) {
        SpmvClass trial = c;
        trial.G = G;
        build_spmv_items(trial, (int)ci);
        WorkItem* d = nullptr;
        FC_TRY_B(upload_items(trial.items, &d));
        trial.item_base = 0;
        float ms = time_launches(s, B.ev[1], B.ev[2], 3, [&]() {
          (void)launch_spmv_class(B, trial, d, (int)trial.items.size(), s);
        });
        (void)hipFree(d);
        rep << "spmv B=" << c.B << " class " << ci << " G=" << G << ": " << ms << " ms\n";
        if (ms < best) {
          best = ms;
          bestG = G;
        }
      }
      c.G = bestG;
      build_spmv_items(c, (int)ci);
    }
    for (auto& c : B.schw) {
      float best = 1e30f;
      int bestv = 0;
      for (int v : {0, 1}) {
        c.variant = v;
        float ms = time_launches(s, B.ev[1], B.ev[2], 3, [&]() {
          (void)launch_schwarz_class(B, c, c.d_items, (int)c.items.size(), nullptr, s);
        });
        rep << "schwarz m=" << c.m << " " << (v ? "dense" : "symmetric") << ": " << ms << " ms\n";
        if (ms < best) {
          best = ms;
          bestv = v;
        }
      }
      c.variant = bestv;
    }
    FC_HIP(hipGetLastError());
    finalize_spmv_ranges();
    for (auto& c : B.spmv) FC_TRY_B(upload_items(c.items, &c.d_items));
    FC_HIP(hipMemcpy(B.d_probs, B.host.data(), nprob * sizeof(BProb), hipMemcpyHostToDevice));
  }
  for (auto& c : B.spmv)
    rep << "chosen spmv B=" << c.B << " G=" << c.G << " items=" << c.items.size() << "\n";
  for (auto& c : B.schw)
    rep << "chosen schwarz m=" << c.m << " " << (c.variant ? "dense" : "symmetric")
        << " items=" << c.items.size() << "\n";
  B.report = rep.str();
  for (auto& c : B.spmv)
    if (!c.items.empty()) FC_HIP(hipMalloc(&c.d_act, c.items.size() * sizeof(WorkItem)));
  for (auto& c : B.schw)
    if (!c.items.empty()) FC_HIP(hipMalloc(&c.d_act, c.items.size() * sizeof(WorkItem)));
  FC_HIP(hipMalloc(&B.d_act_pull, B.pull_items.size() * sizeof(WorkItem)));
  FC_HIP(hipMalloc(&B.d_act_probs, nprob * sizeof(int32_t)));
  B.act_dofs = -1;   // lists not built yet
  FC_HIP(hipStreamSynchronize(s));
  *out = bt.release();
  return FC_OK;
}

extern "C" fc_status fc_batch_info(fc_batch bt, int64_t* total_dofs, int32_t* n_spmv_classes,
                                   int32_t* n_schwarz_classes, char* report, int64_t report_len) {
  if (!bt) return FC_E_ARG;
  if (total_dofs) *total_dofs = bt->total_dofs;
  if (n_spmv_classes) *n_spmv_classes = (int32_t)bt->spmv.size();
  if (n_schwarz_classes) *n_schwarz_classes = (int32_t)bt->schw.size();
  if (report && report_len > 0) {
    const size_t k = std::min<size_t>(bt->report.size(), (size_t)report_len - 1);
    std::memcpy(report, bt->report.data(), k);
    report[k] = '\0';
  }
  return FC_OK;
}

// Launched lists = the tiles of the problems marked running (synchronous
// upload into the full-size arrays allocated at creation).
static fc_status compact_lists(fc_batch_s& B, const std::vector<char>& running) {
  auto filter = [&](const std::vector<WorkItem>& all, WorkItem* d, int* n) -> fc_status {
    std::vector<WorkItem> v;
    v.reserve(all.size());
    for (const WorkItem& w : all)
      if (running[w.prob]) v.push_back(w);
    *n = (int)v.size();
    if (!v.empty()) FC_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    return FC_OK;
  };
  for (auto& c : B.spmv) FC_TRY_B(filter(c.items, c.d_act, &c.n_act));
  for (auto& c : B.schw) FC_TRY_B(filter(c.items, c.d_act, &c.n_act));
  FC_TRY_B(filter(B.pull_items, B.d_act_pull, &B.n_act_pull));
  std::vector<int32_t> ap;
  int64_t dofs = 0;
  for (int k = 0; k < B.nprob; ++k)
    if (running[k]) {
      ap.push_back(k);
      dofs += B.host[k].n_dofs;
    }
  B.n_act_probs = (int)ap.size();
  B.act_dofs = dofs;
  if (!ap.empty())
    FC_HIP(hipMemcpy(B.d_act_probs, ap.data(), ap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return FC_OK;
}

// Capture `chunk` steps over the current lists into the batch's graph.
static fc_status capture_steps(fc_batch_s& B, int chunk, hipStream_t s) {
  if (B.exec) {
    FC_HIP(hipGraphExecDestroy(B.exec));
    B.exec = nullptr;
  }
  if (B.graph) {
    FC_HIP(hipGraphDestroy(B.graph));
    B.graph = nullptr;
  }
  FC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_batch_steps(B, chunk, s);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess) FC_HIP(e);
  FC_HIP(e2);
  B.graph = g;
  FC_HIP(hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0));
  B.key_chunk = chunk;
  return FC_OK;
}

extern "C" fc_status fc_pcg_solve_batch(fc_batch bt, const double* const* b_dev,
                                        double* const* x_dev, const fc_solve_opts* opts,
                                        fc_solve_info* infos, void* stream) {
  if (!bt || !b_dev || !x_dev) {
    set_error("fc_pcg_solve_batch: invalid arguments");
    return FC_E_ARG;
  }
  fc_solve_opts o{1e-8, 300000, FC_STOP_PRECOND, FC_MODE_F64, 16, 1e-4, nullptr, 0};
  if (opts) o = *opts;
  if (o.mode != FC_MODE_F64 || !(o.tol >= 0.0) || o.maxit < 0) {
    set_error("fc_pcg_solve_batch: only FP64 mode with valid tol/maxit is supported");
    return FC_E_UNSUPPORTED;
  }
  fc_batch_s& B = *bt;
  hipStream_t s = B.stream;
  hipStream_t user = (hipStream_t)stream;
  bool changed = false;
  if ((int)B.key_b.size() != B.nprob) {
    B.key_b.assign(B.nprob, nullptr);
    B.key_x.assign(B.nprob, nullptr);
  }
  for (int k = 0; k < B.nprob; ++k) {
    if (!b_dev[k] || !x_dev[k]) {
      set_error("fc_pcg_solve_batch: NULL vector");
      return FC_E_ARG;
    }
    if (B.host[k].b != b_dev[k] || B.host[k].x != x_dev[k]) changed = true;
    B.host[k].b = b_dev[k];
    B.host[k].x = x_dev[k];
  }
  FC_HIP(hipEventRecord(B.ev[0], user));
  FC_HIP(hipStreamWaitEvent(s, B.ev[0], 0));
  if (changed)
    FC_HIP(hipMemcpyAsync(B.d_probs, B.host.data(), B.nprob * sizeof(BProb),
                          hipMemcpyHostToDevice, s));
  std::vector<CgScalars> init(B.nprob);
  for (auto& c : init) {
    std::memset(&c, 0, sizeof(c));
    c.tol = o.tol;
    c.maxit = o.maxit;
    c.stop = o.stop;
  }
  FC_HIP(hipMemcpyAsync(B.sc, init.data(), B.nprob * sizeof(CgScalars), hipMemcpyHostToDevice, s));
  FC_HIP(hipEventRecord(B.ev[1], s));
  const int np = (int)B.pull_items.size();
  // start: r = b, x = 0, z = S r, p = z, scalars
  hipLaunchKernelGGL(kb_vec<0>, dim3(np), dim3(256), 0, s, B.d_probs, B.d_pull, B.sc, B.r, B.p, B.z);
  for (auto& c : B.schw)
    FC_HIP(launch_schwarz_class(B, c, c.d_items, (int)c.items.size(), nullptr, s));
  hipLaunchKernelGGL(kb_pull<0>, dim3(np), dim3(256), 0, s, B.d_probs, B.d_pull, np, B.sc, B.r,
                     B.p, B.q, B.z, B.partial);
  hipLaunchKernelGGL(kb_beta<0>, dim3(B.nprob), dim3(256), 0, s, B.d_probs, B.sc, B.partial, np,
                     nullptr);
  hipLaunchKernelGGL(kb_vec<2>, dim3(np), dim3(256), 0, s, B.d_probs, B.d_pull, B.sc, B.r, B.p, B.z);
  FC_HIP(hipGetLastError());
  const int chunk = o.check_every > 0 ? o.check_every : 16;
  // every problem runs at the start; the lists shrink as problems stop
  std::vector<char> running(B.nprob, 1);
  if (B.act_dofs != B.total_dofs || !B.exec || B.key_chunk != chunk) {
    FC_TRY_B(compact_lists(B, running));
    FC_TRY_B(capture_steps(B, chunk, s));
  }
  const int64_t max_chunks = (o.maxit + chunk - 1) / chunk + 1;
  // FC_BATCH_PROGRESS=k: report the number of converged members on stderr
  // every k chunks (long uneven batches otherwise run silently for minutes)
  const char* prog_env = std::getenv("FC_BATCH_PROGRESS");
  const int64_t prog = prog_env ? std::max<int64_t>(0, std::atoll(prog_env)) : 0;
  int64_t launched = 0;
  for (;;) {
    FC_HIP(hipGraphLaunch(B.exec, s));
    ++launched;
    FC_HIP(hipMemcpyAsync(B.host_sc, B.sc, B.nprob * sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    int ndone = 0;
    int64_t run_dofs = 0;
    for (int k = 0; k < B.nprob; ++k) {
      running[k] = B.host_sc[k].done == 0;
      ndone += !running[k];
      if (running[k]) run_dofs += B.host[k].n_dofs;
    }
    if (prog && launched % prog == 0) {
      std::fprintf(stderr, "[batch] %lld iterations: %d of %d members stopped\n",
                   (long long)(launched * chunk), ndone, B.nprob);
      std::fflush(stderr);
    }
    if (ndone == B.nprob || launched > max_chunks) break;
    // drop stopped problems from the launched lists once they hold 30 % of
    // the unknowns (their tiles would only return at once, but each still
    // costs a workgroup dispatch)
    if (run_dofs < 0.7 * (double)B.act_dofs) {
      FC_TRY_B(compact_lists(B, running));
      FC_TRY_B(capture_steps(B, chunk, s));
    }
  }
  FC_HIP(hipEventRecord(B.ev[2], s));
  FC_HIP(hipStreamSynchronize(s));
  FC_HIP(hipStreamWaitEvent(user, B.ev[2], 0));
  float ms = 0.f;
  FC_HIP(hipEventElapsedTime(&ms, B.ev[1], B.ev[2]));
  fc_status worst = FC_OK;
  for (int k = 0; k < B.nprob; ++k) {
    const CgScalars& h = B.host_sc[k];
    fc_status st = h.done == 1 ? FC_OK : h.done == 3 ? FC_E_BREAKDOWN : h.done == 4 ? FC_E_NAN
                                                                                  : FC_E_NOTCONV;
    if (st != FC_OK && worst == FC_OK) worst = st;
    if (infos) {
      fc_solve_info& I = infos[k];
      std::memset(&I, 0, sizeof(I));
      I.iters = h.iter;
      I.outer_iters = 1;
      I.rel_res_prec = h.zn0 > 0 ? std::sqrt(h.zz) / h.zn0 : 0.0;
      I.rel_res_true = h.rn0 > 0 ? std::sqrt(h.rr) / h.rn0 : 0.0;   // recurrence residual
      I.status = st;
      I.ms_solve = ms;
    }
  }
  return worst;
}

extern "C" void fc_batch_destroy(fc_batch bt) { destroy_batch(bt); }
