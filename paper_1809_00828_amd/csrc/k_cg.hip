// Preconditioned conjugate gradients on the device (Sec. 5, with the
// Schwarz preconditioner of Eq. 6 and the stopping test of Eq. 12).
//
// Recurrences (x_0 = 0):  r_0 = b, z_0 = S r_0, p_0 = z_0, then per step
//   q = A p;  alpha = (r,z)/(p,q);  x += alpha p;  r -= alpha q;
//   z = S r;  beta = (r,z)_new/(r,z);  p = z + beta p.
// One step is six kernels, all reading their scalars from device memory:
//   1. SpMV q = A p with per-workgroup (p,q) partials (k_spmv.hip)
//   2. one workgroup sums them in a fixed order: alpha, step count
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
#include <cmath>
#include <vector>

#include "dev_common.h"
#include "k_schwarz.h"
#include "k_spmv.h"

namespace fc {

struct SolverWs {
  int64_t n = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *t = nullptr;
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
  std::vector<hipEvent_t> tev;  // timing mode: 4 events per step of a chunk
};

void solver_ws_destroy(SolverWs* w) {
  if (!w) return;
  if (w->exec) (void)hipGraphExecDestroy(w->exec);
  if (w->graph) (void)hipGraphDestroy(w->graph);
  for (auto* p : {w->r, w->z, w->p, w->q, w->t, w->partial}) if (p) (void)hipFree(p);
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

// Pull of the Schwarz apply fused with x += alpha p, r -= alpha q and the
// reductions of the new r and z (one partial triple per workgroup; the
// grid loops over the unknowns).
__global__ __launch_bounds__(256) void k_cg_pull(
    const double* __restrict__ y, const int32_t* __restrict__ inv_ptr,
    const int32_t* __restrict__ inv_idx, const double* __restrict__ fb, int bd, int64_t n,
    double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ z, double* __restrict__ partial,
    const CgScalars* __restrict__ sc) {
  __shared__ double lds[16];
  if (sc->done) return;
  const double alpha = sc->alpha;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = i / bd;
    const int cc = (int)(i - node * bd);
    double s = 0.0;
    for (int32_t e = inv_ptr[node]; e < inv_ptr[node + 1]; ++e) s += y[(int64_t)inv_idx[e] + cc];
    const double ri = fma(-alpha, q[i], r[i]);
    x[i] = fma(alpha, p[i], x[i]);
    r[i] = ri;
    const double zi = fma(fb[i], ri, s);
    z[i] = zi;
    a = fma(ri, zi, a);
    b = fma(zi, zi, b);
    c = fma(ri, ri, c);
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  c = block_sum(c, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[gridDim.x + blockIdx.x] = b;
    partial[2 * gridDim.x + blockIdx.x] = c;
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

__global__ __launch_bounds__(256) void k_cg_p(const double* __restrict__ z, double* __restrict__ p,
                                              int64_t n, const CgScalars* sc) {
  if (sc->done) return;
  const double beta = sc->beta;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = fma(beta, p[i], z[i]);
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
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
    w->partial_len = 3 * np + 8;
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

// Enqueue `chunk` PCG steps on stream s (with timing events when tev).
static hipError_t enqueue_steps(fc_precond_s& pc, SolverWs& w, double* x, int chunk,
                                int prec, hipStream_t s, hipEvent_t* tev = nullptr) {
  fc_problem_s& pb = *pc.pb;
  const int64_t n = pb.n_dofs;
  for (int it = 0; it < chunk; ++it) {
    hipError_t e;
    if (tev && (e = hipEventRecord(tev[4 * it + 0], s)) != hipSuccess) return e;
    e = launch_spmv_pq(pb.A, false, w.p, w.q, w.sc, w.partial, s);
    if (e != hipSuccess) return e;
    if (tev && (e = hipEventRecord(tev[4 * it + 1], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, s, w.partial, spmv_num_blocks(pb.A),
                       w.sc);
    if (tev && (e = hipEventRecord(tev[4 * it + 2], s)) != hipSuccess) return e;
    e = launch_schwarz_phase1(pc, prec, w.r, w.q, w.sc, s);
    if (e != hipSuccess) return e;
    if (tev && (e = hipEventRecord(tev[4 * it + 3], s)) != hipSuccess) return e;
    const unsigned pg = pull_grid(n);
    hipLaunchKernelGGL(k_cg_pull, dim3(pg), dim3(kVecThreads), 0, s, pc.y, pc.inv_ptr,
                       pc.inv_idx, pc.fallback, pc.bdim, n, x, w.r, w.p, w.q, w.z, w.partial,
                       w.sc);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(1024), 0, s, w.partial, (int)pg, w.sc);
    hipLaunchKernelGGL(k_cg_p, dim3(nblk(n)), dim3(kVecThreads), 0, s, w.z, w.p, n, w.sc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

fc_status pcg_solve_f64(fc_precond_s& pc, const double* b, double* x, const fc_solve_opts& o,
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

  CgScalars init{};
  init.tol = o.tol;
  init.maxit = o.maxit;
  init.stop = o.stop;
  init.history = o.history_dev;
  FC_HIP(hipMemcpyAsync(w.sc, &init, sizeof(CgScalars), hipMemcpyHostToDevice, s));
  FC_HIP(hipEventRecord(w.ev[1], s));
  // x = 0, r = b, z = S r, p = z
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, x, 0.0, n);
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, b, w.r, n);
  FC_HIP(hipGetLastError());
  FC_HIP(launch_schwarz_apply(pc, w.r, w.z, s));
  hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, s, w.z, w.p, n);
  hipLaunchKernelGGL(k_cg_start, dim3(kRedBlocks), dim3(256), 0, s, w.r, w.z, n, w.partial,
                     w.sc);
  FC_HIP(hipGetLastError());

  const int chunk = o.check_every > 0 ? o.check_every : 16;
  const int prec = 0;
  double t_spmv = 0.0, t_schw = 0.0;
  int64_t n_timed = 0;
  if (o.timing) {
    // direct launches with events around the two streaming kernels
    if ((int)w.tev.size() < 4 * chunk) {
      size_t old = w.tev.size();
      w.tev.resize(4 * chunk, nullptr);
      for (size_t i = old; i < w.tev.size(); ++i) FC_HIP(hipEventCreate(&w.tev[i]));
    }
    int64_t iter_before = 0, launched = 0;
    const int64_t max_chunks = (o.maxit + chunk - 1) / chunk + 1;
    for (;;) {
      FC_HIP(enqueue_steps(pc, w, x, chunk, prec, s, w.tev.data()));
      ++launched;
      FC_HIP(hipMemcpyAsync(w.host, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
      FC_HIP(hipStreamSynchronize(s));
      const int64_t ran = std::min<int64_t>(chunk, w.host->iter - iter_before);
      iter_before = w.host->iter;
      for (int64_t it = 0; it < ran; ++it) {
        float a = 0.f, b = 0.f;
        FC_HIP(hipEventElapsedTime(&a, w.tev[4 * it + 0], w.tev[4 * it + 1]));
        FC_HIP(hipEventElapsedTime(&b, w.tev[4 * it + 2], w.tev[4 * it + 3]));
        t_spmv += a;
        t_schw += b;
      }
      n_timed += ran;
      if (w.host->done != 0 || launched > max_chunks) break;
    }
  } else {
    // (re)capture the chunk when the buffers or the chunk length change
    if (!w.exec || w.key[0] != x || w.key_chunk != chunk || w.key_prec != prec) {
      if (w.exec) {
        FC_HIP(hipGraphExecDestroy(w.exec));
        w.exec = nullptr;
      }
      if (w.graph) {
        FC_HIP(hipGraphDestroy(w.graph));
        w.graph = nullptr;
      }
      FC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_steps(pc, w, x, chunk, prec, s);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(s, &g);
      if (e != hipSuccess) FC_HIP(e);
      FC_HIP(e2);
      w.graph = g;
      FC_HIP(hipGraphInstantiate(&w.exec, g, nullptr, nullptr, 0));
      w.key[0] = x;
      w.key_chunk = chunk;
      w.key_prec = prec;
    }
    int64_t launched = 0;
    const int64_t max_chunks = (o.maxit + chunk - 1) / chunk + 1;
    for (;;) {
      FC_HIP(hipGraphLaunch(w.exec, s));
      ++launched;
      FC_HIP(hipMemcpyAsync(w.host, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
      FC_HIP(hipStreamSynchronize(s));
      if (w.host->done != 0 || launched > max_chunks) break;
    }
  }
  FC_HIP(hipEventRecord(w.ev[2], s));
  // true residual ||b - A x|| / ||b||
  FC_HIP(launch_spmv(pb.A, x, w.t, s));
  double* out2 = w.partial + w.partial_len - 2;
  hipLaunchKernelGGL(k_resid, dim3(kRedBlocks), dim3(256), 0, s, b, w.t, n, w.partial, w.sc,
                     out2);
  FC_HIP(hipGetLastError());
  double res[2] = {0, 0};
  FC_HIP(hipMemcpyAsync(res, out2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  FC_HIP(hipMemcpyAsync(w.host, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
  FC_HIP(hipEventRecord(w.ev[3], s));
  FC_HIP(hipStreamSynchronize(s));
  FC_HIP(hipStreamWaitEvent(user, w.ev[3], 0));
  float ms = 0.f;
  FC_HIP(hipEventElapsedTime(&ms, w.ev[1], w.ev[2]));
  const CgScalars& h = *w.host;
  fc_status result = FC_OK;
  switch (h.done) {
    case 1: result = FC_OK; break;
    case 2: result = FC_E_NOTCONV; break;
    case 3: result = FC_E_BREAKDOWN; break;
    case 4: result = FC_E_NAN; break;
    default: result = FC_E_NOTCONV; break;
  }
  if (info) {
    info->iters = h.iter;
    info->outer_iters = 1;
    info->rel_res_true = res[1] > 0 ? std::sqrt(res[0] / res[1]) : 0.0;
    info->rel_res_prec = h.zn0 > 0 ? std::sqrt(h.zz) / h.zn0 : 0.0;
    info->status = result;
    info->ms_solve = ms;
    info->ms_spmv = t_spmv;
    info->ms_schwarz = t_schw;
    info->n_timed = n_timed;
  }
  return result;
}

}  // namespace fc
