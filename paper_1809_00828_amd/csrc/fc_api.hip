// C ABI of libfc (declared in include/fc.h): handle management, uploads,
// the preconditioner build of Algorithm 1 and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "fc_internal.h"
#include "host_assemble.h"
#include "k_schwarz.h"
#include "k_setup.h"

struct fc_host_system_s {
  fc::HostSystem sys;
};

namespace fc {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

fc_status pcg_solve(fc_precond_s& pc, const double* b, double* x, const fc_solve_opts& o,
                    fc_solve_info* info, hipStream_t user);
fc_status pcg_solve_noalloc(fc_precond_s& pc, const double* b, double* x,
                            const fc_solve_opts& o, fc_solve_info* info, hipStream_t s);

template <class T>
static fc_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return FC_OK;
  hipError_t e = hipMalloc(p, count * sizeof(T));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
              " bytes failed: " + hipGetErrorString(e));
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? FC_E_NOMEM : FC_E_DEVICE;
  }
  return FC_OK;
}

template <class T>
static fc_status upload(T** p, const T* src, size_t count) {
  fc_status st = dev_alloc(p, count);
  if (st != FC_OK || count == 0) return st;
  FC_HIP(hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice));
  return FC_OK;
}

#define FC_TRY(x)                  \
  do {                             \
    fc_status s_ = (x);            \
    if (s_ != FC_OK) return s_;    \
  } while (0)

static void free_problem(fc_problem_s* pb) {
  if (!pb) return;
  for (void* p : {(void*)pb->A.rowptr, (void*)pb->A.col, (void*)pb->A.val, (void*)pb->A.val32,
                  (void*)pb->A.rows_hi, (void*)pb->A.rows_lo, (void*)pb->A.sell_val,
                  (void*)pb->A.sell_off, (void*)pb->A.sell_rest, (void*)pb->rhs,
                  (void*)pb->elem_nodes, (void*)pb->diag})
    if (p) (void)hipFree(p);
  delete pb;
}

static void free_precond(fc_precond_s* pc) {
  if (!pc) return;
  solver_ws_destroy(pc->ws);
  coarse_destroy(pc->coarse);
  for (void* p : {(void*)pc->block_elem, (void*)pc->bnodes, (void*)pc->P, (void*)pc->Q,
                  (void*)pc->Q32,
                  (void*)pc->unsafe32, (void*)pc->unsafe_flag32, (void*)pc->Lbf, (void*)pc->isd,
                  (void*)pc->inv_ptr, (void*)pc->inv_idx, (void*)pc->fallback, (void*)pc->y})
    if (p) (void)hipFree(p);
  delete pc;
}

static fc_status upload_system_body(const HostSystem& S, hipStream_t stream, fc_problem* out) {
  std::unique_ptr<fc_problem_s, void (*)(fc_problem_s*)> pb(new (std::nothrow) fc_problem_s(),
                                                           free_problem);
  if (!pb) return FC_E_NOMEM;
  FC_HIP(hipGetDevice(&pb->device));
  pb->dim = S.dim;
  pb->p = S.p;
  pb->n = S.n;
  pb->bdim = S.bdim;
  pb->nn = S.nn;
  pb->m = S.m;
  pb->n_nodes = S.n_nodes;
  pb->n_dofs = S.n_dofs;
  pb->n_el = S.n_el;
  pb->A.bdim = S.bdim;
  pb->A.n_rows = S.n_nodes;
  pb->A.nnzb = S.rowptr.back();
  int32_t mr = 0;
  for (int64_t i = 0; i < S.n_nodes; ++i) mr = std::max(mr, S.rowptr[i + 1] - S.rowptr[i]);
  pb->A.max_row = mr;
  FC_TRY(upload(&pb->A.rowptr, S.rowptr.data(), S.rowptr.size()));
  FC_TRY(upload(&pb->A.col, S.col.data(), S.col.size()));
  FC_TRY(upload(&pb->A.val, S.val.data(), S.val.size()));
  FC_TRY(upload(&pb->rhs, S.rhs.data(), S.rhs.size()));
  FC_TRY(upload(&pb->elem_nodes, S.elem_nodes.data(), S.elem_nodes.size()));
  FC_TRY(dev_alloc(&pb->diag, (size_t)S.n_dofs));
  pb->eta = S.eta;
  pb->elem_nodes_host = S.elem_nodes;
  FC_HIP(launch_diag(*pb, stream));
  if (S.dim > 0) FC_HIP(spmv_enable_lattice(pb->A, S.dim, S.p * S.n + 1, S.p, stream));
  pb->A.group = spmv_group_for(pb->A);
  FC_HIP(hipStreamSynchronize(stream));
  *out = pb.release();
  return FC_OK;
}

// Host containers of the set-up can run out of memory: report it instead
// of letting the exception cross the C boundary.
static fc_status upload_system(const HostSystem& S, hipStream_t stream, fc_problem* out) {
  try {
    return upload_system_body(S, stream, out);
  } catch (const std::bad_alloc&) {
    set_error("set-up: out of host memory");
    return FC_E_NOMEM;
  }
}

}  // namespace fc

using namespace fc;

extern "C" {

const char* fc_last_error(void) { return g_err.c_str(); }

fc_status fc_assemble(const fc_problem_desc* desc, fc_host_system* out) {
  if (!desc || !out) {
    set_error("fc_assemble: NULL argument");
    return FC_E_ARG;
  }
  *out = nullptr;
  std::unique_ptr<fc_host_system_s> hs(new (std::nothrow) fc_host_system_s());
  if (!hs) return FC_E_NOMEM;
  std::string err;
  fc_status st;
  try {
    st = assemble_host(*desc, &hs->sys, &err);
  } catch (const std::bad_alloc&) {
    set_error("fc_assemble: host allocation failed");
    return FC_E_NOMEM;
  }
  if (st != FC_OK) {
    set_error("fc_assemble: " + err);
    return st;
  }
  *out = hs.release();
  return FC_OK;
}

fc_status fc_host_system_info(fc_host_system hs, int64_t* n_dofs, int64_t* nnzb, int64_t* n_el,
                              int32_t* m, int32_t* bsr_dim) {
  if (!hs) return FC_E_ARG;
  const HostSystem& S = hs->sys;
  if (n_dofs) *n_dofs = S.n_dofs;
  if (nnzb) *nnzb = S.rowptr.empty() ? 0 : S.rowptr.back();
  if (n_el) *n_el = S.n_el;
  if (m) *m = S.m;
  if (bsr_dim) *bsr_dim = S.bdim;
  return FC_OK;
}

static void soa_to_rowmajor(const std::vector<int32_t>& rp, const double* soa, int bd,
                            int64_t n_rows, double* out) {
  const int bb = bd * bd;
  for (int64_t i = 0; i < n_rows; ++i) {
    const int64_t L = rp[i + 1] - rp[i];
    for (int64_t k = 0; k < L; ++k)
      for (int e = 0; e < bb; ++e)
        out[((int64_t)rp[i] + k) * bb + e] = soa[(int64_t)rp[i] * bb + e * L + k];
  }
}

static void elem_dofs_from_nodes(const int32_t* en, int64_t n_el, int nn, int bd, int32_t* out) {
  for (int64_t e = 0; e < n_el; ++e)
    for (int a = 0; a < nn; ++a)
      for (int c = 0; c < bd; ++c)
        out[(e * nn + a) * bd + c] = en[e * nn + a] * bd + c;
}

fc_status fc_host_system_export(fc_host_system hs, int32_t* rowptr, int32_t* col, double* val,
                                double* rhs, int32_t* elem_dofs, double* eta) {
  if (!hs) return FC_E_ARG;
  const HostSystem& S = hs->sys;
  if (rowptr) std::memcpy(rowptr, S.rowptr.data(), S.rowptr.size() * sizeof(int32_t));
  if (col) std::memcpy(col, S.col.data(), S.col.size() * sizeof(int32_t));
  if (val) soa_to_rowmajor(S.rowptr, S.val.data(), S.bdim, S.n_nodes, val);
  if (rhs) std::memcpy(rhs, S.rhs.data(), S.rhs.size() * sizeof(double));
  if (elem_dofs) elem_dofs_from_nodes(S.elem_nodes.data(), S.n_el, S.nn, S.bdim, elem_dofs);
  if (eta) std::memcpy(eta, S.eta.data(), S.eta.size() * sizeof(double));
  return FC_OK;
}

void fc_host_system_destroy(fc_host_system hs) { delete hs; }

fc_status fc_setup_from_host(fc_host_system hs, void* stream, fc_problem* out) {
  if (!hs || !out) {
    set_error("fc_setup_from_host: NULL argument");
    return FC_E_ARG;
  }
  *out = nullptr;
  return upload_system(hs->sys, (hipStream_t)stream, out);
}

fc_status fc_setup(const fc_problem_desc* desc, void* stream, fc_problem* out) {
  fc_host_system hs = nullptr;
  fc_status st = fc_assemble(desc, &hs);
  if (st != FC_OK) return st;
  st = fc_setup_from_host(hs, stream, out);
  fc_host_system_destroy(hs);
  return st;
}

fc_status fc_setup_from_matrix(int64_t n, int32_t bsr_dim, const int32_t* rowptr,
                               const int32_t* col, const double* val, const double* rhs,
                               int64_t n_el, int32_t m, const int32_t* elem_dofs,
                               const double* eta, void* stream, fc_problem* out) {
  if (!out || !rowptr || !col || !val || !rhs || (n_el > 0 && (!elem_dofs || !eta)) ||
      bsr_dim < 1 || bsr_dim > 3 || n <= 0 || n % bsr_dim || m <= 0 || m % bsr_dim ||
      n >= (int64_t(1) << 31)) {
    set_error("fc_setup_from_matrix: invalid arguments");
    return FC_E_ARG;
  }
  *out = nullptr;
  HostSystem S;
  S.bdim = bsr_dim;
  S.n_nodes = n / bsr_dim;
  S.n_dofs = n;
  S.n_el = n_el;
  S.m = m;
  S.nn = m / bsr_dim;
  const int bb = bsr_dim * bsr_dim;
  S.rowptr.assign(rowptr, rowptr + S.n_nodes + 1);
  if (S.rowptr[0] != 0) {
    set_error("fc_setup_from_matrix: rowptr[0] must be 0");
    return FC_E_ARG;
  }
  for (int64_t i = 0; i < S.n_nodes; ++i)
    if (S.rowptr[i + 1] < S.rowptr[i]) {
      set_error("fc_setup_from_matrix: rowptr not monotone");
      return FC_E_ARG;
    }
  const int64_t nnzb = S.rowptr.back();
  S.col.assign(col, col + nnzb);
  for (int64_t i = 0; i < S.n_nodes; ++i)
    for (int32_t k = S.rowptr[i]; k < S.rowptr[i + 1]; ++k)
      if (S.col[k] < 0 || S.col[k] >= S.n_nodes || (k > S.rowptr[i] && S.col[k] <= S.col[k - 1])) {
        set_error("fc_setup_from_matrix: column indices out of range or not sorted");
        return FC_E_ARG;
      }
  S.val.resize((size_t)nnzb * bb);
  for (int64_t i = 0; i < S.n_nodes; ++i) {
    const int64_t L = S.rowptr[i + 1] - S.rowptr[i];
    for (int64_t k = 0; k < L; ++k)
      for (int e = 0; e < bb; ++e)
        S.val[(int64_t)S.rowptr[i] * bb + e * L + k] = val[((int64_t)S.rowptr[i] + k) * bb + e];
  }
  S.rhs.assign(rhs, rhs + n);
  S.elem_nodes.resize((size_t)n_el * S.nn);
  for (int64_t e = 0; e < n_el; ++e)
    for (int a = 0; a < S.nn; ++a) {
      const int32_t d0 = elem_dofs[e * m + a * bsr_dim];
      if (d0 < 0 || d0 >= n || d0 % bsr_dim) {
        set_error("fc_setup_from_matrix: element unknowns must be bsr_dim*node + c");
        return FC_E_ARG;
      }
      for (int c = 1; c < bsr_dim; ++c)
        if (elem_dofs[e * m + a * bsr_dim + c] != d0 + c) {
          set_error("fc_setup_from_matrix: element unknowns must be bsr_dim*node + c");
          return FC_E_ARG;
        }
      S.elem_nodes[e * S.nn + a] = d0 / bsr_dim;
    }
  S.eta.assign(eta, eta + n_el);
  return upload_system(S, (hipStream_t)stream, out);
}

fc_status fc_problem_info(fc_problem pb, int64_t* n_dofs, int64_t* nnzb, int64_t* n_el, int32_t* m,
                          int32_t* bsr_dim) {
  if (!pb) return FC_E_ARG;
  if (n_dofs) *n_dofs = pb->n_dofs;
  if (nnzb) *nnzb = pb->A.nnzb;
  if (n_el) *n_el = pb->n_el;
  if (m) *m = pb->m;
  if (bsr_dim) *bsr_dim = pb->bdim;
  return FC_OK;
}

fc_status fc_get_rhs(fc_problem pb, double* b_dev, void* stream) {
  if (!pb || !b_dev) return FC_E_ARG;
  FC_HIP(hipMemcpyAsync(b_dev, pb->rhs, pb->n_dofs * sizeof(double), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return FC_OK;
}

fc_status fc_get_eta(fc_problem pb, double* eta_host) {
  if (!pb || !eta_host) return FC_E_ARG;
  std::memcpy(eta_host, pb->eta.data(), pb->eta.size() * sizeof(double));
  return FC_OK;
}

fc_status fc_export(fc_problem pb, int32_t* rowptr, int32_t* col, double* val, int32_t* elem_dofs) {
  if (!pb) return FC_E_ARG;
  std::vector<int32_t> rp(pb->A.n_rows + 1);
  FC_HIP(hipMemcpy(rp.data(), pb->A.rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (rowptr) std::memcpy(rowptr, rp.data(), rp.size() * sizeof(int32_t));
  if (col) FC_HIP(hipMemcpy(col, pb->A.col, pb->A.nnzb * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (val) {
    const int bb = pb->bdim * pb->bdim;
    std::vector<double> soa((size_t)pb->A.nnzb * bb);
    FC_HIP(hipMemcpy(soa.data(), pb->A.val, soa.size() * sizeof(double), hipMemcpyDeviceToHost));
    soa_to_rowmajor(rp, soa.data(), pb->bdim, pb->A.n_rows, val);
  }
  if (elem_dofs)
    elem_dofs_from_nodes(pb->elem_nodes_host.data(), pb->n_el, pb->nn, pb->bdim, elem_dofs);
  return FC_OK;
}

fc_status fc_apply_A(fc_problem pb, const double* x_dev, double* y_dev, void* stream) {
  if (!pb || !x_dev || !y_dev || x_dev == y_dev) {
    set_error("fc_apply_A: invalid arguments");
    return FC_E_ARG;
  }
  FC_HIP(launch_spmv(pb->A, x_dev, y_dev, (hipStream_t)stream));
  return FC_OK;
}

static fc_status precond_build_body(fc_problem pb, const fc_precond_opts* opts, void* stream,
                                    fc_precond* out) {
  if (!pb || !out) {
    set_error("fc_precond_build: NULL argument");
    return FC_E_ARG;
  }
  *out = nullptr;
  fc_precond_opts o{1.0, 1e-13, 1, FC_STORE_F64, FC_BLOCK_ELEMENT};
  if (opts) o = *opts;
  if (!(o.eps >= 0.0) || !(o.eta_bar == o.eta_bar) ||
      (o.block_kind != FC_BLOCK_ELEMENT && o.block_kind != FC_BLOCK_VERTEX_PATCH)) {
    set_error("fc_precond_build: invalid options");
    return FC_E_ARG;
  }
  const bool patch = o.block_kind == FC_BLOCK_VERTEX_PATCH;
  int pm = pb->m, pnn = pb->nn;
  if (patch) {
    if (pb->dim < 1 || pb->n < 1 || pb->p < 1) {
      set_error("fc_precond_build: vertex patches need a problem set up from a description");
      return FC_E_UNSUPPORTED;
    }
    if (o.store_mask & (FC_STORE_F32 | FC_STORE_BF16)) {
      set_error("fc_precond_build: vertex patches are built in FP64 only");
      return FC_E_UNSUPPORTED;
    }
    pnn = 1;
    for (int k = 0; k < pb->dim; ++k) pnn *= 2 * pb->p + 1;
    pm = pnn * pb->bdim;
  }
  if (pm > 192) {
    set_error(std::string("fc_precond_build: ") + (patch ? "vertex patches" : "element blocks") +
              " above 192 unknowns are not supported");
    return FC_E_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<fc_precond_s, void (*)(fc_precond_s*)> pc(new (std::nothrow) fc_precond_s(),
                                                           free_precond);
  if (!pc) return FC_E_NOMEM;
  pc->pb = pb;
  pc->m = pm;
  pc->nn = pnn;
  pc->bdim = pb->bdim;
  pc->eps = o.eps;
  pc->stabilize = o.stabilize ? 1 : 0;
  pc->block_kind = o.block_kind;
  const int m = pc->m, nn = pc->nn, bd = pc->bdim;

  // blocks: elements with eta_T <= eta_bar (Sec. 3.2), element order; or
  // the vertex patches with a cell of eta_T <= eta_bar, vertex order (first
  // direction fastest), each listing the nodes of its box in lattice order
  // and padded with -1
  std::vector<int32_t> blocks, pnodes, pad;
  if (!patch) {
    for (int64_t e = 0; e < pb->n_el; ++e)
      if (pb->eta[e] <= o.eta_bar) blocks.push_back((int32_t)e);
  } else {
    const int d = pb->dim, n = pb->n, p = pb->p, n1 = p * n + 1;
    int64_t nv = 1;
    for (int k = 0; k < d; ++k) nv *= n + 1;
    for (int64_t v = 0; v < nv; ++v) {
      int vc[3] = {0, 0, 0}, clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
      int64_t t = v;
      for (int k = 0; k < d; ++k) {
        vc[k] = (int)(t % (n + 1));
        t /= n + 1;
        clo[k] = std::max(0, vc[k] - 1);
        chi[k] = std::min(n - 1, vc[k]);
      }
      double emin = 2.0;
      for (int cz = clo[2]; cz <= chi[2]; ++cz)
        for (int cy = clo[1]; cy <= chi[1]; ++cy)
          for (int cx = clo[0]; cx <= chi[0]; ++cx)
            emin = std::min(emin, pb->eta[cx + (int64_t)n * (cy + (int64_t)n * cz)]);
      if (!(emin <= o.eta_bar)) continue;
      int glo[3] = {0, 0, 0}, ghi[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) {
        glo[k] = std::max(0, p * vc[k] - p);
        ghi[k] = std::min(n1 - 1, p * vc[k] + p);
      }
      const size_t start = pnodes.size();
      for (int gz = glo[2]; gz <= ghi[2]; ++gz)
        for (int gy = glo[1]; gy <= ghi[1]; ++gy)
          for (int gx = glo[0]; gx <= ghi[0]; ++gx)
            pnodes.push_back((int32_t)(gx + (int64_t)n1 * (gy + (int64_t)n1 * gz)));
      const int used = (int)(pnodes.size() - start);
      pad.push_back(nn - used);
      pnodes.resize(start + nn, -1);
      blocks.push_back((int32_t)(blocks.size()));
    }
  }
  const std::vector<int32_t>& bn = patch ? pnodes : pb->elem_nodes_host;
  pc->n_blocks = (int64_t)blocks.size();
  const int64_t nb = pc->n_blocks;
  if (nb * (int64_t)m >= (int64_t(1) << 31)) {
    set_error("fc_precond_build: too many block entries for int32 indices");
    return FC_E_UNSUPPORTED;
  }
  // node -> (block, local node) map, blocks in increasing order
  std::vector<int32_t> ptr(pb->n_nodes + 1, 0), idx((size_t)nb * nn);
  int64_t n_entries = 0;
  for (int64_t k = 0; k < nb; ++k)
    for (int a = 0; a < nn; ++a) {
      const int32_t node = bn[(int64_t)blocks[k] * nn + a];
      if (node >= 0) {
        ptr[node + 1]++;
        ++n_entries;
      }
    }
  for (int64_t i = 0; i < pb->n_nodes; ++i) ptr[i + 1] += ptr[i];
  idx.resize((size_t)n_entries);
  {
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t k = 0; k < nb; ++k)
      for (int a = 0; a < nn; ++a) {
        const int32_t node = bn[(int64_t)blocks[k] * nn + a];
        if (node >= 0) idx[fill[node]++] = (int32_t)(k * m + a * bd);
      }
  }
  if (patch) FC_TRY(upload(&pc->bnodes, pnodes.data(), pnodes.size()));
  FC_TRY(upload(&pc->block_elem, blocks.data(), blocks.size()));
  FC_TRY(upload(&pc->inv_ptr, ptr.data(), ptr.size()));
  FC_TRY(upload(&pc->inv_idx, idx.data(), idx.size()));
  FC_TRY(dev_alloc(&pc->P, (size_t)nb * m * m));
  FC_TRY(dev_alloc(&pc->y, (size_t)nb * m));
  FC_TRY(dev_alloc(&pc->fallback, (size_t)pb->n_dofs));

  int32_t* d_flag = nullptr;
  int32_t* d_drop = nullptr;
  unsigned long long* d_count = nullptr;
  struct Tmp {
    void* p[3] = {nullptr, nullptr, nullptr};
    ~Tmp() {
      for (void* q : p)
        if (q) (void)hipFree(q);
    }
  } tmp;
  FC_TRY(dev_alloc(&d_flag, (size_t)std::max<int64_t>(nb, 1)));
  tmp.p[0] = d_flag;
  FC_TRY(dev_alloc(&d_drop, (size_t)std::max<int64_t>(nb, 1)));
  tmp.p[1] = d_drop;
  FC_TRY(dev_alloc(&d_count, 1));
  tmp.p[2] = d_count;
  FC_HIP(hipMemsetAsync(d_drop, 0, std::max<int64_t>(nb, 1) * sizeof(int32_t), s));
  FC_HIP(hipMemsetAsync(d_count, 0, sizeof(unsigned long long), s));

  if (nb > 0) {
    FC_HIP(launch_block_extract(*pb, *pc, s));
    if (m <= 64 && !pc->stabilize) {
      // the plain inverse (S*): every block by the eigen-decomposition with
      // every nonzero eigenvalue inverted; in LDS when it fits
      const int64_t chunk = jacobi_needs_work(m) ? 16384 : nb;
      double* work = nullptr;
      if (jacobi_needs_work(m)) FC_TRY(dev_alloc(&work, (size_t)std::min(chunk, nb) * 2 * m * m));
      std::vector<int32_t> all(nb);
      for (int64_t k = 0; k < nb; ++k) all[k] = (int32_t)k;
      int32_t* d_all = nullptr;
      fc_status st = upload(&d_all, all.data(), all.size());
      hipError_t e = hipSuccess;
      for (int64_t s0 = 0; st == FC_OK && s0 < nb && e == hipSuccess; s0 += chunk)
        e = launch_jacobi(*pc, d_all + s0, std::min(chunk, nb - s0), work, d_drop, s);
      hipError_t e2 = hipStreamSynchronize(s);
      if (d_all) (void)hipFree(d_all);
      if (work) (void)hipFree(work);
      FC_TRY(st);
      FC_HIP(e);
      FC_HIP(e2);
      pc->n_eig = nb;
    } else {
      // certified direct inverses; the blocks whose certificate fails (some
      // eigenvalue may be near the threshold of Eq. 11) keep A_B and are
      // eigen-decomposed below
      if (m <= 64)
        FC_HIP(launch_sweep_small(*pc, d_flag, s));
      else
        FC_HIP(launch_sweep(*pc, d_flag, s));
      std::vector<int32_t> flag(nb);
      FC_HIP(hipMemcpyAsync(flag.data(), d_flag, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      FC_HIP(hipStreamSynchronize(s));
      std::vector<int32_t> sel;
      for (int64_t k = 0; k < nb; ++k)
        if (flag[k]) sel.push_back((int32_t)k);
      pc->n_eig = (int64_t)sel.size();
      if (!sel.empty()) {
        // blocks whose certificate failed still hold A_B: eigen-decompose
        const int64_t chunk = 2048;
        int32_t* d_sel = nullptr;
        double* work = nullptr;
        FC_TRY(upload(&d_sel, sel.data(), sel.size()));
        fc_status st = dev_alloc(&work, (size_t)std::min<int64_t>(chunk, sel.size()) * 2 * m * m);
        if (st != FC_OK) {
          (void)hipFree(d_sel);
          return st;
        }
        hipError_t e = hipSuccess;
        for (int64_t s0 = 0; s0 < (int64_t)sel.size() && e == hipSuccess; s0 += chunk) {
          const int64_t cnt = std::min<int64_t>(chunk, sel.size() - s0);
          e = launch_jacobi(*pc, d_sel + s0, cnt, work, d_drop, s);
        }
        hipError_t e2 = hipStreamSynchronize(s);
        (void)hipFree(d_sel);
        (void)hipFree(work);
        FC_HIP(e);
        FC_HIP(e2);
      }
    }
  }
  FC_HIP(launch_fallback(*pb, *pc, d_count, s));
  // wrapped-diagonal symmetric copies streamed by the block products
  const size_t qn = (size_t)nb * sym_block_stride(m);
  FC_TRY(dev_alloc(&pc->Q, qn));
  FC_HIP(launch_pack_sym(*pc, pc->Q, 0, s));
  if (o.store_mask & (FC_STORE_F32 | FC_STORE_BF16)) {
    FC_TRY(dev_alloc(&pc->isd, (size_t)pb->n_dofs));
    FC_HIP(launch_inv_sqrt_diag(*pb, pc->isd, s));
  }
  // FP32: the rounded, diagonally scaled inverse D^1/2 P_B D^1/2 in
  // wrapped-diagonal storage; scaling removes most of a cut block's ill
  // conditioning, so the rounding keeps it positive definite.  Blocks where
  // a Cholesky factorisation of the rounded matrix shows otherwise are
  // listed and applied from the FP64 copy.
  if (o.store_mask & FC_STORE_F32) {
    FC_TRY(dev_alloc(&pc->Q32, qn));
    FC_HIP(launch_pack_sym(*pc, pc->Q32, 1, s));
    FC_TRY(dev_alloc(&pc->unsafe_flag32, (size_t)std::max<int64_t>(nb, 1)));
    FC_HIP(launch_chol_pack(*pc, s, pc->unsafe_flag32));
    std::vector<int32_t> hf(std::max<int64_t>(nb, 1), 0);
    FC_HIP(hipMemcpyAsync(hf.data(), pc->unsafe_flag32, nb * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> list;
    for (int64_t k = 0; k < nb; ++k)
      if (hf[k]) list.push_back((int32_t)k);
    pc->n_unsafe32 = (int64_t)list.size();
    if (!list.empty()) FC_TRY(upload(&pc->unsafe32, list.data(), list.size()));
  }
  // BF16: scaled Cholesky factors (positive semi-definite however rounded)
  const size_t ln = (size_t)nb * ((size_t)m * (m + 1) / 2);
  if (o.store_mask & FC_STORE_BF16) FC_TRY(dev_alloc(&pc->Lbf, ln));
  if (pc->Lbf) FC_HIP(launch_chol_pack(*pc, s));
  unsigned long long cnt = 0;
  std::vector<int32_t> drop(std::max<int64_t>(nb, 1));
  FC_HIP(hipMemcpyAsync(&cnt, d_count, sizeof(cnt), hipMemcpyDeviceToHost, s));
  FC_HIP(hipMemcpyAsync(drop.data(), d_drop, drop.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FC_HIP(hipStreamSynchronize(s));
  pc->n_fallback = (int64_t)cnt;
  // scalar lattice problem with every cell a block, in cell order (checked
  // row by row on the device): the block products find a row's unknown and
  // the pull a node's blocks from lattice indices (FC_PULL_LATTICE=0 keeps
  // the node lists and the node-to-block map).  With three components per
  // node the mapped pull is faster (46 against 57 us at 32^3 cells, p = 3),
  // so it stays there.
  {
    const char* env = std::getenv("FC_PULL_LATTICE");
    const bool allowed = !(env && std::atoi(env) == 0);
    if (allowed && !patch && pb->bdim == 1 && pb->dim >= 2 && pb->dim <= 3 && pb->n > 0 &&
        pb->p > 0 && nb == pb->n_el &&
        nb == std::pow((double)pb->n, pb->dim) && pb->nn == (int)std::pow(pb->p + 1.0, pb->dim)) {
      const PullLattice L = make_pull_lattice(pb->dim, pb->n, pb->p);
      bool ok = false;
      FC_HIP(schwarz_check_lattice(*pc, L, &ok, s));
      if (ok) pc->lat = L;
    }
  }
  int64_t nd = 0;
  for (int64_t k = 0; k < nb; ++k) nd += drop[k];
  pc->n_dropped = nd;
  drop.resize((size_t)nb);
  // the zero rows and columns padding a boundary patch give exactly zero
  // eigenvalues, which the threshold drops; they are not counted
  if (patch) {
    nd = 0;
    for (int64_t k = 0; k < nb; ++k) {
      drop[k] -= pad[k] * bd;
      nd += drop[k];
    }
    pc->n_dropped = nd;
  }
  pc->dropped.swap(drop);
  *out = pc.release();
  return FC_OK;
}

fc_status fc_spmv_info(fc_problem pb, int32_t* group, int32_t* lattice) {
  if (!pb) return FC_E_ARG;
  if (group) *group = pb->A.group;
  if (lattice) *lattice = pb->A.lat.dim > 0 ? (pb->A.sell_val ? 2 : 1) : 0;
  return FC_OK;
}

fc_status fc_precond_lowprec_info(fc_precond pc, int64_t* n_f32_blocks,
                                  int64_t* n_f32_from_f64) {
  if (!pc) return FC_E_ARG;
  if (n_f32_blocks) *n_f32_blocks = pc->Q32 ? pc->n_blocks - pc->n_unsafe32 : 0;
  if (n_f32_from_f64) *n_f32_from_f64 = pc->Q32 ? pc->n_unsafe32 : 0;
  return FC_OK;
}

fc_status fc_precond_info(fc_precond pc, int64_t* n_blocks, int64_t* n_fallback,
                          int64_t* n_eig_blocks, int64_t* n_dropped) {
  if (!pc) return FC_E_ARG;
  if (n_blocks) *n_blocks = pc->n_blocks;
  if (n_fallback) *n_fallback = pc->n_fallback;
  if (n_eig_blocks) *n_eig_blocks = pc->n_eig;
  if (n_dropped) *n_dropped = pc->n_dropped;
  return FC_OK;
}

fc_status fc_precond_shape(fc_precond pc, int32_t* m, int32_t* block_kind) {
  if (!pc) return FC_E_ARG;
  if (m) *m = pc->m;
  if (block_kind) *block_kind = pc->block_kind;
  return FC_OK;
}

fc_status fc_precond_block_dropped(fc_precond pc, int32_t* dropped_host) {
  if (!pc || (!dropped_host && pc->n_blocks > 0)) {
    set_error("fc_precond_block_dropped: invalid arguments");
    return FC_E_ARG;
  }
  if (pc->n_blocks > 0)
    std::memcpy(dropped_host, pc->dropped.data(), pc->dropped.size() * sizeof(int32_t));
  return FC_OK;
}

fc_status fc_get_block_inverse(fc_precond pc, int64_t k, double* out_host) {
  if (!pc || !out_host || k < 0 || k >= pc->n_blocks) {
    set_error("fc_get_block_inverse: invalid arguments");
    return FC_E_ARG;
  }
  const size_t mm = (size_t)pc->m * pc->m;
  FC_HIP(hipMemcpy(out_host, pc->P + k * mm, mm * sizeof(double), hipMemcpyDeviceToHost));
  return FC_OK;
}

fc_status fc_apply_M(fc_precond pc, const double* r_dev, double* z_dev, void* stream) {
  if (!pc || !r_dev || !z_dev || r_dev == z_dev) {
    set_error("fc_apply_M: invalid arguments");
    return FC_E_ARG;
  }
  FC_HIP(launch_schwarz_apply(*pc, r_dev, z_dev, (hipStream_t)stream));
  return FC_OK;
}

fc_status fc_precond_build(fc_problem pb, const fc_precond_opts* opts, void* stream,
                           fc_precond* out) {
  try {
    return precond_build_body(pb, opts, stream, out);
  } catch (const std::bad_alloc&) {
    set_error("fc_precond_build: out of host memory");
    return FC_E_NOMEM;
  }
}

static fc_status pcg_solve_body(fc_problem pb, fc_precond pc, const double* b_dev, double* x_dev,
                                const fc_solve_opts* opts, fc_solve_info* info, void* stream) {
  if (!pb || !pc || pc->pb != pb || !b_dev || !x_dev || b_dev == x_dev) {
    set_error("fc_pcg_solve: invalid arguments");
    return FC_E_ARG;
  }
  fc_solve_opts o{1e-10, 300000, FC_STOP_PRECOND, FC_MODE_F64, 16, 1e-4, nullptr, 0};
  if (opts) o = *opts;
  if (!(o.tol >= 0.0) || o.maxit < 0 || (o.stop != FC_STOP_PRECOND && o.stop != FC_STOP_RESIDUAL)) {
    set_error("fc_pcg_solve: invalid options");
    return FC_E_ARG;
  }
  if (o.mode < FC_MODE_F64 || o.mode > FC_MODE_LEARNED) {
    set_error("fc_pcg_solve: unsupported mode");
    return FC_E_UNSUPPORTED;
  }
  return pcg_solve(*pc, b_dev, x_dev, o, info, (hipStream_t)stream);
}

fc_status fc_pcg_solve(fc_problem pb, fc_precond pc, const double* b_dev, double* x_dev,
                       const fc_solve_opts* opts, fc_solve_info* info, void* stream) {
  try {
    return pcg_solve_body(pb, pc, b_dev, x_dev, opts, info, stream);
  } catch (const std::bad_alloc&) {
    set_error("fc_pcg_solve: out of host memory");
    return FC_E_NOMEM;
  }
}

fc_status fc_pcg_solve_noalloc(fc_problem pb, fc_precond pc, const double* b_dev,
                               double* x_dev, const fc_solve_opts* opts, fc_solve_info* info,
                               void* stream) {
  if (!pb || !pc || pc->pb != pb || !b_dev || !x_dev || b_dev == x_dev) {
    set_error("fc_pcg_solve_noalloc: invalid arguments");
    return FC_E_ARG;
  }
  fc_solve_opts o{1e-10, 300000, FC_STOP_PRECOND, FC_MODE_F64, 16, 1e-4, nullptr, 0, 1};
  if (opts) o = *opts;
  if (!(o.tol >= 0.0) || o.maxit < 0 || (o.stop != FC_STOP_PRECOND && o.stop != FC_STOP_RESIDUAL)) {
    set_error("fc_pcg_solve_noalloc: invalid options");
    return FC_E_ARG;
  }
  try {
    return pcg_solve_noalloc(*pc, b_dev, x_dev, o, info, (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    set_error("fc_pcg_solve_noalloc: out of host memory");
    return FC_E_NOMEM;
  }
}

void fc_problem_destroy(fc_problem pb) { free_problem(pb); }
void fc_precond_destroy(fc_precond pc) { free_precond(pc); }

}  // extern "C"
