// Internal structures of libfc shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fc.h"

namespace fc {

void set_error(const std::string& msg);

#define FC_HIP(call)                                                         \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      ::fc::set_error(std::string(#call) + ": " + hipGetErrorString(e_));    \
      return FC_E_DEVICE;                                                    \
    }                                                                        \
  } while (0)

// Scalars of one PCG run kept on the device so the iteration never waits on
// the host.  Dots are reduced per workgroup into `partial`, and the last
// workgroup to finish (found with `ticket`) sums the partials in a fixed
// order, so every run is bitwise reproducible.
struct CgScalars {
  double rz;        // (r, z) of the current iterate
  double pq;        // (p, A p)
  double alpha, beta;
  double zz;        // (z, z) of the newest z
  double rr;        // (r, r) of the newest r
  double crit0;     // ||z_0|| or ||b|| (denominator of the stop test)
  double crit;      // newest relative criterion
  double tol;
  int64_t iter;     // products with A done
  int64_t maxit;
  int32_t done;     // 0 running, 1 converged, 2 maxit, 3 breakdown, 4 non-finite
  int32_t stop;     // FC_STOP_*
  uint32_t ticket;  // last-workgroup counter (reset by the last workgroup)
  uint32_t pad;
  double zn0, rn0;  // ||z_0||, ||r_0||
  double* history;  // optional per-iteration criterion
};

// Tensor-product lattice behind a matrix assembled from a problem
// description (dim = 0 otherwise): the block columns of every row are the
// lattice box spanned by the supports through the row's node, so they can
// be computed instead of read.
// Division of 32-bit unsigned numbers by an invariant d (Granlund and
// Montgomery, division by invariant integers using multiplication): with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, the quotient is
// (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0), t = (m n) >> 32.
struct FastDiv {
  uint32_t d = 1, m = 1, s1 = 0, s2 = 0;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  f.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
  f.s1 = l > 0 ? 1u : 0u;
  f.s2 = l > 0 ? l - 1 : 0u;
  return f;
}

struct LatticeInfo {
  int32_t dim = 0, n1 = 0, p = 0;
  FastDiv dn1, dp;   // division by n1 and by p
};

inline LatticeInfo make_lattice_info(int32_t dim, int32_t n1, int32_t p) {
  LatticeInfo l;
  l.dim = dim;
  l.n1 = n1;
  l.p = p;
  l.dn1 = make_fastdiv((uint32_t)n1);
  l.dp = make_fastdiv((uint32_t)p);
  return l;
}

// Lattice of the element blocks when every cell of a problem set up from a
// description is a block, in cell order (dim = 0 otherwise): the pull then
// finds the blocks holding a node from its lattice indices instead of the
// node-to-block map.
struct PullLattice {
  int32_t dim = 0, n = 0, p = 0, n1 = 0;
  // division by n, p and p + 1, and by the node-tile counts along the
  // first two directions (16 x 4 x 4 node tiles in 3-D, 32 x 8 in 2-D)
  FastDiv dn, dp, dp1, dtx, dty;
};

inline PullLattice make_pull_lattice(int32_t dim, int32_t n, int32_t p) {
  PullLattice l;
  l.dim = dim;
  l.n = n;
  l.p = p;
  l.n1 = p * n + 1;
  l.dn = make_fastdiv((uint32_t)n);
  l.dp = make_fastdiv((uint32_t)p);
  l.dp1 = make_fastdiv((uint32_t)(p + 1));
  const int tx = dim == 3 ? 16 : 32, ty = dim == 3 ? 4 : 8;
  l.dtx = make_fastdiv((uint32_t)((l.n1 + tx - 1) / tx));
  l.dty = make_fastdiv((uint32_t)((l.n1 + ty - 1) / ty));
  return l;
}

struct DeviceBsr {
  int32_t bdim = 1;
  int64_t n_rows = 0;      // block rows
  int64_t nnzb = 0;
  int32_t max_row = 0;     // longest block row
  int32_t group = 0;       // SpMV lanes per block row, fixed at set-up from the row lengths
  LatticeInfo lat;         // set when the columns were verified to be the lattice box
  int32_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;   // row-SoA layout
  float* val32 = nullptr;  // optional FP32 copy, same layout
  // mixed-precision products: block rows read in FP64 (rows_hi) and from
  // the FP32 copy (rows_lo), ascending
  int32_t* rows_hi = nullptr;
  int32_t* rows_lo = nullptr;
  int64_t n_hi = 0, n_lo = 0;
  // Sliced copy of a scalar lattice matrix (degree p <= 4): the rows of one
  // lattice line (fixed y, z) and one x class, interior vertex indices
  // (x = p, 2p, ..) or the other interior indices, in slices of 64 rows
  // whose boxes have equal shape.  A slice's entries are stored in pairs:
  // entries 2j and 2j + 1 of lane l at sell_val[sell_off[s] + 128 j + 2 l]
  // and the next word, an odd last entry alone at sell_off[s] + 128 j + l
  // (zero for lanes past the class's end).
  // The boundary vertex rows (x = 0 and x = n1 - 1) are listed in sell_rest
  // and use the row layout.
  double* sell_val = nullptr;
  int64_t* sell_off = nullptr;   // [n_slices + 1]
  int64_t n_slices = 0;
  int32_t sell_cv = 0, sell_nv = 0, sell_nn = 0;   // vertex slices per line, rows per class
  int32_t* sell_rest = nullptr;
  int64_t n_rest = 0;
};

struct SolverWs;
void solver_ws_destroy(SolverWs* ws);
struct CoarseCtx;
void coarse_destroy(CoarseCtx* c);

}  // namespace fc

struct fc_problem_s {
  int device = 0;
  int32_t dim = 0, p = 0, n = 0;   // lattice (0 when built from a matrix)
  int32_t bdim = 1, nn = 0, m = 0;
  int64_t n_nodes = 0, n_dofs = 0, n_el = 0;
  fc::DeviceBsr A;
  double* rhs = nullptr;           // [n_dofs]
  int32_t* elem_nodes = nullptr;   // [n_el*nn]
  std::vector<double> eta;         // host copy [n_el]
  std::vector<int32_t> elem_nodes_host;
  double* diag = nullptr;          // A_ll [n_dofs]
};

struct fc_precond_s {
  fc_problem pb = nullptr;
  int32_t m = 0, nn = 0, bdim = 1;
  int64_t n_blocks = 0;
  int32_t block_kind = FC_BLOCK_ELEMENT;
  int32_t* block_elem = nullptr;   // [n_blocks] element of each block (patch: its index)
  int32_t* bnodes = nullptr;       // vertex patches: [n_blocks][nn] node lists, -1 padding
  double* P = nullptr;             // [n_blocks*m*m] FP64 local inverses (dense)
  double* Q = nullptr;             // wrapped-diagonal symmetric copy, FP64
  float* Q32 = nullptr;            // optional FP32 wrapped-diagonal copy of D^1/2 P D^1/2
  int32_t* unsafe32 = nullptr;     // blocks whose FP32 copy is not safely positive
  int32_t* unsafe_flag32 = nullptr; // the same as one flag per block
  int64_t n_unsafe32 = 0;          //   (applied from the FP64 copy instead)
  uint16_t* Lbf = nullptr;         // optional BF16 scaled Cholesky factors
  double* isd = nullptr;           // [n_dofs] 1/sqrt(A_ll), scaling of Q32/Lbf
  int32_t* inv_ptr = nullptr;      // [n_nodes+1] node -> (block, local node)
  int32_t* inv_idx = nullptr;      // entries: block*m + local_node*bdim
  double* fallback = nullptr;      // [n_dofs] 1/A_ll where S_ll = 0, else 0
  fc::PullLattice lat;             // set when every cell is a block (lattice pull)
  double* y = nullptr;             // [n_blocks*m] block outputs (workspace)
  int64_t n_fallback = 0, n_eig = 0, n_dropped = 0;
  std::vector<int32_t> dropped;    // host copy: eigenvalues dropped per block
  double eps = 1e-13;
  int32_t stabilize = 1;
  fc::SolverWs* ws = nullptr;      // PCG workspace, created on first solve
  fc::CoarseCtx* coarse = nullptr; // learned coarse correction, when attached
};

namespace fc {

// Node lists of the preconditioner's blocks: the element lists of the
// problem, or the patch lists of a vertex-patch preconditioner.
inline const int32_t* block_nodes(const fc_precond_s& pc) {
  return pc.bnodes ? pc.bnodes : pc.pb->elem_nodes;
}

// ---- launchers (each returns hipSuccess or the first launch error) ----
// y = A x  (and optionally partial dots (x, y) per workgroup)
hipError_t launch_spmv(const DeviceBsr& A, const double* x, double* y,
                       hipStream_t s);
// lanes per block row of A's products, from its mean row length
int spmv_group_for(const DeviceBsr& A);
// verify on the device that A's columns are the lattice boxes of (dim, n1,
// p); if so record it in A.lat, so the SpMV computes columns instead of
// reading them
hipError_t spmv_enable_lattice(DeviceBsr& A, int dim, int n1, int p, hipStream_t s);

hipError_t launch_block_extract(const fc_problem_s& pb, const fc_precond_s& pc,
                                hipStream_t s);

// z = S r
hipError_t launch_schwarz_apply(const fc_precond_s& pc, const double* r,
                                double* z, hipStream_t s);

// drop the captured solver chunk (its kernels hold buffers about to change)
void solver_invalidate_graph(fc_precond_s& pc);

}  // namespace fc
