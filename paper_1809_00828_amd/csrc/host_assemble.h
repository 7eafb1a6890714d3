// Host-side finite cell assembly (Sec. 2.1, Eq. 1) into the row-SoA BSR
// layout used by the device kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "fc.h"

namespace fc {

// Assembled system on the host.
//
// BSR with bdim x bdim blocks (bdim = number of field components).  Values
// use the "row-SoA" layout: the blocks of block row i occupy
// val[rowptr[i]*bb .. rowptr[i+1]*bb) and entry (r, c) of the k-th block of
// the row (k = 0..L-1, L = row length) sits at rowptr[i]*bb + (r*bdim+c)*L + k,
// so that consecutive lanes reading consecutive blocks of one row touch
// consecutive addresses.
struct HostSystem {
  int dim = 0, n = 0, p = 0, bdim = 1;
  int nn = 0;          // nodes per element, (p+1)^dim
  int m = 0;           // unknowns per element block, bdim*nn
  int64_t n_nodes = 0, n_dofs = 0, n_el = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
  std::vector<double> rhs;
  std::vector<int32_t> elem_nodes;   // [n_el*nn], element-local order
  std::vector<double> eta;           // [n_el]
};

// Assemble the description.  Returns FC_OK or an error with *err set.
fc_status assemble_host(const fc_problem_desc& d, HostSystem* out, std::string* err);

// Row-SoA value index helpers shared by host code that builds or reads the
// layout.
inline int64_t soa_index(const std::vector<int32_t>& rp, int64_t row, int bb,
                         int e, int64_t k) {
  int64_t L = rp[row + 1] - rp[row];
  return (int64_t)rp[row] * bb + (int64_t)e * L + k;
}

// Number of worker threads for host loops.
int host_threads();

template <class F>
void parallel_for(int64_t n, F&& f);

}  // namespace fc

#include "host_parallel.inl"
