// Schwarz apply launchers used by the solver.
#pragma once
#include "fc_internal.h"

namespace fc {
// Phase 1 only: y_B = P_B R_B (r - alpha q) for every block (q may be NULL,
// then r is gathered as is).  precision 0 = FP64, 1 = FP32, 2 = BF16 copy of
// the local inverses.  Skipped when sc->done is set (sc may be NULL).
hipError_t launch_schwarz_phase1(const fc_precond_s& pc, int precision, const double* r,
                                 const double* q, const CgScalars* sc, hipStream_t s);
// Phase 2 only: z = sum_B R_B^T y_B + fallback * r.
hipError_t launch_schwarz_pull(const fc_precond_s& pc, const double* r, double* z,
                               hipStream_t s);
// Elements per block of the wrapped-diagonal symmetric layout, (m/2+1)*m.
int64_t sym_block_stride(int m);
// Q = wrapped-diagonal copy of the dense FP64 local inverses pc.P in FP64
// (0), or diagonally scaled in FP32 (1) or BF16 (2) (needs pc.isd).
hipError_t launch_pack_sym(const fc_precond_s& pc, void* Q, int precision, hipStream_t s);
// Whether every row of every block of pc names the unknown the lattice L
// gives it (block b = cell b, rows in the cells' local tensor order);
// synchronises s.
hipError_t schwarz_check_lattice(const fc_precond_s& pc, const PullLattice L, bool* ok,
                                 hipStream_t s);
// isd = 1/sqrt(diag(A)) (1 where the diagonal is not positive).
hipError_t launch_inv_sqrt_diag(const fc_problem_s& pb, double* isd, hipStream_t s);
}  // namespace fc
