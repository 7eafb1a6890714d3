// Schwarz apply launchers used by the solver.
#pragma once
#include "fc_internal.h"

namespace fc {
// Phase 1 only: y_B = P_B R_B (r - alpha q) for every block (q may be NULL,
// then r is gathered as is).  precision 0 = FP64, 1 = FP32, 2 = BF16 copy of
// the local inverses.  Skipped when sc->done is set (sc may be NULL).
hipError_t launch_schwarz_phase1(const fc_precond_s& pc, int precision, const double* r,
                                 const double* q, const CgScalars* sc, hipStream_t s);
}  // namespace fc
