// SpMV launch helpers used by the solver.
#pragma once
#include "fc_internal.h"

namespace fc {
// Number of workgroups (and so of dot partials) of the fused SpMV.
int spmv_num_blocks(const DeviceBsr& A);
// q = A p leaving one partial (p, q) per workgroup in partial[0..nb)
// (skipped when sc->done is set).
// f32: the scaled FP32 copy, p already multiplied by rs = sqrt(diag A)
hipError_t launch_spmv_pq(const DeviceBsr& A, bool f32, const double* p, double* q,
                          CgScalars* sc, double* partial, hipStream_t s,
                          const double* rs = nullptr);
}  // namespace fc
