// SpMV launch helpers used by the solver.
#pragma once
#include "fc_internal.h"

namespace fc {
// Number of workgroups (and so of dot partials) of the fused SpMV.
int spmv_num_blocks(const DeviceBsr& A);
// q = A p leaving one partial (p, q) per workgroup in partial[0..nb)
// (skipped when sc->done is set)
hipError_t launch_spmv_pq(const DeviceBsr& A, const double* p, double* q, CgScalars* sc,
                          double* partial, hipStream_t s);
// q = A p with the rows A.rows_hi from the FP64 values and p, and the rows
// A.rows_lo from the FP32 copy and p32 = fl32(p) (skipped when sc->done is
// set)
hipError_t launch_spmv_mixed(const DeviceBsr& A, const double* p, const float* p32, double* q,
                             const CgScalars* sc, hipStream_t s);
}  // namespace fc
