// Preconditioner set-up launchers.
#pragma once
#include "fc_internal.h"

namespace fc {
hipError_t launch_jacobi(fc_precond_s& pc, const int32_t* sel, int64_t count,
                         double* work, int32_t* dropped, hipStream_t s);
// true when the Jacobi eigen path keeps its blocks in global memory
bool jacobi_needs_work(int m);
hipError_t launch_sweep(fc_precond_s& pc, int32_t* need_eig, hipStream_t s);
// the same certified sweep for m <= 64 (one wave per block)
hipError_t launch_sweep_small(fc_precond_s& pc, int32_t* need_eig, hipStream_t s);
// Scaled Cholesky factors of the local inverses in BF16 into pc.Lbf (needs
// pc.isd); with `unsafe` instead only flag the blocks whose FP32-rounded
// scaled inverse is not safely positive definite
hipError_t launch_chol_pack(fc_precond_s& pc, hipStream_t s, int32_t* unsafe = nullptr);
hipError_t launch_diag(const fc_problem_s& pb, hipStream_t s);
hipError_t launch_fallback(const fc_problem_s& pb, fc_precond_s& pc,
                           unsigned long long* d_count, hipStream_t s);
// A.val32 = FP32 copy of A.val (same layout)
hipError_t launch_cast_matrix(const DeviceBsr& A, hipStream_t s);
}  // namespace fc
