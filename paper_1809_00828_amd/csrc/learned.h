// Learned coarse correction: network state shared by the training and
// solver translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fc_internal.h"

namespace fc {

// Parameters and optimiser state of the 4-level U-Net (device memory).
struct Net {
  int ch[4] = {0, 0, 0, 0};
  int in_ch = 2;
  int ci[15], co[15];
  int64_t woff[15], boff[15];
  int64_t wfoff[15];       // offsets in wpk of each layer's forward and
  int64_t wtoff[15];       // data-gradient (transposed) BF16 weights
  int64_t nparam = 0, nwpk = 0;
  float* p = nullptr;      // FP32 master parameters
  uint16_t* wpk = nullptr; // BF16 weights packed for the matrix-core
                           // convolutions (rows of (tap, channel) runs)
  float* g = nullptr;      // gradient
  float* m = nullptr;      // Adam first moment
  float* v = nullptr;      // Adam second moment
  int64_t step = 0;
  void init(const int32_t* c, int32_t in_channels);
};

// Activations of one forward pass (and gradient scratch) for batch B on an
// N0^3 grid: per level, kSlots tensors of the widest channel count there.
struct NetWs {
  static constexpr int kSlots = 9;
  int B = 0, capB = 0;
  int N[4] = {0, 0, 0, 0};
  int64_t off[4][kSlots];
  int64_t off_y = 0;
  float* buf = nullptr;
  double* partial = nullptr;
  float* wpart = nullptr;   // weight-gradient partials (wslots floats)
  int64_t wslots = 0;
  float* t(int l, int k) const { return buf + off[l][k]; }
  int64_t vox(int l) const { return (int64_t)N[l] * N[l] * N[l]; }
  float* y() const { return buf + off_y; }
  float* gy() const { return buf + off_y + (int64_t)capB * N[0] * N[0] * N[0]; }
  fc_status ensure(const Net& net, int B, int N0);
  void release();
};

int64_t net_param_count(const int32_t* c, int32_t in_channels);
// forward of batch B (input x: B x in_ch x N0^3) into ws.y()
hipError_t net_forward(const Net& net, NetWs& ws, const float* x, int B, hipStream_t s);
// parameter gradient into net.g from gy (B x 1 x N0^3); needs the forward
hipError_t net_backward(Net& net, NetWs& ws, const float* x, float* gy, int B, hipStream_t s);
// mean squared error of ws.y() against target: ws.partial[0..1024) sums,
// gy = d(loss)/d(y)
hipError_t net_mse(NetWs& ws, const float* target, float* gy, int64_t n, hipStream_t s);
hipError_t net_adam(Net& net, float lr, int64_t step, hipStream_t s);
hipError_t net_sync_bf16(Net& net, hipStream_t s);

// Device scalars of the coarse correction of one preconditioner apply.
struct LearnScalars {
  double gamma;      // step along P_c y (0: network term dropped)
  double yrc;        // y . P_c^T r
  double yAy;        // y . A_c y
  double wq;         // (P_c y) . q, q = A p of the current CG step
  double rc_nrm2;    // ||P_c^T r||^2
  int64_t n_apply;   // applies since the last reset
  int64_t n_drop;    // applies whose network term was dropped
  uint32_t ticket[4];
};

// Coarse vertex grid of a scalar 3-D lattice problem with an even number
// n of cells per direction: G = n/2 + 1 vertices per direction, vertex
// (a, b, c) at fine vertex (2a, 2b, 2c), index a + G (b + G c).
struct CoarseCtx {
  int n = 0, p = 0, G = 0;
  int64_t n1 = 0;            // lattice points per direction, p n + 1
  int64_t nvox = 0;          // G^3
  double* Ac = nullptr;      // [27][nvox] Galerkin stencil, tap dz*9+dy*3+dx
  float* xin = nullptr;      // [2][nvox] network input (residual, eta)
  float* mask = nullptr;     // [nvox] 1 where the vertex touches material
  double* rc = nullptr;      // [nvox] P_c^T r
  double* partial = nullptr; // [2 * kCoarsePartials]
  LearnScalars* ls = nullptr;
  fc_model_s* model = nullptr;
  int enabled = 1;           // 0: validation found the network does not pay
  NetWs ws;                  // inference activations (batch 1)
  double* cg = nullptr;      // [5][nvox] coarse CG vectors x, r, z, p, A_c p
  struct CoarseCg* cs = nullptr;
};
constexpr int kCoarsePartials = 2048;

// Scalars of the Jacobi-preconditioned CG on A_c (training targets).
struct CoarseCg {
  double rz, rr0, rr, alpha, beta;
  int64_t iters;
  int32_t done;              // 0 running, 1 converged, 3 breakdown
  uint32_t ticket[3];
};

// Build the coarse context of a preconditioner's problem (transfers,
// Galerkin operator by probing with 27 coloured prolongations, eta and
// mask channels).  Fails with FC_E_UNSUPPORTED unless the problem is a
// scalar 3-D lattice problem with even n.
fc_status coarse_create(fc_precond_s& pc, hipStream_t s, CoarseCtx** out);
void coarse_destroy(CoarseCtx* c);
// build pc.coarse on first use
fc_status coarse_ensure(fc_precond_s& pc, hipStream_t s);
// rc = P_c^T r, xin[0] = rc at unit RMS (skipped when sc->done)
hipError_t coarse_restrict(CoarseCtx& c, const double* r, float* xin0, const CgScalars* sc,
                           hipStream_t s);
// gamma = (y . rc) / (y . A_c y) into c.ls (0 when not positive finite);
// v = A_c y when v is given
hipError_t coarse_gamma(CoarseCtx& c, const float* y, const CgScalars* sc, double* v,
                        hipStream_t s);
// z += gamma P_c y on the vertex unknowns, c.ls->wq = (P_c y) . q when q
hipError_t coarse_prolong(CoarseCtx& c, const float* y, double* z, const double* q,
                          const CgScalars* sc, hipStream_t s);
// the whole correction after z = S r: restrict, network, gamma, prolong
hipError_t coarse_correct(CoarseCtx& c, const double* r, double* z, const double* q,
                          const CgScalars* sc, hipStream_t s);
// training pair at the current iterate: xin (2 channels) from r, target
// t = mask * sample(xs - x - [z]) at unit RMS
hipError_t coarse_snapshot(CoarseCtx& c, const double* r, const double* xs, const double* x,
                           const double* z, float* xin_out, float* t_out, hipStream_t s);
// training pair with the coarse Galerkin projection of the error as the
// target: xin from r, t = y at unit RMS, A_c y = P_c^T r on the material
// vertices (y = 0 elsewhere), solved by Jacobi-preconditioned CG to a
// relative residual of tol (synchronises; FC_E_NOTCONV past maxit)
fc_status coarse_snapshot_projection(CoarseCtx& c, const double* r, float* xin_out,
                                     float* t_out, double tol, int64_t maxit, hipStream_t s);

}  // namespace fc

struct fc_model_s {
  fc::Net net;
  fc::NetWs ws;
};
