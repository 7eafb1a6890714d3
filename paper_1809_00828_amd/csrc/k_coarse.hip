// Coarse level of the learned correction: the transfers between the
// unknowns and the coarse vertex grid, the Galerkin coarse operator, the
// energy-optimal step along the network's correction, and the training
// pairs taken from a running solve.
//
// The vertex functions of the integrated Legendre basis are the Q1 hats of
// the cell grid, so a trilinear function on the mesh with half as many
// cells per direction is represented exactly by its values on the vertex
// unknowns (all higher modes zero).  P_c is that injection; restriction of
// a residual is P_c^T; A_c = P_c^T A P_c couples each coarse vertex with its
// 27 neighbours and is found by 27 products of A with coloured
// prolongations (colours = vertex index mod 3 per direction).
//
// Correction inside flexible CG, after z = S r:
//   rc = P_c^T r; y = N(rc / rms(rc), eta_c); gamma = (y.rc)/(y.A_c y);
//   z += gamma P_c y  (gamma = 0, the network term dropped, unless
//   y.A_c y > 0 and the quotient is finite).
// The kernels gate on the solver's stop flag so captured chunks can run on
// after convergence without changing the iterate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dev_common.h"
#include "learned.h"

namespace fc {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int64_t lattice(int64_t n1, int p, int fx, int fy, int fz) {
  return (int64_t)p * fx + n1 * ((int64_t)p * fy + n1 * (int64_t)p * fz);
}

// value of P_c^T v at coarse vertex (ax, ay, az): weights 1 at the
// coincident fine vertex, 1/2 at the fine neighbours along each axis
__device__ __forceinline__ double restrict_at(const double* __restrict__ v, int n, int p,
                                              int64_t n1, int ax, int ay, int az) {
  double s = 0.0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int fz = 2 * az + dz;
    if (fz < 0 || fz > n) continue;
    const double wz = dz ? 0.5 : 1.0;
    for (int dy = -1; dy <= 1; ++dy) {
      const int fy = 2 * ay + dy;
      if (fy < 0 || fy > n) continue;
      const double wzy = wz * (dy ? 0.5 : 1.0);
      for (int dx = -1; dx <= 1; ++dx) {
        const int fx = 2 * ax + dx;
        if (fx < 0 || fx > n) continue;
        s = fma(wzy * (dx ? 0.5 : 1.0), v[lattice(n1, p, fx, fy, fz)], s);
      }
    }
  }
  return s;
}

__global__ __launch_bounds__(kT) void k_restrict(const double* __restrict__ r, int n, int p,
                                                 int64_t n1, int G, double* __restrict__ rc,
                                                 float* __restrict__ xin0,
                                                 double* __restrict__ partial, LearnScalars* ls,
                                                 const CgScalars* __restrict__ sc) {
  __shared__ double lds[16];
  __shared__ int flag;
  if (sc && sc->done) return;
  const int64_t nvox = (int64_t)G * G * G;
  double ss = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x) {
    const int ax = (int)(a % G), ay = (int)((a / G) % G), az = (int)(a / ((int64_t)G * G));
    const double s = restrict_at(r, n, p, n1, ax, ay, az);
    rc[a] = s;
    ss = fma(s, s, ss);
  }
  ss = block_sum(ss, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = ss;
  if (!last_block(&ls->ticket[0], gridDim.x, &flag)) return;
  const double nrm2 = sum_partials(partial, gridDim.x, lds);
  const double scale = nrm2 > 0.0 ? sqrt((double)nvox / nrm2) : 0.0;
  if (threadIdx.x == 0) ls->rc_nrm2 = nrm2;
  if (xin0)
    for (int64_t i = threadIdx.x; i < nvox; i += blockDim.x) xin0[i] = (float)(rc[i] * scale);
}

// v = A_c y (optional), per-workgroup y.rc and y.v; the last workgroup
// sets gamma
__global__ __launch_bounds__(kT) void k_coarse_gamma(const float* __restrict__ y,
                                                     const double* __restrict__ Ac,
                                                     const double* __restrict__ rc, int G,
                                                     double* __restrict__ v_out,
                                                     double* __restrict__ partial,
                                                     LearnScalars* ls,
                                                     const CgScalars* __restrict__ sc) {
  __shared__ double lds[16];
  __shared__ int flag;
  if (sc && sc->done) return;
  const int64_t nvox = (int64_t)G * G * G;
  double d1 = 0.0, d2 = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x) {
    const int ax = (int)(a % G), ay = (int)((a / G) % G), az = (int)(a / ((int64_t)G * G));
    double v = 0.0;
    for (int o = 0; o < 27; ++o) {
      const int bx = ax + o % 3 - 1, by = ay + (o / 3) % 3 - 1, bz = az + o / 9 - 1;
      if (bx < 0 || bx >= G || by < 0 || by >= G || bz < 0 || bz >= G) continue;
      v = fma(Ac[(int64_t)o * nvox + a], (double)y[bx + (int64_t)G * (by + (int64_t)G * bz)], v);
    }
    if (v_out) v_out[a] = v;
    const double ya = (double)y[a];
    d1 = fma(ya, rc[a], d1);
    d2 = fma(ya, v, d2);
  }
  d1 = block_sum(d1, lds);
  d2 = block_sum(d2, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = d1;
    partial[gridDim.x + blockIdx.x] = d2;
  }
  if (!last_block(&ls->ticket[1], gridDim.x, &flag)) return;
  const double yrc = sum_partials(partial, gridDim.x, lds);
  const double yAy = sum_partials(partial + gridDim.x, gridDim.x, lds);
  if (threadIdx.x == 0) {
    double g = (yAy > 0.0 && isfinite(yAy) && isfinite(yrc)) ? yrc / yAy : 0.0;
    if (!isfinite(g)) g = 0.0;
    ls->gamma = g;
    ls->yrc = yrc;
    ls->yAy = yAy;
    ls->n_apply += 1;
    if (g == 0.0) ls->n_drop += 1;
  }
}

// trilinear value of the coarse field y at fine vertex (fx, fy, fz)
__device__ __forceinline__ double interp_at(const float* __restrict__ y, int G, int fx, int fy,
                                            int fz) {
  const int x0 = fx >> 1, y0 = fy >> 1, z0 = fz >> 1;
  const int nx = (fx & 1) ? 2 : 1, ny = (fy & 1) ? 2 : 1, nz = (fz & 1) ? 2 : 1;
  const double wx = nx == 2 ? 0.5 : 1.0, wy = ny == 2 ? 0.5 : 1.0, wz = nz == 2 ? 0.5 : 1.0;
  double s = 0.0;
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a)
        s += (double)y[(x0 + a) + (int64_t)G * ((y0 + b) + (int64_t)G * (z0 + c))];
  return s * wx * wy * wz;
}

// z += gamma P_c y on the vertex unknowns; partial (P_c y) . q
__global__ __launch_bounds__(kT) void k_prolong(const float* __restrict__ y, int n, int p,
                                                int64_t n1, int G, double* __restrict__ z,
                                                const double* __restrict__ q,
                                                double* __restrict__ partial, LearnScalars* ls,
                                                const CgScalars* __restrict__ sc) {
  __shared__ double lds[16];
  __shared__ int flag;
  if (sc && sc->done) return;
  const double g = ls->gamma;
  const int64_t nv = (int64_t)(n + 1) * (n + 1) * (n + 1);
  double d = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int fx = (int)(i % (n + 1)), fy = (int)((i / (n + 1)) % (n + 1)),
              fz = (int)(i / ((int64_t)(n + 1) * (n + 1)));
    const double w = interp_at(y, G, fx, fy, fz);
    const int64_t k = lattice(n1, p, fx, fy, fz);
    if (g != 0.0) z[k] = fma(g, w, z[k]);
    if (q) d = fma(w, q[k], d);
  }
  if (!q) return;
  d = block_sum(d, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = d;
  if (!last_block(&ls->ticket[2], gridDim.x, &flag)) return;
  const double wq = sum_partials(partial, gridDim.x, lds);
  if (threadIdx.x == 0) ls->wq = wq;
}

// probing: A_c[o][a] = (P_c^T t)[a] for the neighbour b = a + off_o of
// colour (cx, cy, cz), where t = A P_c (indicator of that colour)
__global__ __launch_bounds__(kT) void k_probe_collect(const double* __restrict__ t, int n, int p,
                                                      int64_t n1, int G, int cx, int cy, int cz,
                                                      double* __restrict__ Ac) {
  const int64_t nvox = (int64_t)G * G * G;
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nvox) return;
  const int ax = (int)(a % G), ay = (int)((a / G) % G), az = (int)(a / ((int64_t)G * G));
  // the one coordinate in {a-1, a, a+1} congruent to the colour mod 3
  auto pick = [](int av, int col) {
    const int d = ((col - av) % 3 + 3) % 3;
    return d <= 1 ? av + d : av - 1;
  };
  const int bx = pick(ax, cx), by = pick(ay, cy), bz = pick(az, cz);
  if (bx < 0 || bx >= G || by < 0 || by >= G || bz < 0 || bz >= G) return;
  const int o = (bz - az + 1) * 9 + (by - ay + 1) * 3 + (bx - ax + 1);
  Ac[(int64_t)o * nvox + a] = restrict_at(t, n, p, n1, ax, ay, az);
}

__global__ void k_colour(float* __restrict__ y, int G, int cx, int cy, int cz) {
  const int64_t nvox = (int64_t)G * G * G;
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nvox) return;
  const int ax = (int)(a % G), ay = (int)((a / G) % G), az = (int)(a / ((int64_t)G * G));
  y[a] = (ax % 3 == cx && ay % 3 == cy && az % 3 == cz) ? 1.f : 0.f;
}

__global__ void k_zero(double* __restrict__ v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = 0.0;
}

// target t[a] = mask[a] * (xs - x - [z])[vertex 2a], then unit RMS
__global__ __launch_bounds__(kT) void k_target(const double* __restrict__ xs,
                                               const double* __restrict__ x,
                                               const double* __restrict__ z,
                                               const float* __restrict__ mask, int p, int64_t n1,
                                               int G, float* __restrict__ t,
                                               double* __restrict__ raw,
                                               double* __restrict__ partial, LearnScalars* ls) {
  __shared__ double lds[16];
  __shared__ int flag;
  const int64_t nvox = (int64_t)G * G * G;
  double ss = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x) {
    const int ax = (int)(a % G), ay = (int)((a / G) % G), az = (int)(a / ((int64_t)G * G));
    const int64_t k = lattice(n1, p, 2 * ax, 2 * ay, 2 * az);
    double v = xs[k] - x[k];
    if (z) v -= z[k];
    v *= (double)mask[a];
    raw[a] = v;
    ss = fma(v, v, ss);
  }
  ss = block_sum(ss, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = ss;
  if (!last_block(&ls->ticket[3], gridDim.x, &flag)) return;
  const double nrm2 = sum_partials(partial, gridDim.x, lds);
  const double scale = nrm2 > 0.0 ? sqrt((double)nvox / nrm2) : 0.0;
  for (int64_t i = threadIdx.x; i < nvox; i += blockDim.x) t[i] = (float)(raw[i] * scale);
}

// ---- Jacobi-preconditioned CG on A_c restricted to the material vertices
// (y = 0 on the others), for the projection targets.  Vectors x, r, z, p, v
// of G^3 values each; the diagonal is the centre tap of the stencil.
__device__ __forceinline__ double stencil_apply(const double* __restrict__ Ac,
                                                const double* __restrict__ v, int G,
                                                int64_t nvox, int64_t a) {
  const int ax = (int)(a % G), ay = (int)((a / G) % G), az = (int)(a / ((int64_t)G * G));
  double s = 0.0;
  for (int o = 0; o < 27; ++o) {
    const int bx = ax + o % 3 - 1, by = ay + (o / 3) % 3 - 1, bz = az + o / 9 - 1;
    if (bx < 0 || bx >= G || by < 0 || by >= G || bz < 0 || bz >= G) continue;
    s = fma(Ac[(int64_t)o * nvox + a], v[bx + (int64_t)G * (by + (int64_t)G * bz)], s);
  }
  return s;
}

__device__ __forceinline__ double jacobi_of(const double* __restrict__ Ac,
                                            const float* __restrict__ mask, int64_t nvox,
                                            int64_t a, double ra) {
  const double d = Ac[13 * nvox + a];
  return (mask[a] > 0.f && d > 0.0) ? ra / d : 0.0;
}

__global__ __launch_bounds__(kT) void k_ccg_init(const double* __restrict__ Ac,
                                                 const float* __restrict__ mask,
                                                 const double* __restrict__ rhs, int64_t nvox,
                                                 double* __restrict__ v5,
                                                 double* __restrict__ partial, CoarseCg* cs) {
  __shared__ double lds[16];
  __shared__ int flag;
  double* x = v5;
  double* r = v5 + nvox;
  double* z = v5 + 2 * nvox;
  double* p = v5 + 3 * nvox;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x) {
    const double ra = mask[a] > 0.f ? rhs[a] : 0.0;
    const double za = jacobi_of(Ac, mask, nvox, a, ra);
    x[a] = 0.0;
    r[a] = ra;
    z[a] = za;
    p[a] = za;
    s1 = fma(ra, za, s1);
    s2 = fma(ra, ra, s2);
  }
  s1 = block_sum(s1, lds);
  s2 = block_sum(s2, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s1;
    partial[gridDim.x + blockIdx.x] = s2;
  }
  if (!last_block(&cs->ticket[0], gridDim.x, &flag)) return;
  const double rz = sum_partials(partial, gridDim.x, lds);
  const double rr = sum_partials(partial + gridDim.x, gridDim.x, lds);
  if (threadIdx.x == 0) {
    cs->rz = rz;
    cs->rr0 = rr;
    cs->rr = rr;
    cs->iters = 0;
    cs->done = rr > 0.0 ? 0 : 1;
  }
}

// v = A_c p on the material vertices and (p, v); the last workgroup sets
// alpha (breakdown unless (p, v) > 0)
__global__ __launch_bounds__(kT) void k_ccg_apply(const double* __restrict__ Ac,
                                                  const float* __restrict__ mask, int G,
                                                  int64_t nvox, double* __restrict__ v5,
                                                  double* __restrict__ partial, CoarseCg* cs) {
  __shared__ double lds[16];
  __shared__ int flag;
  if (cs->done) return;
  const double* p = v5 + 3 * nvox;
  double* v = v5 + 4 * nvox;
  double s = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x) {
    const double va = mask[a] > 0.f ? stencil_apply(Ac, p, G, nvox, a) : 0.0;
    v[a] = va;
    s = fma(p[a], va, s);
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
  if (!last_block(&cs->ticket[1], gridDim.x, &flag)) return;
  const double pq = sum_partials(partial, gridDim.x, lds);
  if (threadIdx.x == 0) {
    cs->iters += 1;
    if (!(pq > 0.0) || !(cs->rz > 0.0)) cs->done = 3;
    else cs->alpha = cs->rz / pq;
  }
}

// x += alpha p, r -= alpha v, z = r / diag; the last workgroup sets beta
// and tests ||r|| / ||r_0|| <= tol
__global__ __launch_bounds__(kT) void k_ccg_update(const double* __restrict__ Ac,
                                                   const float* __restrict__ mask, int64_t nvox,
                                                   double* __restrict__ v5, double tol,
                                                   double* __restrict__ partial, CoarseCg* cs) {
  __shared__ double lds[16];
  __shared__ int flag;
  if (cs->done) return;
  const double alpha = cs->alpha;
  double* x = v5;
  double* r = v5 + nvox;
  double* z = v5 + 2 * nvox;
  const double* p = v5 + 3 * nvox;
  const double* v = v5 + 4 * nvox;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x) {
    x[a] = fma(alpha, p[a], x[a]);
    const double ra = fma(-alpha, v[a], r[a]);
    const double za = jacobi_of(Ac, mask, nvox, a, ra);
    r[a] = ra;
    z[a] = za;
    s1 = fma(ra, za, s1);
    s2 = fma(ra, ra, s2);
  }
  s1 = block_sum(s1, lds);
  s2 = block_sum(s2, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s1;
    partial[gridDim.x + blockIdx.x] = s2;
  }
  if (!last_block(&cs->ticket[2], gridDim.x, &flag)) return;
  const double rz = sum_partials(partial, gridDim.x, lds);
  const double rr = sum_partials(partial + gridDim.x, gridDim.x, lds);
  if (threadIdx.x == 0) {
    cs->beta = rz / cs->rz;
    cs->rz = rz;
    cs->rr = rr;
    if (!(rr == rr)) cs->done = 3;
    else if (sqrt(rr) <= tol * sqrt(cs->rr0)) cs->done = 1;
  }
}

__global__ void k_ccg_dir(int64_t nvox, double* __restrict__ v5, const CoarseCg* cs) {
  if (cs->done) return;
  const double beta = cs->beta;
  const double* z = v5 + 2 * nvox;
  double* p = v5 + 3 * nvox;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x)
    p[a] = fma(beta, p[a], z[a]);
}

// t = x at unit RMS
__global__ __launch_bounds__(kT) void k_unit_rms(const double* __restrict__ x, int64_t nvox,
                                                 float* __restrict__ t,
                                                 double* __restrict__ partial, LearnScalars* ls) {
  __shared__ double lds[16];
  __shared__ int flag;
  double ss = 0.0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nvox;
       a += (int64_t)gridDim.x * blockDim.x)
    ss = fma(x[a], x[a], ss);
  ss = block_sum(ss, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = ss;
  if (!last_block(&ls->ticket[3], gridDim.x, &flag)) return;
  const double nrm2 = sum_partials(partial, gridDim.x, lds);
  const double scale = nrm2 > 0.0 ? sqrt((double)nvox / nrm2) : 0.0;
  for (int64_t i = threadIdx.x; i < nvox; i += blockDim.x) t[i] = (float)(x[i] * scale);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kT - 1) / kT); }
// grid of the reducing kernels: at most kCoarsePartials workgroups
inline unsigned red_blocks(int64_t n) {
  return std::min<unsigned>(blocks_for(n), (unsigned)kCoarsePartials);
}

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t coarse_restrict(CoarseCtx& c, const double* r, float* xin0, const CgScalars* sc,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_restrict, dim3(red_blocks(c.nvox)), dim3(kT), 0, s, r, c.n, c.p, c.n1,
                     c.G, c.rc, xin0, c.partial, c.ls, sc);
  return hipGetLastError();
}

hipError_t coarse_gamma(CoarseCtx& c, const float* y, const CgScalars* sc, double* v,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gamma, dim3(red_blocks(c.nvox)), dim3(kT), 0, s, y, c.Ac, c.rc,
                     c.G, v, c.partial, c.ls, sc);
  return hipGetLastError();
}

hipError_t coarse_prolong(CoarseCtx& c, const float* y, double* z, const double* q,
                          const CgScalars* sc, hipStream_t s) {
  const int64_t nv = (int64_t)(c.n + 1) * (c.n + 1) * (c.n + 1);
  const unsigned nb = red_blocks(nv);
  hipLaunchKernelGGL(k_prolong, dim3(nb), dim3(kT), 0, s, y, c.n, c.p, c.n1, c.G, z, q,
                     c.partial, c.ls, sc);
  return hipGetLastError();
}

hipError_t coarse_correct(CoarseCtx& c, const double* r, double* z, const double* q,
                          const CgScalars* sc, hipStream_t s) {
  hipError_t e;
  if ((e = coarse_restrict(c, r, c.xin, sc, s)) != hipSuccess) return e;
  if ((e = net_forward(c.model->net, c.ws, c.xin, 1, s)) != hipSuccess) return e;
  if ((e = coarse_gamma(c, c.ws.y(), sc, nullptr, s)) != hipSuccess) return e;
  return coarse_prolong(c, c.ws.y(), z, q, sc, s);
}

hipError_t coarse_snapshot(CoarseCtx& c, const double* r, const double* xs, const double* x,
                           const double* z, float* xin_out, float* t_out, hipStream_t s) {
  hipError_t e;
  if ((e = coarse_restrict(c, r, xin_out, nullptr, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(xin_out + c.nvox, c.xin + c.nvox, c.nvox * sizeof(float),
                          hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return e;
  // the raw target reuses rc (the restricted residual is no longer needed)
  hipLaunchKernelGGL(k_target, dim3(red_blocks(c.nvox)), dim3(kT), 0, s, xs, x, z, c.mask, c.p,
                     c.n1, c.G, t_out, c.rc, c.partial, c.ls);
  return hipGetLastError();
}

fc_status coarse_snapshot_projection(CoarseCtx& c, const double* r, float* xin_out,
                                     float* t_out, double tol, int64_t maxit, hipStream_t s) {
  const int64_t nv = c.nvox;
  if (!c.cg) FC_HIP(hipMalloc(&c.cg, 5 * nv * sizeof(double)));
  if (!c.cs) {
    FC_HIP(hipMalloc(&c.cs, sizeof(CoarseCg)));
    FC_HIP(hipMemsetAsync(c.cs, 0, sizeof(CoarseCg), s));
  }
  FC_HIP(coarse_restrict(c, r, xin_out, nullptr, s));
  FC_HIP(hipMemcpyAsync(xin_out + nv, c.xin + nv, nv * sizeof(float), hipMemcpyDeviceToDevice,
                        s));
  const unsigned nb = red_blocks(nv);
  hipLaunchKernelGGL(k_ccg_init, dim3(nb), dim3(kT), 0, s, c.Ac, c.mask, c.rc, nv, c.cg,
                     c.partial, c.cs);
  FC_HIP(hipGetLastError());
  constexpr int kChunk = 32;
  CoarseCg h{};
  for (int64_t it = 0;; it += kChunk) {
    for (int k = 0; k < kChunk; ++k) {
      hipLaunchKernelGGL(k_ccg_apply, dim3(nb), dim3(kT), 0, s, c.Ac, c.mask, c.G, nv, c.cg,
                         c.partial, c.cs);
      hipLaunchKernelGGL(k_ccg_update, dim3(nb), dim3(kT), 0, s, c.Ac, c.mask, nv, c.cg, tol,
                         c.partial, c.cs);
      hipLaunchKernelGGL(k_ccg_dir, dim3(nb), dim3(kT), 0, s, nv, c.cg, c.cs);
    }
    FC_HIP(hipGetLastError());
    FC_HIP(hipMemcpyAsync(&h, c.cs, sizeof(h), hipMemcpyDeviceToHost, s));
    FC_HIP(hipStreamSynchronize(s));
    if (h.done != 0 || h.iters >= maxit) break;
  }
  if (h.done != 1) {
    set_error(h.done == 3 ? "coarse projection target: CG breakdown on A_c"
                          : "coarse projection target: CG on A_c did not converge");
    return h.done == 3 ? FC_E_BREAKDOWN : FC_E_NOTCONV;
  }
  hipLaunchKernelGGL(k_unit_rms, dim3(nb), dim3(kT), 0, s, c.cg, nv, t_out, c.partial, c.ls);
  FC_HIP(hipGetLastError());
  return FC_OK;
}

void coarse_destroy(CoarseCtx* c) {
  if (!c) return;
  c->ws.release();
  for (void* p : {(void*)c->Ac, (void*)c->xin, (void*)c->mask, (void*)c->rc, (void*)c->partial,
                  (void*)c->ls, (void*)c->cg, (void*)c->cs})
    if (p) (void)hipFree(p);
  delete c;
}

// Host: coarse volume fraction (mean over the coarse cells touching a
// vertex of their fine cells' eta) and the material mask of every vertex.
static void host_channels(const fc_problem_s& pb, int G, std::vector<float>& eta_c,
                          std::vector<float>& mask) {
  const int n = pb.n, nc = n / 2;
  auto eta = [&](int x, int y, int z) { return pb.eta[(size_t)x + (size_t)n * (y + (size_t)n * z)]; };
  std::vector<double> cc((size_t)nc * nc * nc, 0.0);
  for (int z = 0; z < nc; ++z)
    for (int y = 0; y < nc; ++y)
      for (int x = 0; x < nc; ++x) {
        double s = 0.0;
        for (int c = 0; c < 8; ++c) s += eta(2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2));
        cc[(size_t)x + (size_t)nc * (y + (size_t)nc * z)] = s / 8.0;
      }
  eta_c.assign((size_t)G * G * G, 0.f);
  mask.assign((size_t)G * G * G, 0.f);
  for (int az = 0; az < G; ++az)
    for (int ay = 0; ay < G; ++ay)
      for (int ax = 0; ax < G; ++ax) {
        double s = 0.0;
        int cnt = 0;
        for (int cz = az - 1; cz <= az; ++cz)
          for (int cy = ay - 1; cy <= ay; ++cy)
            for (int cx = ax - 1; cx <= ax; ++cx) {
              if (cx < 0 || cy < 0 || cz < 0 || cx >= nc || cy >= nc || cz >= nc) continue;
              s += cc[(size_t)cx + (size_t)nc * (cy + (size_t)nc * cz)];
              ++cnt;
            }
        bool phys = false;
        for (int fz = 2 * az - 1; fz <= 2 * az; ++fz)
          for (int fy = 2 * ay - 1; fy <= 2 * ay; ++fy)
            for (int fx = 2 * ax - 1; fx <= 2 * ax; ++fx) {
              if (fx < 0 || fy < 0 || fz < 0 || fx >= n || fy >= n || fz >= n) continue;
              if (eta(fx, fy, fz) > 0.0) phys = true;
            }
        const size_t a = (size_t)ax + (size_t)G * (ay + (size_t)G * az);
        eta_c[a] = (float)(s / cnt);
        mask[a] = phys ? 1.f : 0.f;
      }
}

fc_status coarse_create(fc_precond_s& pc, hipStream_t s, CoarseCtx** out) {
  const fc_problem_s& pb = *pc.pb;
  if (pb.dim != 3 || pb.bdim != 1 || pb.n < 2 || (pb.n % 2) != 0 || pb.p < 1 ||
      (int64_t)pb.eta.size() != (int64_t)pb.n * pb.n * pb.n) {
    set_error("learned coarse correction: needs a scalar 3-D lattice problem with even n");
    return FC_E_UNSUPPORTED;
  }
  CoarseCtx* c = new (std::nothrow) CoarseCtx();
  if (!c) return FC_E_NOMEM;
  struct Guard {
    CoarseCtx* c;
    ~Guard() { if (c) coarse_destroy(c); }
  } guard{c};
  c->n = pb.n;
  c->p = pb.p;
  c->G = pb.n / 2 + 1;
  c->n1 = (int64_t)pb.p * pb.n + 1;
  c->nvox = (int64_t)c->G * c->G * c->G;
  const int64_t nvox = c->nvox;
  FC_HIP(hipMalloc(&c->Ac, 27 * nvox * sizeof(double)));
  FC_HIP(hipMalloc(&c->xin, 2 * nvox * sizeof(float)));
  FC_HIP(hipMalloc(&c->mask, nvox * sizeof(float)));
  FC_HIP(hipMalloc(&c->rc, nvox * sizeof(double)));
  FC_HIP(hipMalloc(&c->partial, 2 * kCoarsePartials * sizeof(double)));
  FC_HIP(hipMalloc(&c->ls, sizeof(LearnScalars)));
  FC_HIP(hipMemsetAsync(c->ls, 0, sizeof(LearnScalars), s));
  FC_HIP(hipMemsetAsync(c->Ac, 0, 27 * nvox * sizeof(double), s));
  std::vector<float> eta_c, mask;
  host_channels(pb, c->G, eta_c, mask);
  FC_HIP(hipMemcpyAsync(c->xin + nvox, eta_c.data(), nvox * sizeof(float),
                        hipMemcpyHostToDevice, s));
  FC_HIP(hipMemcpyAsync(c->mask, mask.data(), nvox * sizeof(float), hipMemcpyHostToDevice, s));
  // probing with the 27 colours
  double *u = nullptr, *t = nullptr;
  float* yc = nullptr;
  const int64_t nd = pb.n_dofs;
  FC_HIP(hipMalloc(&u, nd * sizeof(double)));
  FC_HIP(hipMalloc(&t, nd * sizeof(double)));
  FC_HIP(hipMalloc(&yc, nvox * sizeof(float)));
  const double one = 1.0;
  FC_HIP(hipMemcpyAsync(&c->ls->gamma, &one, sizeof(double), hipMemcpyHostToDevice, s));
  hipError_t e = hipSuccess;
  for (int col = 0; col < 27 && e == hipSuccess; ++col) {
    const int cx = col % 3, cy = (col / 3) % 3, cz = col / 9;
    hipLaunchKernelGGL(k_colour, dim3(blocks_for(nvox)), dim3(kT), 0, s, yc, c->G, cx, cy, cz);
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(kT), 0, s, u, nd);
    if ((e = coarse_prolong(*c, yc, u, nullptr, nullptr, s)) != hipSuccess) break;
    if ((e = launch_spmv(pb.A, u, t, s)) != hipSuccess) break;
    hipLaunchKernelGGL(k_probe_collect, dim3(blocks_for(nvox)), dim3(kT), 0, s, t, c->n, c->p,
                       c->n1, c->G, cx, cy, cz, c->Ac);
    e = hipGetLastError();
  }
  const hipError_t es = hipStreamSynchronize(s);
  (void)hipFree(u);
  (void)hipFree(t);
  (void)hipFree(yc);
  FC_HIP(e);
  FC_HIP(es);
  FC_HIP(hipMemsetAsync(c->ls, 0, sizeof(LearnScalars), s));
  FC_HIP(hipStreamSynchronize(s));
  guard.c = nullptr;
  *out = c;
  return FC_OK;
}

}  // namespace fc

using namespace fc;

fc_status fc::coarse_ensure(fc_precond_s& pc, hipStream_t s) {
  if (pc.coarse) return FC_OK;
  CoarseCtx* c = nullptr;
  fc_status st = coarse_create(pc, s, &c);
  if (st != FC_OK) return st;
  pc.coarse = c;
  return FC_OK;
}

// ------------------------------------------------------------ C ABI
namespace {
fc_status ensure_coarse(fc_precond pc, hipStream_t s) { return coarse_ensure(*pc, s); }
}  // namespace

extern "C" {

fc_status fc_learned_attach(fc_precond pc, fc_model m) {
  if (!pc) {
    set_error("fc_learned_attach: NULL preconditioner");
    return FC_E_ARG;
  }
  hipStream_t s = nullptr;
  fc_status st = ensure_coarse(pc, s);
  if (st != FC_OK) return st;
  CoarseCtx& c = *pc->coarse;
  c.ws.release();
  c.model = m;
  c.enabled = 1;
  if (m) {
    st = c.ws.ensure(m->net, 1, c.G);
    if (st != FC_OK) return st;
  }
  // a captured solver chunk holds the old network buffers
  solver_invalidate_graph(*pc);
  FC_HIP(hipMemset(c.ls, 0, sizeof(LearnScalars)));
  FC_HIP(hipDeviceSynchronize());
  return FC_OK;
}

fc_status fc_coarse_grid(fc_precond pc, int32_t* G) {
  if (!pc || !G) return FC_E_ARG;
  fc_status st = ensure_coarse(pc, nullptr);
  if (st != FC_OK) return st;
  *G = pc->coarse->G;
  return FC_OK;
}

fc_status fc_coarse_channels(fc_precond pc, float* eta_dev, float* mask_dev) {
  if (!pc) return FC_E_ARG;
  fc_status st = ensure_coarse(pc, nullptr);
  if (st != FC_OK) return st;
  const CoarseCtx& c = *pc->coarse;
  if (eta_dev)
    FC_HIP(hipMemcpy(eta_dev, c.xin + c.nvox, c.nvox * sizeof(float), hipMemcpyDeviceToDevice));
  if (mask_dev)
    FC_HIP(hipMemcpy(mask_dev, c.mask, c.nvox * sizeof(float), hipMemcpyDeviceToDevice));
  return FC_OK;
}

fc_status fc_coarse_restrict(fc_precond pc, const double* r_dev, double* rc_dev, void* stream) {
  if (!pc || !r_dev || !rc_dev) return FC_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  fc_status st = ensure_coarse(pc, s);
  if (st != FC_OK) return st;
  CoarseCtx& c = *pc->coarse;
  FC_HIP(coarse_restrict(c, r_dev, nullptr, nullptr, s));
  FC_HIP(hipMemcpyAsync(rc_dev, c.rc, c.nvox * sizeof(double), hipMemcpyDeviceToDevice, s));
  return FC_OK;
}

fc_status fc_coarse_prolong(fc_precond pc, const float* y_dev, double gamma, double* z_dev,
                            void* stream) {
  if (!pc || !y_dev || !z_dev) return FC_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  fc_status st = ensure_coarse(pc, s);
  if (st != FC_OK) return st;
  CoarseCtx& c = *pc->coarse;
  FC_HIP(hipMemcpyAsync(&c.ls->gamma, &gamma, sizeof(double), hipMemcpyHostToDevice, s));
  FC_HIP(coarse_prolong(c, y_dev, z_dev, nullptr, nullptr, s));
  FC_HIP(hipStreamSynchronize(s));
  return FC_OK;
}

fc_status fc_coarse_apply(fc_precond pc, const float* y_dev, double* v_dev, double* gamma,
                          void* stream) {
  if (!pc || !y_dev || !v_dev) return FC_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  fc_status st = ensure_coarse(pc, s);
  if (st != FC_OK) return st;
  CoarseCtx& c = *pc->coarse;
  FC_HIP(coarse_gamma(c, y_dev, nullptr, v_dev, s));
  double g = 0.0;
  FC_HIP(hipMemcpyAsync(&g, &c.ls->gamma, sizeof(double), hipMemcpyDeviceToHost, s));
  FC_HIP(hipStreamSynchronize(s));
  if (gamma) *gamma = g;
  return FC_OK;
}

fc_status fc_learned_stats(fc_precond pc, int64_t* n_apply, int64_t* n_drop) {
  if (!pc || !pc->coarse) return FC_E_ARG;
  LearnScalars h;
  FC_HIP(hipMemcpy(&h, pc->coarse->ls, sizeof(h), hipMemcpyDeviceToHost));
  if (n_apply) *n_apply = h.n_apply;
  if (n_drop) *n_drop = h.n_drop;
  return FC_OK;
}

}  // extern "C"
