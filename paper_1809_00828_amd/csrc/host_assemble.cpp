// Host-side finite cell assembly (Sec. 2.1, Eq. 1; cut-cell integration of
// Sec. 5.1) into the row-SoA BSR layout consumed by the device kernels.
//
// Weak forms, with the indicator alpha weighting every volume term:
//   Poisson     a(u,v) = int alpha (grad u . grad v + u v),  l(v) = int alpha f v
//   elasticity  a(u,v) = int alpha eps(v):C:eps(u),        l(v) = int_top t.v
// Elasticity is assembled from the gradient moments
//   G^{kl}_{ab} = int alpha dN_a/dx_k dN_b/dx_l
// as K[(a,i),(b,j)] = lam G^{ij}_{ab} + mu G^{ji}_{ab} + mu delta_ij sum_k G^{kk}_{ab}.
// Boxes on which alpha is constant (uncut cells and uncut tree leaves) are
// integrated by sum factorisation of 1-D Gauss moments; leaves of the cut
// tree at full depth are integrated point by point with alpha evaluated at
// each Gauss point.  The basis is the integrated Legendre family
// N_0 = (1-xi)/2, N_1 = (1+xi)/2, N_j = (P_j - P_{j-2})/sqrt(2(2j-1)).
#include "host_assemble.h"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>

namespace fc {

int host_threads() {
  static int nt = [] {
    const char* e = std::getenv("FC_HOST_THREADS");
    int v = e ? std::atoi(e) : 0;
    if (v <= 0) v = (int)std::thread::hardware_concurrency();
    if (v <= 0) v = 1;
    return std::min(v, 64);
  }();
  return nt;
}

namespace {

constexpr int kMaxDim = 3;
constexpr int kMaxP = 8;

// ---------------------------------------------------------------- basis
// Legendre P_0..P_{p} at xi by the three-term recurrence.
void legendre_all(int p, double xi, double* P) {
  P[0] = 1.0;
  if (p >= 1) P[1] = xi;
  for (int j = 1; j < p; ++j)
    P[j + 1] = ((2.0 * j + 1.0) * xi * P[j] - j * P[j - 1]) / (j + 1.0);
}

// Shape values N[0..p] and xi-derivatives dN[0..p].
void shape1d(int p, double xi, double* N, double* dN) {
  double P[kMaxP + 2];
  legendre_all(p, xi, P);
  N[0] = 0.5 * (1.0 - xi);
  N[1] = 0.5 * (1.0 + xi);
  dN[0] = -0.5;
  dN[1] = 0.5;
  for (int j = 2; j <= p; ++j) {
    double s = std::sqrt(2.0 * (2.0 * j - 1.0));
    N[j] = (P[j] - P[j - 2]) / s;
    dN[j] = (2.0 * j - 1.0) * P[j - 1] / s;   // (P_j - P_{j-2})' = (2j-1) P_{j-1}
  }
}

// Gauss-Legendre rule on [-1,1] by Newton iteration on P_n.
void gauss_rule(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 1; j < n; ++j) {
        double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 0) ? 1.0 : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 1; j < n; ++j) {
      double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
      p0 = p1;
      p1 = p2;
    }
    double pm = (n == 1) ? 1.0 : p0;
    dp = n * (z * p1 - pm) / (z * z - 1.0);
    x[n - 1 - i] = z;                      // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// ------------------------------------------------------------- geometry
enum BoxState { kPhys = 0, kFict = 1, kCut = 2 };

struct Geometry {
  int dim = 2;
  bool voids = true;
  int ns = 0;
  std::vector<double> c, s;   // [ns*dim]

  bool inside_any(const double* x) const {
    for (int k = 0; k < ns; ++k) {
      double r2 = 0.0;
      for (int j = 0; j < dim; ++j) {
        double u = (x[j] - c[k * dim + j]) / s[k * dim + j];
        r2 += u * u;
      }
      if (r2 <= 1.0) return true;
    }
    return false;
  }
  bool physical(const double* x) const {
    bool in = inside_any(x);
    return voids ? !in : in;
  }
  // Exact classification of [lo, hi] in coordinates scaled by the semi-axes.
  int classify(const double* lo, const double* hi) const {
    bool in_some = false, out_all = true;
    for (int k = 0; k < ns; ++k) {
      double dmin2 = 0.0, dmax2 = 0.0;
      for (int j = 0; j < dim; ++j) {
        double ul = (lo[j] - c[k * dim + j]) / s[k * dim + j];
        double uh = (hi[j] - c[k * dim + j]) / s[k * dim + j];
        double nr = std::min(std::max(0.0, ul), uh);
        dmin2 += nr * nr;
        dmax2 += std::max(ul * ul, uh * uh);
      }
      if (dmax2 <= 1.0) in_some = true;
      if (!(dmin2 > 1.0)) out_all = false;
    }
    if (voids) {
      if (in_some) return kFict;
      return out_all ? kPhys : kCut;
    }
    if (in_some) return kPhys;
    return out_all ? kFict : kCut;
  }
};

struct Box {
  double lo[kMaxDim], hi[kMaxDim];
  int state;
};

void tree_leaves(const Geometry& g, const double* lo, const double* hi, int depth,
                 std::vector<Box>& out) {
  int st = g.classify(lo, hi);
  if (st != kCut || depth == 0) {
    Box b;
    for (int j = 0; j < g.dim; ++j) {
      b.lo[j] = lo[j];
      b.hi[j] = hi[j];
    }
    b.state = st;
    out.push_back(b);
    return;
  }
  double mid[kMaxDim];
  for (int j = 0; j < g.dim; ++j) mid[j] = 0.5 * (lo[j] + hi[j]);
  for (int corner = 0; corner < (1 << g.dim); ++corner) {
    double clo[kMaxDim], chi[kMaxDim];
    for (int j = 0; j < g.dim; ++j) {
      if ((corner >> j) & 1) {
        clo[j] = mid[j];
        chi[j] = hi[j];
      } else {
        clo[j] = lo[j];
        chi[j] = mid[j];
      }
    }
    tree_leaves(g, clo, chi, depth - 1, out);
  }
}

// ------------------------------------------------------- element kernels
struct Ctx {
  int dim, p, n, q, nn, ncomp, m;
  double h, alpha, lam, mu;
  bool elastic;
  std::vector<double> gx, gw;            // Gauss rule, q = p+1 points
  Geometry geo;
  std::vector<double> mk, ma, mph;       // load modes
  int nmodes = 0;
  int depth = 3;
  double traction[3];
};

// Local node a -> per-direction local indices.
inline void split_local(int a, int p, int dim, int* ak) {
  for (int k = 0; k < dim; ++k) {
    ak[k] = a % (p + 1);
    a /= (p + 1);
  }
}

// Gradient moments on a box where alpha is constant, by sum factorisation.
// Gkl has (dim*dim) matrices nn x nn: index (k*dim+l)*nn*nn + a*nn + b.
// Mass moment M (nn x nn) for the scalar problem.
void box_moments_sumfact(const Ctx& C, const double* x0, const Box& bx,
                         double alpha, double* Gkl, double* M) {
  const int p1 = C.p + 1, nn = C.nn, dim = C.dim;
  // 1-D moments per direction: K1 (D,D), M1 (V,V), E1 (D,V)
  double K1[kMaxDim][(kMaxP + 1) * (kMaxP + 1)];
  double M1[kMaxDim][(kMaxP + 1) * (kMaxP + 1)];
  double E1[kMaxDim][(kMaxP + 1) * (kMaxP + 1)];
  for (int k = 0; k < dim; ++k) {
    std::memset(K1[k], 0, sizeof(K1[k]));
    std::memset(M1[k], 0, sizeof(M1[k]));
    std::memset(E1[k], 0, sizeof(E1[k]));
    double len = bx.hi[k] - bx.lo[k];
    for (int i = 0; i < C.q; ++i) {
      double x = bx.lo[k] + 0.5 * (C.gx[i] + 1.0) * len;
      double w = 0.5 * len * C.gw[i];
      double xi = 2.0 * (x - x0[k]) / C.h - 1.0;
      double N[kMaxP + 1], dN[kMaxP + 1];
      shape1d(C.p, xi, N, dN);
      for (int a = 0; a < p1; ++a) dN[a] *= 2.0 / C.h;
      for (int a = 0; a < p1; ++a)
        for (int b = 0; b < p1; ++b) {
          K1[k][a * p1 + b] += w * dN[a] * dN[b];
          M1[k][a * p1 + b] += w * N[a] * N[b];
          E1[k][a * p1 + b] += w * dN[a] * N[b];
        }
    }
  }
  int ak[kMaxDim], bk[kMaxDim];
  for (int a = 0; a < nn; ++a) {
    split_local(a, C.p, dim, ak);
    for (int b = 0; b < nn; ++b) {
      split_local(b, C.p, dim, bk);
      if (M) {
        double v = alpha;
        for (int j = 0; j < dim; ++j) v *= M1[j][ak[j] * p1 + bk[j]];
        M[a * nn + b] += v;
      }
      for (int k = 0; k < dim; ++k)
        for (int l = 0; l < dim; ++l) {
          if (!C.elastic && k != l) continue;
          double v = alpha;
          for (int j = 0; j < dim; ++j) {
            int ij = ak[j] * p1 + bk[j];
            int ji = bk[j] * p1 + ak[j];
            double f;
            if (j == k && j == l) f = K1[j][ij];
            else if (j == k) f = E1[j][ij];          // dN_a, N_b
            else if (j == l) f = E1[j][ji];          // N_a, dN_b
            else f = M1[j][ij];
            v *= f;
          }
          Gkl[(k * dim + l) * nn * nn + a * nn + b] += v;
        }
    }
  }
}

// Tensor shape values and physical gradients at one point.
void point_basis(const Ctx& C, const double* x0, const double* x, double* N,
                 double* dN /* [dim][nn] */) {
  const int p1 = C.p + 1, dim = C.dim, nn = C.nn;
  double V[kMaxDim][kMaxP + 1], D[kMaxDim][kMaxP + 1];
  for (int k = 0; k < dim; ++k) {
    double xi = 2.0 * (x[k] - x0[k]) / C.h - 1.0;
    shape1d(C.p, xi, V[k], D[k]);
    for (int a = 0; a < p1; ++a) D[k][a] *= 2.0 / C.h;
  }
  int ak[kMaxDim];
  for (int a = 0; a < nn; ++a) {
    split_local(a, C.p, dim, ak);
    double v = 1.0;
    for (int j = 0; j < dim; ++j) v *= V[j][ak[j]];
    N[a] = v;
    for (int k = 0; k < dim; ++k) {
      double g = 1.0;
      for (int j = 0; j < dim; ++j) g *= (j == k) ? D[j][ak[j]] : V[j][ak[j]];
      dN[k * nn + a] = g;
    }
  }
}

// Gauss points of a box (first direction fastest).
void box_points(const Ctx& C, const Box& bx, std::vector<double>& pts,
                std::vector<double>& wts) {
  int np = 1;
  for (int k = 0; k < C.dim; ++k) np *= C.q;
  pts.resize((size_t)np * C.dim);
  wts.resize(np);
  for (int t = 0; t < np; ++t) {
    int r = t;
    double w = 1.0;
    for (int k = 0; k < C.dim; ++k) {
      int i = r % C.q;
      r /= C.q;
      double len = bx.hi[k] - bx.lo[k];
      pts[(size_t)t * C.dim + k] = bx.lo[k] + 0.5 * (C.gx[i] + 1.0) * len;
      w *= 0.5 * len * C.gw[i];
    }
    wts[t] = w;
  }
}

double load_f(const Ctx& C, const double* x) {
  double f = 0.0;
  for (int k = 0; k < C.nmodes; ++k) {
    double kx = 0.0;
    for (int j = 0; j < C.dim; ++j) kx += C.mk[k * C.dim + j] * x[j];
    f += C.ma[k] * std::cos(2.0 * M_PI * kx + C.mph[k]);
  }
  return f;
}

// Convert gradient/mass moments into the element matrix Ke (m x m).
void moments_to_Ke(const Ctx& C, const double* Gkl, const double* M, double* Ke) {
  const int nn = C.nn, dim = C.dim, m = C.m;
  if (!C.elastic) {
    for (int a = 0; a < nn; ++a)
      for (int b = 0; b < nn; ++b) {
        double v = M[a * nn + b];
        for (int k = 0; k < dim; ++k) v += Gkl[(k * dim + k) * nn * nn + a * nn + b];
        Ke[a * m + b] = v;
      }
    return;
  }
  for (int a = 0; a < nn; ++a)
    for (int b = 0; b < nn; ++b) {
      double tr = 0.0;
      for (int k = 0; k < dim; ++k) tr += Gkl[(k * dim + k) * nn * nn + a * nn + b];
      for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
          double gij = Gkl[(i * dim + j) * nn * nn + a * nn + b];
          double gji = Gkl[(j * dim + i) * nn * nn + a * nn + b];
          double v = C.lam * gij + C.mu * gji + (i == j ? C.mu * tr : 0.0);
          Ke[(a * dim + i) * m + (b * dim + j)] = v;
        }
    }
}

struct CellResult {
  std::vector<double> Ke;     // element matrix of a cut cell (m x m)
  std::vector<double> fe;     // element volume load (m)
  double eta = 0.0;
  int kind = 0;               // 0 uncut physical, 1 uncut fictitious, 2 cut
};

// Element matrix (cut cells), volume load and eta_T of one cell.  eta_T is
// the fraction of the cell's quadrature weight at physical points, so it is
// exactly 1 (0) when every point is physical (fictitious).
void cell_compute(const Ctx& C, const int* cell, CellResult& R) {
  const int nn = C.nn, dim = C.dim, m = C.m;
  const size_t nn2 = (size_t)nn * nn;
  double x0[kMaxDim], hi[kMaxDim];
  for (int k = 0; k < dim; ++k) {
    x0[k] = cell[k] * C.h;
    hi[k] = x0[k] + C.h;
  }
  std::vector<Box> leaves;
  tree_leaves(C.geo, x0, hi, C.depth, leaves);
  const bool uncut = leaves.size() == 1 && leaves[0].state != kCut;

  std::vector<double> pts, wts, N(nn), dN((size_t)dim * nn);
  double wphys = 0.0, wall = 0.0;
  R.fe.assign(m, 0.0);
  std::vector<double> G, Gp, M;
  if (!uncut) {
    G.assign((size_t)dim * dim * nn2, 0.0);
    Gp.assign((size_t)dim * dim * nn2, 0.0);
    M.assign(nn2, 0.0);
  }
  const bool scalar_load = !C.elastic && C.nmodes > 0;
  for (const Box& bx : leaves) {
    box_points(C, bx, pts, wts);
    const int np = (int)wts.size();
    const bool pointwise = !uncut && bx.state == kCut;
    if (!uncut && !pointwise)
      box_moments_sumfact(C, x0, bx, bx.state == kPhys ? 1.0 : C.alpha, G.data(),
                          C.elastic ? nullptr : M.data());
    for (int t = 0; t < np; ++t) {
      const double* x = &pts[(size_t)t * dim];
      const bool phys = C.geo.physical(x);
      wall += wts[t];
      if (phys) wphys += wts[t];
      if (!pointwise && !scalar_load) continue;
      const double wa = wts[t] * (phys ? 1.0 : C.alpha);
      point_basis(C, x0, x, N.data(), dN.data());
      if (scalar_load) {
        double f = wa * load_f(C, x);
        for (int a = 0; a < nn; ++a) R.fe[a] += f * N[a];
      }
      if (!pointwise) continue;
      if (!C.elastic) {
        for (int a = 0; a < nn; ++a) {
          double ca = wa * N[a];
          double* Mr = &M[(size_t)a * nn];
          for (int b = 0; b < nn; ++b) Mr[b] += ca * N[b];
        }
      }
      for (int k = 0; k < dim; ++k)
        for (int l = k; l < dim; ++l) {
          if (!C.elastic && l != k) continue;
          double* Gr = &Gp[(size_t)(k * dim + l) * nn2];
          const double* dk = &dN[(size_t)k * nn];
          const double* dl = &dN[(size_t)l * nn];
          for (int a = 0; a < nn; ++a) {
            double ca = wa * dk[a];
            double* row = Gr + (size_t)a * nn;
            for (int b = 0; b < nn; ++b) row[b] += ca * dl[b];
          }
        }
    }
  }
  R.eta = wphys / wall;
  if (uncut) {
    R.kind = leaves[0].state == kPhys ? 0 : 1;
    return;
  }
  R.kind = 2;
  // pointwise moments were accumulated for k <= l; G^{lk}_{ab} = G^{kl}_{ba}
  for (int k = 0; k < dim; ++k)
    for (int l = k; l < dim; ++l) {
      if (!C.elastic && l != k) continue;
      const double* src = &Gp[(size_t)(k * dim + l) * nn2];
      double* dkl = &G[(size_t)(k * dim + l) * nn2];
      for (size_t t = 0; t < nn2; ++t) dkl[t] += src[t];
      if (k == l) continue;
      double* dlk = &G[(size_t)(l * dim + k) * nn2];
      for (int a = 0; a < nn; ++a)
        for (int b = 0; b < nn; ++b) dlk[(size_t)a * nn + b] += src[(size_t)b * nn + a];
    }
  R.Ke.assign((size_t)m * m, 0.0);
  moments_to_Ke(C, G.data(), M.data(), R.Ke.data());
}

// Traction load of a cell touching x_{dim-1} = 1 (elasticity only).
void traction_load(const Ctx& C, const int* cell, double* fe) {
  const int dim = C.dim, nn = C.nn;
  double x0[kMaxDim];
  for (int k = 0; k < dim; ++k) x0[k] = cell[k] * C.h;
  int nf = 1;
  for (int k = 0; k < dim - 1; ++k) nf *= C.q;
  std::vector<double> N(nn), dN((size_t)dim * nn);
  for (int t = 0; t < nf; ++t) {
    int r = t;
    double x[kMaxDim], w = 1.0;
    for (int k = 0; k < dim - 1; ++k) {
      int i = r % C.q;
      r /= C.q;
      x[k] = x0[k] + 0.5 * (C.gx[i] + 1.0) * C.h;
      w *= 0.5 * C.h * C.gw[i];
    }
    x[dim - 1] = 1.0;
    point_basis(C, x0, x, N.data(), dN.data());
    for (int a = 0; a < nn; ++a)
      for (int c = 0; c < dim; ++c) fe[a * dim + c] += C.traction[c] * w * N[a];
  }
}

// Local 1-D index -> global 1-D index on cell e.
inline int l2g(int p, int e, int a) { return a == 0 ? p * e : (a == 1 ? p * e + p : p * e + a - 1); }

}  // namespace

fc_status assemble_host(const fc_problem_desc& d, HostSystem* out, std::string* err) {
  if (d.dim < 2 || d.dim > 3 || d.n < 1 || d.p < 1 || d.p > kMaxP ||
      d.quad_depth < 0 || d.quad_depth > 16 || d.n_shapes < 0 || d.n_modes < 0 ||
      (d.pde != FC_PDE_POISSON && d.pde != FC_PDE_ELASTICITY) ||
      (d.domain != FC_DOMAIN_VOIDS && d.domain != FC_DOMAIN_INCLUSIONS) ||
      !(d.alpha >= 0.0)) {
    *err = "invalid problem description";
    return FC_E_ARG;
  }
  if ((d.n_shapes > 0 && (!d.shape_centre || !d.shape_semi)) ||
      (d.n_modes > 0 && (!d.mode_k || !d.mode_amp || !d.mode_phase))) {
    *err = "missing shape or mode arrays";
    return FC_E_ARG;
  }
  for (int k = 0; k < d.n_shapes * d.dim; ++k)
    if (!(d.shape_semi[k] > 0.0)) {
      *err = "shape semi-axes must be positive";
      return FC_E_ARG;
    }
  Ctx C;
  C.dim = d.dim;
  C.p = d.p;
  C.n = d.n;
  C.q = d.p + 1;
  C.elastic = d.pde == FC_PDE_ELASTICITY;
  C.ncomp = C.elastic ? d.dim : 1;
  C.nn = 1;
  for (int k = 0; k < d.dim; ++k) C.nn *= (d.p + 1);
  C.m = C.ncomp * C.nn;
  C.h = 1.0 / d.n;
  C.alpha = d.alpha;
  C.lam = d.E * d.nu / ((1.0 + d.nu) * (1.0 - 2.0 * d.nu));
  C.mu = d.E / (2.0 * (1.0 + d.nu));
  C.depth = d.quad_depth;
  C.gx.resize(C.q);
  C.gw.resize(C.q);
  gauss_rule(C.q, C.gx.data(), C.gw.data());
  C.geo.dim = d.dim;
  C.geo.voids = d.domain == FC_DOMAIN_VOIDS;
  C.geo.ns = d.n_shapes;
  C.geo.c.assign(d.shape_centre, d.shape_centre + (size_t)d.n_shapes * d.dim);
  C.geo.s.assign(d.shape_semi, d.shape_semi + (size_t)d.n_shapes * d.dim);
  if (!C.elastic) {
    C.nmodes = d.n_modes;
    C.mk.assign(d.mode_k, d.mode_k + (size_t)d.n_modes * d.dim);
    C.ma.assign(d.mode_amp, d.mode_amp + d.n_modes);
    C.mph.assign(d.mode_phase, d.mode_phase + d.n_modes);
  }
  for (int k = 0; k < 3; ++k) C.traction[k] = d.traction[k];

  const int dim = C.dim, p = C.p, n = C.n, nn = C.nn, m = C.m, bd = C.ncomp;
  const int bb = bd * bd;
  const int64_t n1 = (int64_t)p * n + 1;
  int64_t n_nodes = 1, n_el = 1;
  for (int k = 0; k < dim; ++k) {
    n_nodes *= n1;
    n_el *= n;
  }
  if (n_nodes * bd >= (int64_t(1) << 31)) {
    *err = "too many unknowns for int32 indices";
    return FC_E_UNSUPPORTED;
  }

  // reference matrix of an uncut cell with alpha = 1
  std::vector<double> Kref((size_t)m * m, 0.0);
  {
    std::vector<double> G((size_t)dim * dim * nn * nn, 0.0), M((size_t)nn * nn, 0.0);
    Box bx;
    double x0[kMaxDim] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
      bx.lo[k] = 0.0;
      bx.hi[k] = C.h;
    }
    bx.state = kPhys;
    box_moments_sumfact(C, x0, bx, 1.0, G.data(), C.elastic ? nullptr : M.data());
    moments_to_Ke(C, G.data(), M.data(), Kref.data());
  }

  // per-cell element data
  std::vector<CellResult> res(n_el);
  parallel_for(n_el, [&](int64_t e) {
    int cell[kMaxDim];
    int64_t r = e;
    for (int k = 0; k < dim; ++k) {
      cell[k] = (int)(r % n);
      r /= n;
    }
    cell_compute(C, cell, res[e]);
    if (C.elastic && cell[dim - 1] == n - 1) traction_load(C, cell, res[e].fe.data());
  });

  HostSystem& S = *out;
  S.dim = dim;
  S.n = n;
  S.p = p;
  S.bdim = bd;
  S.nn = nn;
  S.m = m;
  S.n_nodes = n_nodes;
  S.n_dofs = n_nodes * bd;
  S.n_el = n_el;

  // element nodes, element-local order (a_0 fastest)
  S.elem_nodes.resize((size_t)n_el * nn);
  S.eta.resize(n_el);
  for (int64_t e = 0; e < n_el; ++e) {
    int cell[kMaxDim];
    int64_t r = e;
    for (int k = 0; k < dim; ++k) {
      cell[k] = (int)(r % n);
      r /= n;
    }
    for (int a = 0; a < nn; ++a) {
      int ak[kMaxDim];
      split_local(a, p, dim, ak);
      int64_t node = 0, stride = 1;
      for (int k = 0; k < dim; ++k) {
        node += (int64_t)l2g(p, cell[k], ak[k]) * stride;
        stride *= n1;
      }
      S.elem_nodes[(size_t)e * nn + a] = (int32_t)node;
    }
    S.eta[e] = res[e].eta;
  }

  // 1-D column range of global index g
  auto range1d = [&](int64_t g, int64_t* lo, int64_t* hi) {
    if (g % p == 0) {
      *lo = std::max<int64_t>(0, g - p);
      *hi = std::min<int64_t>(n1 - 1, g + p);
    } else {
      int64_t e = g / p;
      *lo = p * e;
      *hi = p * e + p;
    }
  };
  // row pattern
  S.rowptr.assign(n_nodes + 1, 0);
  for (int64_t nd = 0; nd < n_nodes; ++nd) {
    int64_t r = nd, L = 1;
    for (int k = 0; k < dim; ++k) {
      int64_t g = r % n1, lo, hi;
      r /= n1;
      range1d(g, &lo, &hi);
      L *= (hi - lo + 1);
    }
    S.rowptr[nd + 1] = (int32_t)L;
  }
  for (int64_t nd = 0; nd < n_nodes; ++nd) {
    int64_t next = (int64_t)S.rowptr[nd] + S.rowptr[nd + 1];
    if (next >= (int64_t(1) << 31)) {
      *err = "too many matrix blocks for int32 indices";
      return FC_E_UNSUPPORTED;
    }
    S.rowptr[nd + 1] = (int32_t)next;
  }
  const int64_t nnzb = S.rowptr[n_nodes];
  S.col.resize(nnzb);
  S.val.assign((size_t)nnzb * bb, 0.0);

  const bool clamp = d.clamp_zmin != 0;
  // functions that touch no cell with physical material: removed in place
  // (rows and columns zeroed, diagonal kept) when the description asks
  const bool discard = d.discard_fictitious != 0;
  std::vector<uint8_t> gone;
  if (discard) {
    gone.assign(n_nodes, 1);
    for (int64_t e = 0; e < n_el; ++e)
      if (res[e].eta > 0.0)
        for (int a = 0; a < nn; ++a) gone[S.elem_nodes[(size_t)e * nn + a]] = 0;
  }
  parallel_for(n_nodes, [&](int64_t nd) {
    int64_t g[kMaxDim], lo[kMaxDim], hi[kMaxDim], len[kMaxDim];
    int64_t r = nd;
    for (int k = 0; k < dim; ++k) {
      g[k] = r % n1;
      r /= n1;
      range1d(g[k], &lo[k], &hi[k]);
      len[k] = hi[k] - lo[k] + 1;
    }
    const int64_t base = S.rowptr[nd];
    const int64_t L = S.rowptr[nd + 1] - base;
    // columns: last direction outermost so node ids increase
    for (int64_t t = 0; t < L; ++t) {
      int64_t rr = t, col = 0, stride = 1;
      for (int k = 0; k < dim; ++k) {
        col += (lo[k] + rr % len[k]) * stride;
        rr /= len[k];
        stride *= n1;
      }
      S.col[base + t] = (int32_t)col;
    }
    double* V = &S.val[(size_t)base * bb];
    // cells containing this node, increasing cell index
    int64_t clo[kMaxDim], chi[kMaxDim];
    for (int k = 0; k < dim; ++k) {
      if (g[k] % p == 0) {
        clo[k] = std::max<int64_t>(0, g[k] / p - 1);
        chi[k] = std::min<int64_t>(n - 1, g[k] / p);
      } else {
        clo[k] = chi[k] = g[k] / p;
      }
    }
    int64_t ncell = 1, cl[kMaxDim];
    for (int k = 0; k < dim; ++k) ncell *= (chi[k] - clo[k] + 1);
    for (int64_t t = 0; t < ncell; ++t) {
      int64_t rr = t, cidx = 0, cstride = 1;
      for (int k = 0; k < dim; ++k) {
        int64_t w = chi[k] - clo[k] + 1;
        cl[k] = clo[k] + rr % w;
        rr /= w;
        cidx += cl[k] * cstride;
        cstride *= n;
      }
      const CellResult& cr = res[cidx];
      const double* K = cr.kind == 2 ? cr.Ke.data() : Kref.data();
      const double scale = cr.kind == 2 ? 1.0 : (cr.kind == 0 ? 1.0 : C.alpha);
      // local index of this node in the cell
      int a = 0, astride = 1;
      for (int k = 0; k < dim; ++k) {
        int64_t off = g[k] - (int64_t)p * cl[k];
        int ak = off == 0 ? 0 : (off == p ? 1 : (int)off + 1);
        a += ak * astride;
        astride *= (p + 1);
      }
      for (int b = 0; b < nn; ++b) {
        int bk[kMaxDim];
        split_local(b, p, dim, bk);
        int64_t pos = 0, pstride = 1;
        for (int k = 0; k < dim; ++k) {
          int64_t gb = l2g(p, (int)cl[k], bk[k]);
          pos += (gb - lo[k]) * pstride;
          pstride *= len[k];
        }
        for (int i = 0; i < bd; ++i)
          for (int j = 0; j < bd; ++j)
            V[(size_t)(i * bd + j) * L + pos] += scale * K[(size_t)(a * bd + i) * m + (b * bd + j)];
      }
    }
    if (clamp || discard) {
      const bool row_cl = (clamp && g[dim - 1] == 0) || (discard && gone[nd]);
      for (int64_t t = 0; t < L; ++t) {
        int64_t cnode = S.col[base + t];
        int64_t gz = cnode;
        for (int k = 0; k < dim - 1; ++k) gz /= n1;
        const bool col_cl = (clamp && gz == 0) || (discard && gone[cnode]);
        if (!row_cl && !col_cl) continue;
        for (int i = 0; i < bd; ++i)
          for (int j = 0; j < bd; ++j)
            if (!(cnode == nd && i == j)) V[(size_t)(i * bd + j) * L + t] = 0.0;
      }
    }
  });

  // load vector
  S.rhs.assign(S.n_dofs, 0.0);
  for (int64_t e = 0; e < n_el; ++e)
    for (int a = 0; a < nn; ++a) {
      int64_t node = S.elem_nodes[(size_t)e * nn + a];
      for (int c = 0; c < bd; ++c) S.rhs[node * bd + c] += res[e].fe[(size_t)a * bd + c];
    }
  if (clamp) {
    int64_t plane = 1;
    for (int k = 0; k < dim - 1; ++k) plane *= n1;
    for (int64_t nd = 0; nd < plane; ++nd)
      for (int c = 0; c < bd; ++c) S.rhs[nd * bd + c] = 0.0;
  }
  if (discard)
    for (int64_t nd = 0; nd < n_nodes; ++nd)
      if (gone[nd])
        for (int c = 0; c < bd; ++c) S.rhs[nd * bd + c] = 0.0;
  return FC_OK;
}

}  // namespace fc
