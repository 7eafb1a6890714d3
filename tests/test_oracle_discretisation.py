"""Pins of the oracle's discretisation against facts fixed by mathematics.

Each test compares the oracle with something it does not compute itself:
closed-form integrals of the integrated Legendre basis, Gauss exactness,
exact energies of linear displacement fields, rigid-body null spaces, areas
and volumes of the immersed geometry, and the optimal L2 convergence rate
p+1 on a manufactured solution.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import fcgen
from oracle import assemble, basis, geometry


def _gauss_matrix(p, f, g, npts=None):
    x, w = basis.gauss(npts or p + 3)
    N, dN = basis.shape_1d(p, x)
    A = {"N": N, "dN": dN}
    return (A[f].T * w) @ A[g]


# ---------------------------------------------------------------- 1-D basis
@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_1d_stiffness_closed_form(p):
    """int N_i' N_j' on [-1,1] is [[1/2,-1/2],[-1/2,1/2]] (+) identity."""
    K = _gauss_matrix(p, "dN", "dN")
    ref = np.zeros((p + 1, p + 1))
    ref[:2, :2] = [[0.5, -0.5], [-0.5, 0.5]]
    ref[2:, 2:] = np.eye(p - 1)
    np.testing.assert_allclose(K, ref, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_1d_mass_closed_form(p):
    """Mass entries of the integrated Legendre functions (by hand)."""
    M = _gauss_matrix(p, "N", "N")
    ref = np.zeros((p + 1, p + 1))
    ref[:2, :2] = [[2 / 3, 1 / 3], [1 / 3, 2 / 3]]
    for j in range(2, p + 1):
        ref[j, j] = 2.0 / ((2 * j - 3) * (2 * j + 1))
    ref[0, 2] = ref[2, 0] = ref[1, 2] = ref[2, 1] = -1.0 / math.sqrt(6.0)
    if p >= 3:
        ref[0, 3] = ref[3, 0] = 1.0 / math.sqrt(90.0)
        ref[1, 3] = ref[3, 1] = -1.0 / math.sqrt(90.0)
    for i in range(2, p - 1):
        v = -1.0 / ((2 * i + 1) * math.sqrt((2 * i - 1) * (2 * i + 3)))
        ref[i, i + 2] = ref[i + 2, i] = v
    np.testing.assert_allclose(M, ref, atol=1e-14)


def test_bubbles_vanish_at_ends():
    N, _ = basis.shape_1d(5, np.array([-1.0, 1.0]))
    np.testing.assert_allclose(N[:, 2:], 0.0, atol=1e-15)
    np.testing.assert_allclose(N[:, :2], [[1, 0], [0, 1]], atol=0)


@pytest.mark.parametrize("npts", [1, 2, 3, 4, 5])
def test_gauss_exactness(npts):
    x, w = basis.gauss(npts)
    for k in range(2 * npts):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


# ------------------------------------------------------- element matrices
def _closed_1d(p, h):
    """Closed-form 1-D stiffness and mass on a cell of width h."""
    K = np.zeros((p + 1, p + 1))
    K[:2, :2] = [[0.5, -0.5], [-0.5, 0.5]]
    K[2:, 2:] = np.eye(p - 1)
    M = _gauss_matrix(p, "N", "N", npts=p + 4)   # pinned above
    return K * 2.0 / h, M * h / 2.0


def _kron_rev(mats):
    """Kronecker product with the first direction fastest."""
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(m, out)
    return out


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 3), (3, 2)])
def test_uncut_scalar_element_is_tensor_product(dim, p):
    n = 4
    desc = fcgen.custom(dim, n, p, "poisson", alpha=1.0, shapes=[])
    Ke, _, eta = assemble.element_system(desc, (1,) * dim)
    K1, M1 = _closed_1d(p, 1.0 / n)
    ref = _kron_rev([M1] * dim)
    for k in range(dim):
        ref = ref + _kron_rev([K1 if j == k else M1 for j in range(dim)])
    np.testing.assert_allclose(Ke, ref, rtol=0, atol=1e-13 * abs(ref).max())
    assert eta == 1.0


def _vertex_interpolant(desc, field):
    """Vector whose vertex unknowns hold field(x_node), bubbles zero."""
    p, d = desc["p"], desc["dim"]
    n1 = assemble.n_nodes_1d(desc)
    nc = assemble.ncomp_of(desc)
    u = np.zeros(assemble.n_dofs(desc))
    h = 1.0 / desc["n"]
    for g in itertools.product(range(n1), repeat=d):
        g = tuple(reversed(g))
        if any(gk % p for gk in g):
            continue
        x = np.array([gk // p * h for gk in g])
        node = sum(gk * n1 ** k for k, gk in enumerate(g))
        u[nc * node: nc * node + nc] = field(x)
    return u


def test_rigid_body_modes_in_nullspace():
    desc = fcgen.custom(3, 2, 2, "elasticity", alpha=1.0, shapes=[],
                        traction=[0, 0, 0], clamp_zmin=False)
    A = assemble.assemble(desc)["A"]
    amax = abs(A).max()
    fields = [lambda x: np.array([1.0, 0, 0]), lambda x: np.array([0, 1.0, 0]),
              lambda x: np.array([0, 0, 1.0]),
              lambda x: np.array([-x[1], x[0], 0.0]),
              lambda x: np.array([0.0, -x[2], x[1]]),
              lambda x: np.array([x[2], 0.0, -x[0]])]
    for f in fields:
        u = _vertex_interpolant(desc, f)
        assert np.linalg.norm(A @ u) <= 1e-13 * amax * np.linalg.norm(u)


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_field_energy(dim):
    """u = G x with symmetric G: u^T A u = lam tr(eps)^2 + 2 mu eps:eps
    times the volume of the unit box."""
    desc = fcgen.custom(dim, 2, 2, "elasticity", alpha=1.0, shapes=[],
                        E=2.5, nu=0.27, traction=[0] * dim)
    A = assemble.assemble(desc)["A"]
    E, nu = 2.5, 0.27
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    rng = np.random.default_rng(3)
    for _ in range(3):
        G = rng.standard_normal((dim, dim))
        eps = 0.5 * (G + G.T)
        u = _vertex_interpolant(desc, lambda x: G @ x)
        exact = lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)
        assert abs(u @ (A @ u) - exact) <= 1e-12 * abs(exact)


def test_traction_load_is_exact_on_linear_fields():
    desc = fcgen.custom(3, 2, 3, "elasticity", alpha=1.0, shapes=[],
                        traction=[0.3, -0.2, -1.0], clamp_zmin=False)
    b = assemble.assemble(desc)["b"]
    # integral over the top face of t . u for u = (1,0,0), (0,x,0), (0,0,y)
    assert abs(b @ _vertex_interpolant(desc, lambda x: np.array([1.0, 0, 0]))
               - 0.3) < 1e-14
    assert abs(b @ _vertex_interpolant(desc, lambda x: np.array([0, x[0], 0]))
               + 0.1) < 1e-14
    assert abs(b @ _vertex_interpolant(desc, lambda x: np.array([0, 0, x[1]]))
               + 0.5) < 1e-14


def test_clamp_rows_and_columns():
    desc = fcgen.custom(3, 2, 2, "elasticity", alpha=1.0, shapes=[],
                        clamp_zmin=True)
    free = fcgen.custom(3, 2, 2, "elasticity", alpha=1.0, shapes=[],
                        clamp_zmin=False)
    A = assemble.assemble(desc)["A"].toarray()
    A0 = assemble.assemble(free)["A"].toarray()
    cd = assemble.clamped_dofs(desc)
    assert cd.size == 3 * 5 * 5
    off = A[cd].copy()
    off[np.arange(cd.size), cd] = 0.0
    assert not off.any()
    np.testing.assert_array_equal(np.diag(A)[cd], np.diag(A0)[cd])
    np.linalg.cholesky(A)


# ------------------------------------------------------------- geometry
def test_disk_area_from_eta():
    desc = fcgen.disk_poisson_2d(0)
    h = 1.0 / desc["n"]
    area = sum(assemble.cell_quadrature(desc, c)[3]
               for c in assemble.cells(desc)) * h * h
    R = desc["shapes"][0]["semi"][0]
    # error per cut leaf is at most its area; leaves are h/8 wide and the
    # number of cut leaves is at most ~2 * perimeter / (h/8)
    bound = 2 * (2 * math.pi * R) / (h / 8) * (h / 8) ** 2
    assert abs(area - math.pi * R * R) < bound
    assert abs(area - math.pi * R * R) < 1e-3 * math.pi * R * R


def test_porous_volume_from_eta():
    desc = fcgen.porous_elasticity_3d(seed=5, n=8, p=1, n_voids=6,
                                      rmin=0.1, rmax=0.2)
    h = 1.0 / desc["n"]
    vol = sum(assemble.cell_quadrature(desc, c)[3]
              for c in assemble.cells(desc)) * h ** 3
    exact = 1.0 - sum(4.0 / 3.0 * math.pi * s["semi"][0] ** 3
                      for s in desc["shapes"])
    assert abs(vol - exact) < 2e-3


def test_box_classification_exact():
    desc = fcgen.custom(2, 4, 1, shapes=[{"centre": [0.5, 0.5],
                                          "semi": [0.2, 0.1]}],
                        domain="voids")
    assert geometry.classify_box(desc, [0.45, 0.48], [0.55, 0.52]) == geometry.FICT
    assert geometry.classify_box(desc, [0.0, 0.0], [0.2, 0.2]) == geometry.PHYS
    assert geometry.classify_box(desc, [0.5, 0.5], [0.8, 0.8]) == geometry.CUT
    # a box touching the ellipse only beyond its semi-axis in y stays physical
    assert geometry.classify_box(desc, [0.45, 0.61], [0.55, 0.7]) == geometry.PHYS


def test_eta_is_exactly_one_or_zero_on_uncut_cells():
    desc = fcgen.porous_elasticity_3d(seed=1, n=4, p=1, n_voids=2,
                                      rmin=0.05, rmax=0.08)
    h = 1.0 / desc["n"]
    for c in assemble.cells(desc):
        lo = np.array(c) * h
        st = geometry.classify_box(desc, lo, lo + h)
        eta = assemble.cell_quadrature(desc, c)[3]
        if st == geometry.PHYS:
            assert eta == 1.0
        elif st == geometry.FICT:
            assert eta == 0.0


# ------------------------------------------------ manufactured solution
def _l2_error_cos(desc, x):
    """L2 error of u_h against u = cos(pi x) cos(pi y) (cos(pi z))."""
    err2 = 0.0
    d, p = desc["dim"], desc["p"]
    h = 1.0 / desc["n"]
    for c in assemble.cells(desc):
        lo = np.array(c) * h
        pts, w = basis.tensor_rule(p + 3, lo, lo + h)
        N, _ = assemble.element_basis(desc, c, pts)
        uh = N @ x[assemble.element_dofs(desc, c)]
        u = np.prod(np.cos(np.pi * pts), axis=1)
        err2 += np.sum(w * (uh - u) ** 2)
    return math.sqrt(err2)


def _cos_modes(dim):
    """cos(pi x)cos(pi y)[cos(pi z)] as a sum of cos(2 pi k.x) with
    half-integer k, times (1 + dim pi^2): the load of -lap u + u = f."""
    c = 1.0 + dim * math.pi ** 2
    modes = []
    for signs in itertools.product([1, -1], repeat=dim - 1):
        k = [0.5] + [0.5 * s for s in signs]
        modes.append({"k": k, "amp": c / 2 ** (dim - 1), "phase": 0.0})
    return modes


@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_l2_rate_2d(p):
    errs = []
    for n in (2, 4, 8):
        desc = fcgen.custom(2, n, p, "poisson", alpha=1.0, shapes=[],
                            modes=_cos_modes(2))
        s = assemble.assemble(desc)
        x = scipy.linalg.solve(s["A"].toarray(), s["b"], assume_a="pos")
        errs.append(_l2_error_cos(desc, x))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] > p + 1 - 0.25, (errs, rates)


def test_manufactured_l2_rate_3d():
    p = 2
    errs = []
    for n in (2, 4):
        desc = fcgen.custom(3, n, p, "poisson", alpha=1.0, shapes=[],
                            modes=_cos_modes(3))
        s = assemble.assemble(desc)
        x = scipy.linalg.solve(s["A"].toarray(), s["b"], assume_a="pos")
        errs.append(_l2_error_cos(desc, x))
    assert math.log2(errs[0] / errs[1]) > p + 1 - 0.35, errs


# ------------------------------------------------------- global system
def test_config1_system_symmetric_positive_definite():
    desc = fcgen.disk_poisson_2d(0)
    s = assemble.assemble(desc)
    A = s["A"]
    assert A.shape == (1089, 1089)
    assert abs(A - A.T).max() == 0.0 or abs(A - A.T).max() < 1e-15 * abs(A).max()
    np.linalg.cholesky(A.toarray())


def test_cut_elasticity_system_symmetric_positive_definite():
    desc = fcgen.porous_elasticity_3d(seed=2, n=3, p=2, n_voids=2,
                                      rmin=0.1, rmax=0.15)
    s = assemble.assemble(desc)
    A = s["A"].toarray()
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-15 * abs(A).max())
    np.linalg.cholesky(A)
    assert (s["eta"] < 1).any() and (s["eta"] > 0).any()


def test_discard_fictitious_removes_exactly_the_functions_of_void_cells():
    """With discard_fictitious the functions that touch no cell with
    physical material (found here by brute force over the cells of each
    unknown) keep only their diagonal entry and get no load; every other
    entry of A and b is unchanged."""
    import fcgen
    from oracle import assemble as ASM
    void = [{"centre": [0.5, 0.52, 0.48], "semi": [0.33, 0.33, 0.33]}]
    base = fcgen.custom(3, 6, 2, "poisson", 1e-6, shapes=void)
    disc = dict(base, discard_fictitious=True)
    s1, s2 = ASM.assemble(base), ASM.assemble(disc)
    A1, A2 = s1["A"].toarray(), s2["A"].toarray()
    n = A1.shape[0]
    cells_of = [[] for _ in range(n)]
    for c, dofs in enumerate(s1["elem_dofs"]):
        for d in dofs:
            cells_of[d].append(c)
    gone = np.array([all(s1["eta"][c] == 0.0 for c in cells_of[d]) for d in range(n)])
    assert 0 < gone.sum() < n
    keep = ~gone
    assert np.array_equal(A2[np.ix_(keep, keep)], A1[np.ix_(keep, keep)])
    assert np.all(A2[np.ix_(gone, keep)] == 0.0) and np.all(A2[np.ix_(keep, gone)] == 0.0)
    sub = A2[np.ix_(gone, gone)]
    assert np.array_equal(sub, np.diag(np.diag(A1)[gone]))
    assert np.all(s2["b"][gone] == 0.0) and np.array_equal(s2["b"][keep], s1["b"][keep])
