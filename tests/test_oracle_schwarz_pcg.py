"""Pins of the oracle's Schwarz preconditioner and PCG.

Checked against what the paper and linear algebra fix: the single all-DOF
block gives S = A^-1 and one CG step (Sec. 3.1), one-function blocks give
Jacobi (Sec. 3.1), the pseudo-inverse identities of Eqs. (9)-(11), block
size (p+1)^d and overlap 2^d on uniform grids (Sec. 3.2; the gearbox table
at refinement depth 0), the diagonal-scaling fallback of Algorithm 1, dense
direct solves, CG's conjugacy and monotone energy error, and the paper's
robustness claim: Schwarz iterations stay bounded as a cut cell shrinks
while Jacobi's grow (Sec. 3.1, remark; Sec. 5.2).
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import fcgen
from oracle import assemble, pcg, schwarz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cfg1():
    desc = fcgen.disk_poisson_2d(0)
    return desc, assemble.assemble(desc)


@pytest.fixture(scope="module")
def elast():
    desc = fcgen.porous_elasticity_3d(seed=4, n=3, p=2, n_voids=3,
                                      rmin=0.08, rmax=0.14)
    return desc, assemble.assemble(desc)


# ---------------------------------------------------------- pseudo-inverse
def test_pseudo_inverse_equals_inverse_when_well_conditioned():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.logspace(0, -8, 12)
    A = (Q * lam) @ Q.T
    P = schwarz.pseudo_inverse(A)
    np.testing.assert_allclose(P @ A, np.eye(12), atol=1e-6)
    np.testing.assert_allclose(P, np.linalg.inv(A), rtol=1e-6)


def test_pseudo_inverse_drops_small_and_negative_modes():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    lam = np.array([5.0, 2.0, 1.0, 0.5, 1e-3, 1e-9, 4e-13, 1e-14, -1e-15, 0.0])
    A = (Q * lam) @ Q.T
    P = schwarz.pseudo_inverse(A, eps=1e-13)
    np.testing.assert_allclose(P, P.T, atol=1e-12)
    # P A P = P and A P A = A restricted to the kept modes
    np.testing.assert_allclose(P @ A @ P, P, rtol=1e-6, atol=1e-6 * abs(P).max())
    kept = lam > 1e-13 * 5.0
    ref = (Q[:, kept] / lam[kept]) @ Q[:, kept].T
    np.testing.assert_allclose(P, ref, rtol=1e-6, atol=1e-6 * abs(ref).max())
    assert np.linalg.matrix_rank(P, tol=1e-3) == kept.sum()
    w = np.linalg.eigvalsh(P)
    assert w.min() > -1e-6 * w.max()


def test_pseudo_inverse_of_nonpositive_block_is_zero():
    assert not schwarz.pseudo_inverse(-np.eye(3)).any()


def test_unstabilised_inverse_keeps_negative_mode():
    A = np.diag([1.0, -1e-16])
    P = schwarz.pseudo_inverse(A, stabilize=False)
    assert P[1, 1] < -1e15


# ---------------------------------------------------------- blocks
def test_block_size_and_overlap(cfg1, elast):
    for desc, s in (cfg1, elast):
        d, p = desc["dim"], desc["p"]
        nc = assemble.ncomp_of(desc)
        blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], 1.0)
        assert len(blocks) == desc["n"] ** d
        assert all(B.size == nc * (p + 1) ** d for B in blocks)
        ov = schwarz.block_overlap(blocks, s["A"].shape[0])
        with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
            facts = json.load(f)
        # maximum overlap n_max on a uniform 3-D grid: 8 = 2^d
        if d == 3:
            assert ov.max() == facts["n_max_uniform_3d"]
        assert ov.max() == 2 ** d and ov.min() == 1


def test_pattern_of_S_equals_pattern_of_A(cfg1):
    desc, s = cfg1
    A = s["A"]
    blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], 1.0)
    S, fall = schwarz.compute_preconditioner(A, blocks)
    assert fall.size == 0
    pa = set(zip(*A.nonzero()))
    ps = set(zip(*S.nonzero()))
    assert ps <= pa
    assert len(ps) > 0.97 * len(pa)


def test_single_block_is_exact_inverse():
    desc = fcgen.custom(2, 3, 2, "poisson", alpha=1e-2,
                        shapes=[{"centre": [0.5, 0.5], "semi": [0.4, 0.4]}],
                        domain="inclusions")
    s = assemble.assemble(desc)
    A, b = s["A"], s["b"]
    S, _ = schwarz.compute_preconditioner(A, [np.arange(A.shape[0])])
    np.testing.assert_allclose(S.toarray() @ A.toarray(), np.eye(A.shape[0]),
                               atol=1e-8)
    x, info = pcg.pcg(A, b, S, tol=1e-10)
    assert info["iters"] == 1
    xr = pcg.direct_solve(A, b)
    assert pcg.energy_error(A, xr, x) < 1e-9


def test_unit_blocks_are_jacobi(cfg1):
    _, s = cfg1
    A = s["A"]
    n = A.shape[0]
    S, fall = schwarz.compute_preconditioner(A, [np.array([i]) for i in range(n)])
    assert fall.size == 0
    np.testing.assert_allclose(S.diagonal(), 1.0 / A.diagonal(), rtol=1e-14)
    assert S.nnz == n


def test_diagonal_fallback_exactly_on_uncovered(cfg1):
    _, s = cfg1
    A = s["A"]
    eta_bar = 0.5
    blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], eta_bar)
    covered = schwarz.block_overlap(blocks, A.shape[0]) > 0
    S, fall = schwarz.compute_preconditioner(A, blocks)
    assert 0 < len(blocks) < len(s["eta"])
    np.testing.assert_array_equal(np.sort(fall), np.nonzero(~covered)[0])
    np.testing.assert_allclose(S.diagonal()[fall], 1.0 / A.diagonal()[fall],
                               rtol=0)
    # eta_bar = 0 keeps only cells without any physical point: diagonal
    # scaling everywhere else
    blocks0 = schwarz.select_blocks(s["elem_dofs"], s["eta"], 0.0)
    assert len(blocks0) == int(np.sum(s["eta"] == 0.0))


# ---------------------------------------------------------------- PCG
def _schwarz(s, eta_bar=1.0, **kw):
    blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], eta_bar)
    return schwarz.compute_preconditioner(s["A"], blocks, **kw)[0]


def test_pcg_matches_direct_solve(cfg1, elast):
    for _desc, s in (cfg1, elast):
        A, b = s["A"], s["b"]
        xr = pcg.direct_solve(A, b)
        x, info = pcg.pcg(A, b, _schwarz(s), tol=1e-12)
        assert info["status"] == pcg.OK
        assert pcg.energy_error(A, xr, x) < 1e-9
        assert np.linalg.norm(A @ x - b) < 1e-9 * np.linalg.norm(b)


def test_pcg_conjugacy_and_monotone_energy(cfg1):
    _, s = cfg1
    A, b = s["A"], s["b"]
    S = _schwarz(s)
    xr = pcg.direct_solve(A, b)
    _, info = pcg.pcg(A, b, S, tol=1e-10, maxit=12, x_ref=xr,
                      keep_directions=True)
    P = np.array(info["dirs"][:10]).T
    G = P.T @ (A @ P)
    off = G - np.diag(np.diag(G))
    assert abs(off).max() < 1e-6 * np.diag(G).max()
    e = np.array(info["err"])
    assert np.all(np.diff(e) <= 1e-12)


def test_pcg_iteration_count_is_deterministic(cfg1):
    _, s = cfg1
    S = _schwarz(s)
    it = [pcg.pcg(s["A"], s["b"], S, tol=1e-10)[1]["iters"] for _ in range(2)]
    assert it[0] == it[1]


def _corner_sliver(frac, p=3, n=4):
    """Physical domain below a straight cut across the top-right corner
    cell (a huge disk), so that cell keeps a small triangle whose volume
    fraction shrinks like frac^2; alpha = 0 as in the remark of Sec. 3.2."""
    h = 1.0 / n
    R = 1000.0
    edge = 1.0 - h + frac * h
    c = [edge - R / np.sqrt(2.0), edge - R / np.sqrt(2.0)]
    return fcgen.custom(2, n, p, "poisson", alpha=0.0,
                        shapes=[{"centre": c, "semi": [R, R]}],
                        domain="inclusions", quad_depth=8, seed=7)


def test_schwarz_robust_where_jacobi_is_not():
    it_s, it_j, etas = [], [], []
    for frac in (0.3, 0.03, 0.003):
        s = assemble.assemble(_corner_sliver(frac))
        A, b = s["A"], s["b"]
        etas.append(s["eta"].min())
        it_s.append(pcg.pcg(A, b, _schwarz(s), tol=1e-8)[1]["iters"])
        D = sp.diags(1.0 / A.diagonal())
        it_j.append(pcg.pcg(A, b, D, tol=1e-8, maxit=20000)[1]["iters"])
    assert etas[-1] < 1e-4
    assert max(it_s) <= 1.25 * min(it_s), it_s
    assert it_j[-1] > 3 * it_j[0], it_j
    assert it_j[-1] > 10 * it_s[-1], (it_j, it_s)


# ------------------------------------------------------ vertex patches
def _patch_case(name):
    import fcgen
    from oracle import assemble
    d = {"disk": lambda: fcgen.disk_poisson_2d(0),
         "cube": lambda: fcgen.porous_poisson_3d(seed=1, n=3, p=2, n_voids=2, rmin=0.1,
                                                  rmax=0.2)}[name]()
    return d, assemble.assemble(d)


@pytest.mark.parametrize("name", ["disk", "cube"])
def test_vertex_patches_contain_every_element_block(name):
    """Every element block lies inside the patch of each of its cell's
    vertices; interior patches hold (2p+1)^dim functions; a vertex function
    belongs to 3^dim patches away from the boundary, an interior function
    of a cell edge or face to fewer (2 per direction where it is not a
    vertex index): counted here by brute force over the lattice."""
    d, s = _patch_case(name)
    n, p, dim = d["n"], d["p"], d["dim"]
    patches = schwarz.vertex_patch_blocks(d, s["elem_dofs"], s["eta"], 1.0)
    assert len(patches) == (n + 1) ** dim
    sets = [set(b.tolist()) for b in patches]
    for e, B in enumerate(s["elem_dofs"]):
        cell = [(e // n ** k) % n for k in range(dim)]
        for corner in itertools.product((0, 1), repeat=dim):
            vid = sum((cell[k] + corner[k]) * (n + 1) ** k for k in range(dim))
            assert set(B.tolist()) <= sets[vid]
    assert max(len(b) for b in patches) == (2 * p + 1) ** dim
    n1 = p * n + 1
    count = schwarz.block_overlap(patches, s["A"].shape[0])
    for node in range(n1 ** dim):
        g = [(node // n1 ** k) % n1 for k in range(dim)]
        expect = 1
        for gk in g:
            lo, hi = -((-(gk - p)) // p), (gk + p) // p    # vertices v with |gk - p v| <= p
            expect *= min(hi, n) - max(lo, 0) + 1
        assert count[node] == expect, (node, g)


def test_vertex_patch_pcg_solves_config_1():
    """Schwarz-PCG with vertex patches on the 16^2-cell disk reaches the
    direct solution, and, its blocks containing the element blocks, needs
    no more iterations than element blocks."""
    d, s = _patch_case("disk")
    A, b = s["A"], s["b"]
    Sp, fp = schwarz.compute_preconditioner(A, schwarz.vertex_patch_blocks(
        d, s["elem_dofs"], s["eta"], 1.0))
    Se, _ = schwarz.compute_preconditioner(A, schwarz.select_blocks(s["elem_dofs"], s["eta"]))
    assert fp.size == 0
    xp, ip = pcg.pcg(A, b, Sp, tol=1e-12)
    _, ie = pcg.pcg(A, b, Se, tol=1e-12)
    xr = pcg.direct_solve(A, b)
    assert ip["status"] == pcg.OK
    assert pcg.energy_error(A, xr, xp) <= 1e-8
    assert ip["iters"] <= ie["iters"]
