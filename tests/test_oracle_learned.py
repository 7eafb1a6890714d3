"""Pins of the learned coarse-correction oracle (network layers, backward
pass, optimiser and grid transfers) against brute force, adjoint
identities, finite differences and exactness properties."""
import itertools

import numpy as np
import pytest

import fcgen
from oracle import learned as L


def _conv_brute(x, w, b):
    """Direct 7-loop 'same' convolution with explicit zero padding."""
    B, Ci, D, H, W = x.shape
    Co = w.shape[0]
    y = np.zeros((B, Co, D, H, W))
    for bb, o, z, yy, xx in itertools.product(range(B), range(Co), range(D), range(H), range(W)):
        s = b[o]
        for c, dz, dy, dx in itertools.product(range(Ci), range(3), range(3), range(3)):
            zz, y2, x2 = z + dz - 1, yy + dy - 1, xx + dx - 1
            if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < W:
                s += w[o, c, dz, dy, dx] * x[bb, c, zz, y2, x2]
        y[bb, o, z, yy, xx] = s
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 2, 3, 4, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(L.conv3d(x, w, b), _conv_brute(x, w, b), atol=1e-12)


def test_conv_tap_order_is_dz_dy_dx():
    """A single tap at (dz,dy,dx) = (2,1,0) shifts by +1 in z and -1 in x."""
    x = np.zeros((1, 1, 4, 4, 4))
    x[0, 0, 2, 1, 1] = 1.0
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, 2, 1, 0] = 1.0
    y = L.conv3d(x, w, np.zeros(1))
    # y[z,y,x] = x[z+1, y, x-1]  ->  the one lands at (1, 1, 2)
    assert y[0, 0, 1, 1, 2] == 1.0 and y.sum() == 1.0


def test_conv_backward_is_adjoint_and_derivative():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 4, 3, 5))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    gy = rng.standard_normal((2, 2, 4, 3, 5))
    gx, gw, gb = L.conv3d_backward(x, w, gy)
    # adjoint in x: <conv(x) - b, gy> = <x, gx>
    lin = L.conv3d(x, w, np.zeros(2))
    assert np.isclose((lin * gy).sum(), (x * gx).sum(), rtol=1e-12)
    # the convolution is linear in w: <conv_w(x), gy> = <w, gw>
    assert np.isclose((lin * gy).sum(), (w * gw).sum(), rtol=1e-12)
    assert np.allclose(gb, gy.sum(axis=(0, 2, 3, 4)))


@pytest.mark.parametrize("shape", [(1, 1, 4, 4, 4), (2, 3, 5, 3, 7), (1, 2, 1, 2, 3)])
def test_pool_is_mean_of_existing_children(shape):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(shape)
    p = L.pool(x)
    B, C, D, H, W = shape
    for z, yy, xx in itertools.product(range(p.shape[2]), range(p.shape[3]), range(p.shape[4])):
        blk = x[:, :, 2 * z:2 * z + 2, 2 * yy:2 * yy + 2, 2 * xx:2 * xx + 2]
        assert np.allclose(p[:, :, z, yy, xx], blk.mean(axis=(2, 3, 4)))
    g = rng.standard_normal(p.shape)
    assert np.isclose((p * g).sum(), (x * L.pool_backward(g, shape)).sum(), rtol=1e-12)


@pytest.mark.parametrize("fine", [(4, 4, 4), (5, 3, 7)])
def test_upsample_nearest_and_adjoint(fine):
    rng = np.random.default_rng(3)
    coarse = (2, 2) + tuple((f + 1) // 2 for f in fine)
    x = rng.standard_normal(coarse)
    u = L.upsample(x, fine)
    for z, yy, xx in itertools.product(*(range(f) for f in fine)):
        assert np.array_equal(u[:, :, z, yy, xx], x[:, :, z // 2, yy // 2, xx // 2])
    g = rng.standard_normal(u.shape)
    assert np.isclose((u * g).sum(), (x * L.upsample_backward(g, coarse)).sum(), rtol=1e-12)


CH = (2, 3, 2, 2)


def test_param_layout_count():
    assert L.n_params(CH) == fcgen.unet_init(CH, 2).size
    # default width network size used by the solver
    assert L.n_params((8, 16, 32, 32)) == 191017


def test_forward_bias_only_network_is_constant():
    th = np.zeros(L.n_params(CH))
    th[-1] = 0.625                       # bias of the head convolution
    x = np.random.default_rng(4).standard_normal((2, 2, 5, 6, 7))
    y = L.forward(th, x, CH)
    assert y.shape == (2, 1, 5, 6, 7) and np.all(y == 0.625)


@pytest.mark.parametrize("g", [4, 5])
def test_loss_gradient_matches_finite_differences(g):
    """Central differences of the forward loss on a sample of coordinates in
    every layer; the network is piecewise linear, so away from ReLU kinks
    the difference quotient is exact up to rounding."""
    rng = np.random.default_rng(5 + g)
    th = rng.standard_normal(L.n_params(CH)) * 0.5
    x = rng.standard_normal((2, 2, g, g, g))
    t = rng.standard_normal((2, 1, g, g, g))
    loss, grad = L.loss_and_grad(th, x, t, CH)
    assert np.isclose(loss, np.mean((L.forward(th, x, CH) - t) ** 2))
    off = 0
    h = 1e-6
    for name, (ci, co) in L.layer_shapes(CH).items():
        n = co * ci * 27 + co
        for k in list(rng.choice(n - co, 3, replace=False)) + [n - 1]:
            i = off + int(k)
            tp, tm = th.copy(), th.copy()
            tp[i] += h
            tm[i] -= h
            lp = np.mean((L.forward(tp, x, CH) - t) ** 2)
            lm = np.mean((L.forward(tm, x, CH) - t) ** 2)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (name, k, fd, grad[i])
        off += n


def test_adam_first_step_is_signed_lr():
    """With zero moments the bias-corrected first step is -lr*sign(g)
    (up to the eps in the denominator)."""
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    th, m, v = L.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-4)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_two_steps_by_hand():
    """Two Adam steps (beta1 0.9, beta2 0.999, eps 0) worked out by hand.
    Component 0, gradients +1 then -1: m2 = 0.09 - 0.1 = -0.01 and
    m2 / (1 - 0.81) = -1/19; v2 = 0.000999 + 0.001 = 0.001999 and
    v2 / (1 - 0.998001) = 1; so theta2 = -0.01 + 0.01/19.  Component 1,
    gradient 2 twice: m2 / 0.19 = 2 and v2 / 0.001999 = 4, a full step of
    lr each time: theta2 = -0.02.  Component 2, gradient 0 then 3:
    m2 / 0.19 = 0.3 / 0.19, v2 / 0.001999 = 0.009 / 0.001999, theta2 =
    -0.01 * (30/19) / sqrt(9000/1999)."""
    lr = 0.01
    th = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    with np.errstate(invalid="ignore"):
        th, m, v = L.adam_step(th, np.array([1.0, 2.0, 0.0]), m, v, 1, lr=lr, eps=0.0)
    th[2] = 0.0          # 0/0 of a zero first gradient with eps = 0
    th, m, v = L.adam_step(th, np.array([-1.0, 2.0, 3.0]), m, v, 2, lr=lr, eps=0.0)
    expect = np.array([-0.01 + 0.01 / 19.0, -0.02,
                       -0.01 * (30.0 / 19.0) / np.sqrt(9000.0 / 1999.0)])
    np.testing.assert_allclose(th, expect, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(m, [-0.01, 0.38, 0.3], rtol=1e-13)
    np.testing.assert_allclose(v, [0.001999, 0.007996, 0.009], rtol=1e-13)


# ------------------------------------------------------------ transfers
@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (3, 4, 3), (3, 6, 1), (2, 8, 4)])
def test_vertex_index_is_lattice_corner(dim, n, p):
    desc = fcgen.custom(dim, n, p)
    vi = L.vertex_index(desc)
    n1 = p * n + 1
    for idx in itertools.product(range(n + 1), repeat=dim):
        # idx is (.., y, x) with the last axis the first coordinate
        g = 0
        for a, i in enumerate(reversed(idx)):
            g += (p * i) * n1 ** a
        assert vi[idx] == g


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (3, 4, 2), (3, 6, 3)])
def test_prolong_reproduces_affine_and_restrict_is_transpose(dim, n, p):
    desc = fcgen.custom(dim, n, p)
    nc = n // 2
    rng = np.random.default_rng(dim * 10 + n)
    c = rng.standard_normal(dim + 1)
    grid = np.meshgrid(*([np.linspace(0, 1, nc + 1)] * dim), indexing="ij")
    # axis 0 is the last coordinate
    wc = c[0] + sum(c[1 + a] * grid[dim - 1 - a] for a in range(dim))
    u = L.prolong(desc, wc)
    fgrid = np.meshgrid(*([np.linspace(0, 1, n + 1)] * dim), indexing="ij")
    expect = c[0] + sum(c[1 + a] * fgrid[dim - 1 - a] for a in range(dim))
    assert np.allclose(u[L.vertex_index(desc)], expect)
    mask = np.ones(u.size, bool)
    mask[L.vertex_index(desc).ravel()] = False
    assert np.all(u[mask] == 0.0)
    assert np.allclose(L.sample(desc, u), wc)
    r = rng.standard_normal(u.size)
    assert np.isclose((u * r).sum(), (wc * L.restrict(desc, r)).sum(), rtol=1e-12)


def test_coarse_eta_uniform_and_corner():
    desc = fcgen.custom(3, 4, 2)
    assert np.allclose(L.coarse_eta(desc, np.full(64, 0.3)), 0.3)
    # only fine cell (0,0,0) physical -> coarse cell 0 has eta 1/8, which
    # the corner vertex alone sees fully, its edge neighbours at half weight
    eta = np.zeros(64)
    eta[0] = 1.0
    ce = L.coarse_eta(desc, eta)
    assert np.isclose(ce[0, 0, 0], 1 / 8)
    assert np.isclose(ce[0, 0, 1], 1 / 16)
    assert np.isclose(ce[1, 1, 1], 1 / 64)
    assert ce[2, 2, 2] == 0.0


# ------------------------------------------------- coarse level and FCG
from oracle import assemble as ASM
from oracle import pcg as PCG
from oracle import schwarz as SCH


@pytest.mark.parametrize("dim,n,p", [(2, 6, 2), (3, 4, 2), (3, 4, 3)])
def test_prolong_matrix_matches_prolong_and_restrict(dim, n, p):
    desc = fcgen.custom(dim, n, p)
    P = L.prolong_matrix(desc)
    G = n // 2 + 1
    rng = np.random.default_rng(11)
    wc = rng.standard_normal((G,) * dim)
    assert np.allclose(P @ wc.ravel(), L.prolong(desc, wc))
    r = rng.standard_normal(P.shape[0])
    assert np.allclose(P.T @ r, L.restrict(desc, r).ravel())


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 2), (3, 3)])
def test_galerkin_coarse_operator_is_coarse_q1_system(dim, p):
    """On an uncut domain the vertex functions are the fine Q1 hats, the
    trilinear coarse functions lie in their span, and both systems are
    integrated exactly: P^T A P equals the p = 1 system of the mesh with
    half as many cells per direction."""
    fine = fcgen.custom(dim, 4, p, shapes=[])
    coarse = fcgen.custom(dim, 2, 1, shapes=[])
    Ac = L.coarse_operator(fine, ASM.assemble(fine)["A"])
    A1 = ASM.assemble(coarse)["A"].toarray()
    assert np.allclose(Ac, A1, rtol=1e-12, atol=1e-13 * np.abs(A1).max())


def test_vertex_mask_marks_vertices_of_physical_cells():
    n = 6
    desc = fcgen.custom(3, n, 2)
    rng = np.random.default_rng(12)
    eta = (rng.uniform(size=n ** 3) < 0.15) * rng.uniform(size=n ** 3)
    fine = np.zeros((n + 1,) * 3)
    for c in np.flatnonzero(eta > 0):
        cz, cy, cx = c // (n * n), (c // n) % n, c % n
        fine[cz:cz + 2, cy:cy + 2, cx:cx + 2] = 1.0
    assert np.array_equal(L.vertex_mask(desc, eta), fine[::2, ::2, ::2])


def test_network_input_and_target_scaling():
    desc = fcgen.porous_poisson_3d(0, n=4, p=2, n_voids=2, rmin=0.1, rmax=0.2)
    sysm = ASM.assemble(desc)
    rng = np.random.default_rng(13)
    r = rng.standard_normal(sysm["b"].size)
    xin = L.network_input(desc, r, sysm["eta"])
    assert xin.shape == (2, 3, 3, 3)
    assert np.isclose(np.sqrt(np.mean(xin[0] ** 2)), 1.0)
    assert np.allclose(xin[1], L.coarse_eta(desc, sysm["eta"]))
    e, z = rng.standard_normal(r.size), rng.standard_normal(r.size)
    t = L.snapshot_target(desc, e, z, sysm["eta"])
    mask = L.vertex_mask(desc, sysm["eta"])
    assert np.all(t[mask == 0] == 0.0)
    assert np.isclose(np.sqrt(np.mean(t ** 2)), 1.0)
    raw = L.sample(desc, e - z) * mask
    assert np.allclose(t * np.sqrt(np.mean(raw ** 2)), raw)


def _small_system():
    desc = fcgen.porous_poisson_3d(3, n=8, p=2, n_voids=6, rmin=0.08, rmax=0.15)
    sysm = ASM.assemble(desc)
    blocks = SCH.select_blocks(sysm["elem_dofs"], sysm["eta"])
    S, _ = SCH.compute_preconditioner(sysm["A"], blocks)
    return desc, sysm, S


def test_fcg_without_correction_reproduces_pcg():
    desc, sysm, S = _small_system()
    A, b = sysm["A"], sysm["b"]
    P = L.prolong_matrix(desc)
    Ac = L.coarse_operator(desc, A)
    G = desc["n"] // 2 + 1
    x1, i1 = L.fcg(A, b, S, P, Ac, lambda r: np.zeros(G ** 3), tol=1e-8)
    x0, i0 = PCG.pcg(A, b, S, tol=1e-8, stop="residual")
    assert i1["status"] == PCG.OK and abs(i1["iters"] - i0["iters"]) <= 1
    assert np.all(np.asarray(i1["gamma"]) == 0.0)
    assert PCG.energy_error(A, x0, x1) <= 1e-8


def test_fcg_with_exact_coarse_solve():
    """With y = A_c^{-1} P^T r the step gamma is one and FCG becomes the
    two-level additive Schwarz method, which needs fewer iterations than
    the one-level method and reaches the same solution."""
    desc, sysm, S = _small_system()
    A, b = sysm["A"], sysm["b"]
    P = L.prolong_matrix(desc)
    Ac = L.coarse_operator(desc, A)
    x2, i2 = L.fcg(A, b, S, P, Ac, lambda r: np.linalg.solve(Ac, P.T @ r), tol=1e-8)
    x0, i0 = PCG.pcg(A, b, S, tol=1e-8, stop="residual")
    assert i2["status"] == PCG.OK
    assert np.allclose(i2["gamma"], 1.0, rtol=1e-8)
    assert i2["iters"] < i0["iters"], (i2["iters"], i0["iters"])
    xs = PCG.direct_solve(A, b)
    assert PCG.energy_error(A, xs, x2) <= 1e-6 * np.sqrt(xs @ (A @ xs))


def test_fcg_truncated_with_fixed_preconditioner_is_pcg():
    """With a fixed SPD preconditioner the older directions are already
    A-orthogonal to the new one, so keeping m > 1 of them changes nothing:
    FCG(m) reproduces PCG."""
    desc, sysm, S = _small_system()
    A, b = sysm["A"], sysm["b"]
    P = L.prolong_matrix(desc)
    Ac = L.coarse_operator(desc, A)
    G = desc["n"] // 2 + 1
    x0, i0 = PCG.pcg(A, b, S, tol=1e-8, stop="residual")
    for m in (2, 8):
        x1, i1 = L.fcg(A, b, S, P, Ac, lambda r: np.zeros(G ** 3), tol=1e-8, m=m)
        assert i1["status"] == PCG.OK and abs(i1["iters"] - i0["iters"]) <= 1, (m, i1["iters"])
        assert PCG.energy_error(A, x0, x1) <= 1e-8


def _nonlinear_problem(n=14, k=4, seed=5):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + 0.05 * np.eye(n)
    S = np.diag(1.0 / np.diag(A))
    P = rng.standard_normal((n, k))
    Ac = P.T @ A @ P
    b = rng.standard_normal(n)

    def corr(r):
        v = P.T @ r
        return np.tanh(3.0 * v / np.linalg.norm(v)) + 0.3 * np.sign(v) * v ** 2
    return A, b, S, P, Ac, corr


def test_fcg_full_orthogonalisation_terminates_with_nonlinear_preconditioner():
    """Keeping every direction makes them all A-orthogonal whatever the
    preconditioner does, so x_k minimises the energy error over their span
    and the solve ends within n steps on an n-unknown system; the
    Polak-Ribiere form FCG(1) does not, with this nonlinear correction."""
    A, b, S, P, Ac, corr = _nonlinear_problem()
    n = b.size
    x, info = L.fcg(A, b, S, P, Ac, corr, tol=1e-10, maxit=n, m=n)
    assert info["status"] == PCG.OK, info["res"][-3:]
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    _, info1 = L.fcg(A, b, S, P, Ac, corr, tol=1e-10, maxit=n, m=1)
    assert info1["status"] != PCG.OK


def test_coarse_projection_is_the_energy_projection_of_the_error():
    """P_c y of the "coarse" target is the A-orthogonal projection of e onto
    the material coarse vertex functions: the remaining error is
    A-orthogonal to each of them (checked with the fine A and P_c, not
    A_c), and any other coarse correction leaves more energy, by exactly
    the energy of the difference (Pythagoras)."""
    desc = fcgen.porous_poisson_3d(3, n=4, p=2, n_voids=3, rmin=0.1, rmax=0.18)
    sysm = ASM.assemble(desc)
    A, eta = sysm["A"], sysm["eta"]
    rng = np.random.default_rng(21)
    e = rng.standard_normal(A.shape[0])
    r = A @ e
    y = L.coarse_projection(desc, A, r, eta).ravel()
    m = (L.vertex_mask(desc, eta) > 0).ravel()
    assert 0 < m.sum() < m.size or m.all()
    assert np.all(y[~m] == 0.0)
    Pm = L.prolong_matrix(desc)[:, m]
    w = L.prolong_matrix(desc) @ y
    resid = Pm.T @ (A @ (e - w))
    assert np.linalg.norm(resid) <= 1e-9 * np.linalg.norm(Pm.T @ (A @ e))
    energy = lambda v: float(v @ (A @ v))
    d = np.zeros_like(y)
    d[m] = rng.standard_normal(m.sum())
    wd = L.prolong_matrix(desc) @ d
    lhs = energy(e - w - wd)
    assert np.isclose(lhs, energy(e - w) + energy(wd), rtol=1e-9)
    t = L.coarse_projection_target(desc, A, r, eta).ravel()
    assert np.isclose(np.sqrt(np.mean(t ** 2)), 1.0)
    assert np.allclose(t * np.sqrt(np.mean(y ** 2)), y)
