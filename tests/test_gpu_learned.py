"""GPU network kernels against the FP64 NumPy network of the oracle.

The GPU convolutions use BF16 weights with FP32 activations and
accumulation, so the oracle is evaluated with the same BF16-rounded weights
in FP64; forward outputs agree to FP32 accumulation error and parameter
gradients to a few 1e-4 relative."""
import numpy as np
import pytest

import fcgen
import paper_1809_00828_amd as fc
from oracle import learned as L
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu

CH = (4, 6, 8, 8)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def bf16_round(a):
    """Round float32 to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _case(seed, B, g):
    rng = np.random.default_rng(seed)
    theta = fcgen.unet_init(CH, 2, seed=seed)
    # random biases too, so every code path is exercised
    theta = theta.copy()
    off = 0
    for name, (ci, co) in L.layer_shapes(CH).items():
        off += co * ci * 27
        theta[off: off + co] = rng.standard_normal(co).astype(np.float32) * 0.1
        off += co
    x = rng.standard_normal((B, 2, g, g, g)).astype(np.float32)
    t = rng.standard_normal((B, 1, g, g, g)).astype(np.float32)
    return theta, x, t


def _oracle_theta(theta):
    """Weights rounded to BF16 as the GPU uses them, biases in FP32."""
    th = theta.astype(np.float64).copy()
    off = 0
    for name, (ci, co) in L.layer_shapes(CH).items():
        th[off: off + co * ci * 27] = bf16_round(theta[off: off + co * ci * 27])
        off += co * ci * 27 + co
    return th


@pytest.mark.parametrize("B,g", [(1, 9), (2, 7), (3, 6)])
def test_forward_matches_oracle(torch, B, g):
    theta, x, t = _case(B * 10 + g, B, g)
    m = fc.Model(theta, CH)
    xd = torch.as_tensor(x, device="cuda")
    yd = torch.empty((B, 1, g, g, g), dtype=torch.float32, device="cuda")
    m.forward(xd, yd)
    torch.cuda.synchronize()
    ref = L.forward(_oracle_theta(theta), x.astype(np.float64), CH)
    err = np.abs(yd.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 2e-5, err


@pytest.mark.parametrize("B,g", [(2, 7), (1, 10)])
def test_gradient_matches_oracle(torch, B, g):
    theta, x, t = _case(B * 7 + g, B, g)
    m = fc.Model(theta, CH)
    loss, grad = m.loss_grad(torch.as_tensor(x, device="cuda"), torch.as_tensor(t, device="cuda"))
    lo, go = L.loss_and_grad(_oracle_theta(theta), x.astype(np.float64), t.astype(np.float64), CH)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    off = 0
    for name, (ci, co) in L.layer_shapes(CH).items():
        n = co * ci * 27 + co
        gg, gr = grad[off: off + n], go[off: off + n]
        off += n
        scale = np.abs(gr).max() + 1e-30
        assert np.abs(gg - gr).max() <= 2e-4 * scale, name


def test_training_reduces_loss(torch):
    """Learn a fixed linear map (a smoothing of channel 0) from 32 samples."""
    rng = np.random.default_rng(1)
    g, n = 9, 32
    x = rng.standard_normal((n, 2, g, g, g)).astype(np.float32)
    k = np.ones((3, 3, 3)) / 27.0
    w = np.zeros((1, 2, 3, 3, 3))
    w[0, 0] = k
    t = L.conv3d(x.astype(np.float64), w, np.zeros(1)).astype(np.float32)
    m = fc.Model(fcgen.unet_init(CH, 2, seed=3), CH)
    hist = m.train(torch.as_tensor(x, device="cuda"), torch.as_tensor(t, device="cuda"),
                   epochs=40, batch=8, lr=3e-3)
    print("loss history", hist[[0, 9, 19, 39]], flush=True)
    assert hist[-1] < 0.2 * hist[0]
    # parameters moved and stayed finite
    p = m.params()
    assert np.isfinite(p).all()


def test_adam_steps_match_oracle(torch):
    """Three Adam steps of the library's training loop (one full-batch
    mini-batch per call, so the moments and the bias-correction step count
    carry over between calls) against the oracle's adam_step fed with the
    same gradients: the library's gradient at the current parameters is
    read with loss_grad (the training step computes the same kernels on the
    same batch), then one training step runs, and the oracle repeats the
    update in FP64 from the library's parameters.  The FP32 update must
    match to rounding: 1e-6 of the step plus the FP32 spacing of the
    parameter."""
    theta, x, t = _case(77, 4, 7)
    m = fc.Model(theta, CH)
    xd = torch.as_tensor(x, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    lr = 1e-3
    mo = np.zeros(theta.size)
    vo = np.zeros(theta.size)
    th = m.params().astype(np.float64)
    for step in range(1, 4):
        _, g = m.loss_grad(xd, td)
        m.train(xd, td, epochs=1, batch=x.shape[0], lr=lr)
        got = m.params().astype(np.float64)
        ref, mo, vo = L.adam_step(th, g.astype(np.float64), mo, vo, step, lr=lr)
        tol = 1e-6 * lr + 2.0 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        err = np.abs(got - ref)
        print(f"[adam] step {step}: max |diff| {err.max():.2e}, moved {np.abs(got - th).max():.2e}",
              flush=True)
        assert np.all(err <= tol), (step, int(np.argmax(err - tol)))
        # every parameter with a nonzero gradient moved by about lr
        assert np.abs(got - th).max() <= 1.01 * lr * step
        th = got


# --------------------------------------------- coarse level and learned FCG
import functools

from oracle import assemble as ASM
from oracle import pcg as PCG
from oracle import schwarz as SCH

COARSE_PROBLEMS = {
    # 3-D Poisson, porous cube, 8^3 cells, p = 2 (coarse grid 5^3)
    "pois8_p2": lambda: fcgen.porous_poisson_3d(3, n=8, p=2, n_voids=6, rmin=0.08, rmax=0.15),
    # p = 3 and a 6^3 grid (coarse grid 4^3)
    "pois6_p3": lambda: fcgen.porous_poisson_3d(4, n=6, p=3, n_voids=4, rmin=0.08, rmax=0.15),
}


@functools.lru_cache(maxsize=None)
def coarse_case(name):
    desc = COARSE_PROBLEMS[name]()
    s = ASM.assemble(desc)
    blocks = SCH.select_blocks(s["elem_dofs"], s["eta"])
    S, _ = SCH.compute_preconditioner(s["A"], blocks)
    P = L.prolong_matrix(desc)
    Ac = L.coarse_operator(desc, s["A"])
    return desc, s, S, P, Ac


def _lib_case(name):
    desc = COARSE_PROBLEMS[name]()
    pb = fc.Problem.setup(desc)
    pc = fc.Precond(pb)
    return desc, pb, pc


@pytest.mark.parametrize("name", list(COARSE_PROBLEMS))
def test_coarse_transfers_and_operator_match_oracle(torch, name):
    print(f"[coarse] {name}", flush=True)
    desc, s, S, P, Ac = coarse_case(name)
    _, pb, pc = _lib_case(name)
    G = pc.coarse_grid()
    assert G == desc["n"] // 2 + 1
    nv = G ** 3
    rng = np.random.default_rng(21)
    # restriction
    r = rng.standard_normal(pb.n)
    rc = torch.empty(nv, dtype=torch.float64, device="cuda")
    pc.coarse_restrict(torch.as_tensor(r, device="cuda"), rc)
    ref = P.T @ r
    assert np.abs(rc.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max() * 8
    # prolongation (added to z)
    y = rng.standard_normal(nv).astype(np.float32)
    z0 = rng.standard_normal(pb.n)
    z = torch.as_tensor(z0.copy(), device="cuda")
    pc.coarse_prolong(torch.as_tensor(y, device="cuda"), -0.75, z)
    ref = z0 - 0.75 * (P @ y.astype(np.float64))
    assert np.abs(z.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max() * 8
    # Galerkin operator and the step gamma
    v = torch.empty(nv, dtype=torch.float64, device="cuda")
    gamma = pc.coarse_apply(torch.as_tensor(y, device="cuda"), v)
    yd = y.astype(np.float64)
    vref = Ac @ yd
    assert np.abs(v.cpu().numpy() - vref).max() <= 1e-12 * np.abs(vref).max()
    gref = float(yd @ (P.T @ r)) / float(yd @ vref)
    assert abs(gamma - gref) <= 1e-11 * abs(gref)
    # input channels
    eta = torch.empty(nv, dtype=torch.float32, device="cuda")
    mask = torch.empty(nv, dtype=torch.float32, device="cuda")
    pc.coarse_channels(eta, mask)
    assert np.allclose(eta.cpu().numpy(), L.coarse_eta(desc, s["eta"]).ravel(), atol=1e-6)
    assert np.array_equal(mask.cpu().numpy(), L.vertex_mask(desc, s["eta"]).ravel())


@pytest.mark.parametrize("name", list(COARSE_PROBLEMS))
def test_snapshots_match_oracle(torch, name):
    """Training pairs at iterations 0, 1, 4, 9 from the GPU solve against
    the oracle's iterates with the same converged solution x*."""
    print(f"[snapshots] {name}", flush=True)
    desc, s, S, P, Ac = coarse_case(name)
    _, pb, pc = _lib_case(name)
    A, b = s["A"], s["b"]
    xs = PCG.direct_solve(A, b)
    G = pc.coarse_grid()
    nv = G ** 3
    iters = [0, 1, 4, 9]
    bd = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(bd)
    xin = torch.zeros((len(iters), 2, nv), dtype=torch.float32, device="cuda")
    t = torch.zeros((len(iters), nv), dtype=torch.float32, device="cuda")
    for kind in ("e-Sr", "e"):
        k = pc.snapshots(bd, torch.as_tensor(xs, device="cuda"), iters, xin, t, kind=kind,
                         tol=1e-12)
        assert k == len(iters)
        for j, it in enumerate(iters):
            xk, _ = PCG.pcg(A, b, S, tol=0.0, maxit=it, stop="residual")
            rk = b - A @ xk
            zk = S @ rk
            ref_in = L.network_input(desc, rk, s["eta"]).reshape(2, -1)
            ref_t = L.snapshot_target(desc, xs - xk, zk if kind == "e-Sr" else 0 * zk,
                                      s["eta"]).ravel()
            got_in = xin[j].cpu().numpy()
            assert np.abs(got_in - ref_in).max() <= 1e-5 * max(1.0, np.abs(ref_in).max()), (kind, it)
            assert np.abs(t[j].cpu().numpy() - ref_t).max() <= 1e-5 * np.abs(ref_t).max(), (kind, it)
    # the coarse Galerkin projection of the error, solved on the device by
    # CG on A_c to a relative residual of 1e-8: error at most kappa * 1e-8
    msk = L.vertex_mask(desc, s["eta"]).ravel() > 0
    Acm = Ac[np.ix_(msk, msk)]
    dm = np.sqrt(np.diag(Acm))
    lam = np.linalg.eigvalsh(Acm / dm[:, None] / dm[None, :])
    tol_c = max(1e-5, 10.0 * (lam[-1] / lam[0]) * 1e-8)
    k = pc.snapshots(bd, torch.as_tensor(xs, device="cuda"), iters, xin, t, kind="coarse",
                     tol=1e-12)
    assert k == len(iters)
    for j, it in enumerate(iters):
        xk, _ = PCG.pcg(A, b, S, tol=0.0, maxit=it, stop="residual")
        rk = b - A @ xk
        ref_in = L.network_input(desc, rk, s["eta"]).reshape(2, -1)
        ref_t = L.coarse_projection_target(desc, A, rk, s["eta"]).ravel()
        got_in = xin[j].cpu().numpy()
        assert np.abs(got_in - ref_in).max() <= 1e-5 * max(1.0, np.abs(ref_in).max()), ("coarse", it)
        err = np.abs(t[j].cpu().numpy() - ref_t).max() / np.abs(ref_t).max()
        assert err <= tol_c, ("coarse", it, err, tol_c)


def _learned_solve(torch, pb, pc, tol=1e-8, mode="learned", fcg_m=1):
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    info = fc.pcg_solve(pb, pc, b, x, tol=tol, stop="residual", mode=mode, check_every=8,
                        fcg_m=fcg_m)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


def test_learned_fcg_with_zero_network_reproduces_pcg(torch):
    print("[learned] zero network", flush=True)
    desc, s, S, P, Ac = coarse_case("pois8_p2")
    _, pb, pc = _lib_case("pois8_p2")
    m = fc.Model(np.zeros(L.n_params(CH), np.float32), CH)
    pc.attach(m)
    xl, il = _learned_solve(torch, pb, pc)
    xp, ip = _learned_solve(torch, pb, pc, mode="f64")
    xo, io = PCG.pcg(s["A"], s["b"], S, tol=1e-8, stop="residual")
    assert il["status"] == "OK" and ip["status"] == "OK"
    assert abs(il["iters"] - ip["iters"]) <= 1 and abs(il["iters"] - io["iters"]) <= 2
    st = pc.learned_stats()
    # one apply at the start and one per step
    assert st["applied"] == il["iters"] + 1 and st["dropped"] == st["applied"], st
    A = s["A"]
    en = np.sqrt(xo @ (A @ xo))
    assert np.sqrt((xl - xp) @ (A @ (xl - xp))) <= 1e-7 * en


def test_learned_fcg_m_with_zero_network_reproduces_pcg(torch):
    """Keeping 8 directions changes nothing for a fixed preconditioner."""
    print("[learned] zero network, fcg_m 8", flush=True)
    desc, s, S, P, Ac = coarse_case("pois8_p2")
    _, pb, pc = _lib_case("pois8_p2")
    m = fc.Model(np.zeros(L.n_params(CH), np.float32), CH)
    pc.attach(m)
    xl, il = _learned_solve(torch, pb, pc, fcg_m=8)
    xp, ip = _learned_solve(torch, pb, pc, mode="f64")
    assert il["status"] == "OK" and abs(il["iters"] - ip["iters"]) <= 1
    A = s["A"]
    en = np.sqrt(xp @ (A @ xp))
    assert np.sqrt((xl - xp) @ (A @ (xl - xp))) <= 1e-7 * en


@pytest.mark.parametrize("name,fcg_m", [("pois8_p2", 4), ("pois8_p2", 64), ("pois6_p3", 16)])
def test_learned_fcg_m_matches_oracle(torch, name, fcg_m):
    """A seeded network inside flexible CG keeping fcg_m directions: GPU
    against the oracle's FCG(m) with the same network."""
    print(f"[learned] oracle fcg({fcg_m}) {name}", flush=True)
    desc, s, S, P, Ac = coarse_case(name)
    _, pb, pc = _lib_case(name)
    theta = fcgen.unet_init(CH, 2, seed=7)
    m = fc.Model(theta, CH)
    pc.attach(m)
    xl, il = _learned_solve(torch, pb, pc, fcg_m=fcg_m)
    th = _oracle_theta(theta)

    def corr(r):
        xin = L.network_input(desc, r, s["eta"])[None]
        return L.forward(th, xin, CH).ravel()

    xo, io = L.fcg(s["A"], s["b"], S, P, Ac, corr, tol=1e-8, m=fcg_m)
    assert il["status"] == "OK" and io["status"] == PCG.OK
    assert abs(il["iters"] - io["iters"]) <= max(2, 0.1 * io["iters"]), (il["iters"], io["iters"])
    assert il["rel_res_true"] <= 1.5e-8
    A = s["A"]
    xs = PCG.direct_solve(A, s["b"])
    en = np.sqrt(xs @ (A @ xs))
    assert np.sqrt((xl - xs) @ (A @ (xl - xs))) <= 1e-5 * en


@pytest.mark.parametrize("name", list(COARSE_PROBLEMS))
def test_learned_fcg_matches_oracle_fcg(torch, name):
    """A seeded network inside flexible CG: GPU against the oracle's FCG
    with the same network evaluated in FP64 on BF16-rounded weights."""
    print(f"[learned] oracle fcg {name}", flush=True)
    desc, s, S, P, Ac = coarse_case(name)
    _, pb, pc = _lib_case(name)
    theta = fcgen.unet_init(CH, 2, seed=7)
    m = fc.Model(theta, CH)
    pc.attach(m)
    xl, il = _learned_solve(torch, pb, pc)
    th = _oracle_theta(theta)
    G = desc["n"] // 2 + 1

    def corr(r):
        xin = L.network_input(desc, r, s["eta"])[None]
        return L.forward(th, xin, CH).ravel()

    xo, io = L.fcg(s["A"], s["b"], S, P, Ac, corr, tol=1e-8)
    assert il["status"] == "OK" and io["status"] == PCG.OK
    assert abs(il["iters"] - io["iters"]) <= max(2, 0.1 * io["iters"]), (il["iters"], io["iters"])
    assert il["rel_res_true"] <= 1.5e-8
    A = s["A"]
    xs = PCG.direct_solve(A, s["b"])
    en = np.sqrt(xs @ (A @ xs))
    assert np.sqrt((xl - xs) @ (A @ (xl - xs))) <= 1e-5 * en
    st = pc.learned_stats()
    assert st["applied"] == il["iters"] + 1
    assert st["dropped"] == 0


def test_trained_network_gain_and_fallback(torch):
    """Train on pairs (coarse Galerkin projections of the error) from three
    16^3 problems, then let plain Schwarz-PCG judge the network, inside
    flexible CG keeping 16 directions, on a fourth: the learned solve is kept only where it
    is faster, and otherwise FC_MODE_LEARNED runs exactly the plain solve.
    Prints what the trained network gains (or loses) in iterations and time."""
    from paper_1809_00828_amd import learned as LR
    print("[learned] gain test: data", flush=True)
    descs = [fcgen.porous_poisson_3d(500 + i, n=16, p=2, n_voids=24, rmin=0.04, rmax=0.1)
             for i in range(3)]
    xin, t, G = LR.training_set(descs, 80, kind="coarse")
    assert xin.shape == (240, 2, G ** 3) and G == 9
    m = fc.Model(fcgen.unet_init(CH, 2, seed=1), CH)
    hist = LR.train(m, xin, t, G, epochs=30, batch=8, lr=3e-4)
    print("[learned] loss", hist[0], "->", hist[-1], flush=True)
    assert hist[-1] < hist[0]
    desc = fcgen.porous_poisson_3d(599, n=16, p=2, n_voids=24, rmin=0.04, rmax=0.1)
    pb = fc.Problem.setup(desc)
    pc = fc.Precond(pb)
    pc.attach(m)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    use, ip, il = pc.validate(b, tol=1e-8, fcg_m=16)
    print(f"[learned] plain {ip['iters']} it {ip['ms_solve']:.2f} ms, learned {il['iters']} it "
          f"{il['ms_solve']:.2f} ms, network kept: {use}", flush=True)
    assert ip["status"] == "OK" and il["status"] == "OK"
    assert use == (il["ms_solve"] < ip["ms_solve"])
    x = torch.zeros_like(b)
    info = fc.pcg_solve(pb, pc, b, x, tol=1e-8, stop="residual", mode="learned", fcg_m=16)
    xp = torch.zeros_like(b)
    infp = fc.pcg_solve(pb, pc, b, xp, tol=1e-8, stop="residual", mode="f64")
    assert info["status"] == "OK"
    if use:
        assert info["fallbacks"] == 0 and info["iters"] == il["iters"]
    else:
        assert info["fallbacks"] == 1 and info["iters"] == infp["iters"]
        assert torch.equal(x, xp)


def test_fcg_m_above_limit_is_rejected(torch):
    _, pb, pc = _lib_case("pois8_p2")
    m = fc.Model(fcgen.unet_init(CH, 2, seed=7), CH)
    pc.attach(m)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    with pytest.raises(fc.FcError) as ei:
        fc.pcg_solve(pb, pc, b, x, tol=1e-8, stop="residual", mode="learned", fcg_m=65)
    assert ei.value.status == 1   # FC_E_ARG
    info = fc.pcg_solve(pb, pc, b, x, tol=1e-8, stop="residual", mode="learned", fcg_m=64)
    assert info["status"] == "OK"
