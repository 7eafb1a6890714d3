"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Sizes span several tiles and ragged tails of every kernel while the oracle
still finishes in seconds.  Tolerances:
  * y = A x: relative 1e-13 (assembly and SpMV are both rounding-level).
  * local inverses: both sides are backward stable, so they differ by
    ~ m * eps_mach * kappa(A_B) relative; the test bounds the difference by
    1e-15 * m * kappa(A_B) + 1e-13 and requires identical dropped counts.
  * z = S r: bounded by the block-level tolerance summed over the blocks.
  * PCG solutions: relative energy-norm difference <= 1e-10 (the parity bar
    on the solution) wherever the largest block condition number is at most
    1e10; iteration counts within +-2 up to 1e8 (and on the 16^2 disk),
    within 15 % above it, where the oracle's own count moves by several
    percent when only its eigensolver changes.
"""
import numpy as np
import pytest

import paper_1809_00828_amd as fc
from oracle import pcg, schwarz
from tests.gpu_common import (ITERATION_DETERMINED_KAPPA, PROBLEMS, WELL_DETERMINED_KAPPA,
                              energy, max_block_kappa, oracle_direct, oracle_precond,
                              oracle_system, require_gpu)

pytestmark = pytest.mark.gpu

NAMES = sorted(PROBLEMS)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


_lib_cache = {}


def lib_problem(name):
    if name not in _lib_cache:
        d, _ = oracle_system(name)
        _lib_cache[name] = fc.Problem.setup(d)
    return _lib_cache[name]


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name", NAMES)
def test_apply_A(torch, name):
    print(f"[apply_A] {name}", flush=True)
    _, s = oracle_system(name)
    pb = lib_problem(name)
    n = pb.n
    assert n == s["A"].shape[0]
    x = np.random.default_rng(11).standard_normal(n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    pb.apply_A(_dev(torch, x), y)
    torch.cuda.synchronize()
    ref = s["A"] @ x
    err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-13, err


@pytest.mark.parametrize("name", NAMES)
def test_rhs_and_eta(torch, name):
    _, s = oracle_system(name)
    pb = lib_problem(name)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    torch.cuda.synchronize()
    bo = s["b"]
    np.testing.assert_allclose(b.cpu().numpy(), bo, rtol=0,
                               atol=1e-13 * max(abs(bo).max(), 1e-300))
    np.testing.assert_allclose(pb.eta(), s["eta"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", NAMES)
def test_local_inverses(torch, name):
    print(f"[local_inverses] {name}", flush=True)
    _, s = oracle_system(name)
    pc = fc.Precond(lib_problem(name))
    info = pc.info()
    assert info["n_blocks"] == len(s["eta"])
    assert info["n_fallback"] == 0
    rng = np.random.default_rng(5)
    picks = sorted(set(rng.integers(0, info["n_blocks"], size=8).tolist()) | {0, info["n_blocks"] - 1})
    dropped = 0
    for k in range(info["n_blocks"]):
        B = s["elem_dofs"][k]
        AB = schwarz.extract_submatrix(s["A"], B)
        lam = np.linalg.eigvalsh(AB)
        dropped += int(np.sum(~(lam > 1e-13 * lam.max())))
        if k not in picks:
            continue
        ref = schwarz.pseudo_inverse(AB)
        got = pc.block_inverse(k)
        kept = lam[lam > 1e-13 * lam.max()]
        kappa = kept.max() / kept.min()
        tol = 1e-15 * AB.shape[0] * kappa + 1e-13
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= tol, (k, err, kappa)
        np.testing.assert_allclose(got, got.T, rtol=0, atol=1e-14 * abs(got).max())
    assert info["n_dropped"] == dropped


def _block_bound(s, blocks, r):
    """Norm-wise bound on |S_gpu r - S_oracle r| implied by the block-level
    tolerance of test_local_inverses: sum_B tol_B ||P_B||_F ||r_B||."""
    A = s["A"]
    total = 0.0
    for B in blocks:
        AB = schwarz.extract_submatrix(A, B)
        lam = np.linalg.eigvalsh(AB)
        if lam.max() <= 0:
            continue
        kept = lam[lam > 1e-13 * lam.max()]
        kappa = kept.max() / kept.min()
        tol = 1e-15 * AB.shape[0] * kappa + 1e-13
        total += tol * np.sqrt(np.sum(1.0 / kept ** 2)) * np.linalg.norm(r[B])
    return total


@pytest.mark.parametrize("name", NAMES)
def test_apply_M(torch, name):
    """z = S r.  With alpha = 1e-10 the local inverses carry entries ~1/alpha
    on fictitious unknowns, so the two sides can only agree to rounding of
    those entries: the difference is bounded by the block-level tolerance
    summed over the blocks."""
    print(f"[apply_M] {name}", flush=True)
    _, s = oracle_system(name)
    S, _, blocks = oracle_precond(name)
    pc = fc.Precond(lib_problem(name))
    n = S.shape[0]
    r = np.random.default_rng(12).standard_normal(n)
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    pc.apply_M(_dev(torch, r), z)
    torch.cuda.synchronize()
    ref = S @ r
    d = z.cpu().numpy() - ref
    assert np.linalg.norm(d) <= _block_bound(s, blocks, r)
    assert np.linalg.norm(d) <= 1e-6 * np.linalg.norm(ref)


def _solve(torch, name, tol, maxit=100000, stop="precond", **kw):
    d, s = oracle_system(name)
    pb = lib_problem(name)
    pc = fc.Precond(pb, **kw)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros(pb.n, dtype=torch.float64, device="cuda")
    info = fc.pcg_solve(pb, pc, b, x, tol=tol, maxit=maxit, stop=stop, check_every=8)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


@pytest.mark.parametrize("name", NAMES)
def test_pcg_matches_oracle(torch, name):
    print(f"[pcg] {name}", flush=True)
    _, s = oracle_system(name)
    A, b = s["A"], s["b"]
    S, _, _ = oracle_precond(name)
    tol = 1e-10
    x, info = _solve(torch, name, tol)
    xo, io = pcg.pcg(A, b, S, tol=tol)
    assert info["status"] == "OK", info
    kappa = max_block_kappa(name)
    strict = name == "disk16_p2" or kappa <= WELL_DETERMINED_KAPPA
    print(f"[pcg] {name}: iters {info['iters']} (oracle {io['iters']}), largest block "
          f"kappa {kappa:.1e}", flush=True)
    if name == "disk16_p2" or kappa <= ITERATION_DETERMINED_KAPPA:
        assert abs(info["iters"] - io["iters"]) <= 2, (info["iters"], io["iters"])
    else:
        # local inverses fixed by FP64 data only to eps*kappa; the CPU tests
        # of tests/test_oracle_conditioning.py show the oracle's own count
        # moving by this much when only its eigensolver changes
        assert abs(info["iters"] - io["iters"]) <= max(2, 0.15 * io["iters"]), \
            (info["iters"], io["iters"])
    # both solved tighter: the two solutions agree in the energy norm.  On
    # ill-determined problems the directions the pseudo-inverses drop or
    # barely keep differ between the two eigensolvers, and the paper's own
    # remark on the stabilised preconditioner bounds the attainable energy
    # error only by sqrt(eps); there the bar is 1e-8.
    x2, info2 = _solve(torch, name, 1e-13)
    xo2, _ = pcg.pcg(A, b, S, tol=1e-13)
    xr = oracle_direct(name)
    bar = 1e-10 if strict else 1e-8
    assert energy(A, x2 - xo2) <= bar * energy(A, xo2)
    assert energy(A, x2 - xr) <= max(bar, 1e-9) * energy(A, xr)
    assert info2["rel_res_true"] <= 1e-9


@pytest.mark.parametrize("name", ["disk16_p2", "elast3d_p3", "elast3d_p3_thin"])
def test_pcg_fixed_iterations_match(torch, name):
    """Iterate k of both sides, k well before convergence."""
    _, s = oracle_system(name)
    A, b = s["A"], s["b"]
    S, _, _ = oracle_precond(name)
    k = 15
    x, info = _solve(torch, name, 0.0, maxit=k)
    xo, io = pcg.pcg(A, b, S, tol=0.0, maxit=k)
    assert info["status"] == "E_NOTCONV" and info["iters"] == k == io["iters"]
    tol = 1e-10 if max_block_kappa(name) <= WELL_DETERMINED_KAPPA else 1e-9
    assert energy(A, x - xo) <= tol * energy(A, xo)


def test_pcg_is_bitwise_reproducible(torch):
    x1, i1 = _solve(torch, "pois3d_p2", 1e-10)
    x2, i2 = _solve(torch, "pois3d_p2", 1e-10)
    assert i1["iters"] == i2["iters"]
    np.testing.assert_array_equal(x1, x2)


def test_residual_stop_rule(torch):
    name = "disk16_p2"
    _, s = oracle_system(name)
    S, _, _ = oracle_precond(name)
    x, info = _solve(torch, name, 1e-9, stop="residual")
    _, io = pcg.pcg(s["A"], s["b"], S, tol=1e-9, stop="residual")
    assert info["status"] == "OK"
    assert abs(info["iters"] - io["iters"]) <= 2
    assert info["rel_res_true"] <= 2e-9


def test_zero_rhs_gives_zero_solution(torch):
    pb = lib_problem("disk16_p2")
    pc = fc.Precond(pb)
    b = torch.zeros(pb.n, dtype=torch.float64, device="cuda")
    x = torch.full((pb.n,), 7.0, dtype=torch.float64, device="cuda")
    info = fc.pcg_solve(pb, pc, b, x, tol=1e-10)
    assert info["status"] == "OK" and info["iters"] == 0
    assert float(x.abs().max()) == 0.0


def test_eta_bar_fallback_matches_oracle(torch):
    name = "disk16_p2"
    _, s = oracle_system(name)
    S, fall, blocks = oracle_precond(name, eta_bar=0.5)
    pb = lib_problem(name)
    pc = fc.Precond(pb, eta_bar=0.5)
    info = pc.info()
    assert info["n_blocks"] == len(blocks)
    assert info["n_fallback"] == fall.size > 0
    r = np.random.default_rng(3).standard_normal(pb.n)
    z = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pc.apply_M(_dev(torch, r), z)
    torch.cuda.synchronize()
    ref = S @ r
    d = z.cpu().numpy() - ref
    assert np.linalg.norm(d) <= _block_bound(s, blocks, r)
    x, inf2 = _solve(torch, name, 1e-10, eta_bar=0.5)
    _, io = pcg.pcg(s["A"], s["b"], S, tol=1e-10)
    assert abs(inf2["iters"] - io["iters"]) <= 2


def test_setup_from_oracle_matrix(torch):
    """The solver on the oracle's own matrix (isolates the solver from the
    assembler)."""
    from tests.gpu_common import csr_to_bsr_arrays
    name = "elast3d_p2"
    d, s = oracle_system(name)
    bd = 3
    rowptr, col, val = csr_to_bsr_arrays(s["A"], bd)
    pb = fc.Problem.from_matrix(s["A"].shape[0], bd, rowptr, col, val, s["b"],
                                s["elem_dofs"], s["eta"])
    pc = fc.Precond(pb)
    b = _dev(torch, s["b"])
    x = torch.zeros_like(b)
    info = fc.pcg_solve(pb, pc, b, x, tol=1e-10)
    S, _, _ = oracle_precond(name)
    xo, io = pcg.pcg(s["A"], s["b"], S, tol=1e-10)
    assert info["status"] == "OK" and abs(info["iters"] - io["iters"]) <= 2
    xr = oracle_direct(name)
    assert energy(s["A"], x.cpu().numpy() - xr) <= 1e-8 * energy(s["A"], xr)


def test_invalid_arguments_raise(torch):
    pb = lib_problem("disk16_p2")
    x = torch.zeros(pb.n, dtype=torch.float64, device="cuda")
    with pytest.raises(fc.FcError):
        pb.apply_A(x, x)
    with pytest.raises(fc.FcError):
        fc.Precond(pb, eps=-1.0)


# ------------------------------------------------------ precision forms
FORMS = ["s_f32", "s_bf16", "ir_f32", "ir_bf16"]


@pytest.mark.parametrize("name", ["disk16_p2", "elast3d_p3", "pois3d_p2"])
@pytest.mark.parametrize("mode", FORMS)
def test_precision_forms_reach_tolerance(torch, name, mode):
    """Low-precision forms solve to the same FP64 residual; their error
    against the oracle's direct solution is reported and must stay within
    10x of what plain FP64 PCG reaches at the same tolerance."""
    print(f"[form] {name} {mode}", flush=True)
    _, s = oracle_system(name)
    A = s["A"]
    pb = lib_problem(name)
    pc = fc.Precond(pb, store=fc.STORE_F64 | fc.STORE_F32 | fc.STORE_BF16)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    tol = 1e-8
    x64 = torch.zeros_like(b)
    i64 = fc.pcg_solve(pb, pc, b, x64, tol=tol, stop="residual")
    x = torch.zeros_like(b)
    info = fc.pcg_solve(pb, pc, b, x, tol=tol, stop="residual", mode=mode, inner_tol=1e-2,
                        maxit=200000)
    assert info["status"] == "OK", info
    assert info["rel_res_true"] <= tol
    xr = oracle_direct(name)
    e64 = energy(A, x64.cpu().numpy() - xr) / energy(A, xr)
    e = energy(A, x.cpu().numpy() - xr) / energy(A, xr)
    print(f"[form] {name} {mode}: iters {info['iters']} (fp64 {i64['iters']}), "
          f"outer {info['outer_iters']}, fallbacks {info['fallbacks']}, "
          f"energy error {e:.2e} (fp64 {e64:.2e})", flush=True)
    assert e <= 10 * e64 + 1e-12
    if mode.startswith("ir"):
        # the row-mixed matrix keeps the cut cells' rows in FP64: no step of
        # the refinement has to fall back to the FP64 matrix
        assert info["fallbacks"] == 0, info


def test_low_precision_copies_required(torch):
    pb = lib_problem("disk16_p2")
    pc = fc.Precond(pb)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    with pytest.raises(fc.FcError):
        fc.pcg_solve(pb, pc, b, x, mode="s_bf16", raise_on_error=True)


def _min_rel_pivot(M):
    """Smallest Cholesky pivot of M relative to its largest diagonal entry
    (negative where the factorisation breaks down)."""
    M = M.copy()
    n = M.shape[0]
    dmax = max(float(np.max(np.diag(M))), 1e-300)
    worst = np.inf
    for k in range(n):
        d = M[k, k]
        worst = min(worst, d / dmax)
        if d <= 0:
            return worst
        l = M[k + 1:, k] / np.sqrt(d)
        M[k + 1:, k + 1:] -= np.outer(l, l)
        M[k + 1:, k] = l
    return worst


@pytest.mark.parametrize("name", ["elast3d_p2", "pois3d_p3", "disk7_p4"])
def test_f32_copy_certificate_counts(torch, name):
    """The FP32 copy keeps exactly the blocks whose rounded, diagonally
    scaled inverse factors with every pivot above 1e-10 of the largest
    diagonal entry.  Recomputed here from each block's FP64 inverse (the
    library's own: on ill-determined blocks the oracle's differs by
    eps * kappa, enough to move a pivot across the threshold) and the
    oracle's matrix diagonal: blocks far from the threshold on either side
    must be classified the same way."""
    print(f"[f32 certificate] {name}", flush=True)
    _, s = oracle_system(name)
    A = s["A"]
    S, _, blocks = oracle_precond(name)
    pc = fc.Precond(lib_problem(name), store=fc.STORE_F64 | fc.STORE_F32)
    clearly_bad = maybe = 0
    for k, B in enumerate(blocks):
        AB = schwarz.extract_submatrix(A, B)
        P = pc.block_inverse(k)
        dg = np.sqrt(np.maximum(np.diag(AB), 0.0))
        dg[dg == 0] = 1.0
        Ph = (P * dg[:, None] * dg[None, :]).astype(np.float32).astype(np.float64)
        piv = _min_rel_pivot(Ph)
        if piv < 1e-12:
            clearly_bad += 1
        elif piv < 1e-8:
            maybe += 1
    info = pc.info()
    assert info["n_f32_blocks"] + info["n_f32_from_f64"] == info["n_blocks"]
    assert clearly_bad <= info["n_f32_from_f64"] <= clearly_bad + maybe, \
        (info, clearly_bad, maybe)
