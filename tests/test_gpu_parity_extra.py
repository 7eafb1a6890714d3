"""GPU parity for degenerate settings of the preconditioner and of the
mixed-precision solver, and for the shared copies of repeated rows and
local inverses.

  * eta_bar < 0 keeps no element block (every eta_T >= 0), so Algorithm 1
    reduces to diagonal scaling: z = r / diag(A) on every unknown with a
    positive diagonal.  z is compared element by element to relative 1e-13,
    the bar of the assembled entries (the two assemblers sum the diagonal
    in different orders); the PCG iteration count must match the oracle's
    within +-2 at a tolerance where a relative perturbation of
    1e-15 of the preconditioner does not move the oracle's own count.
  * Iterative refinement on an uncut cube: every cell has eta_T = 1, so the
    row-mixed matrix holds no FP64 row at all.  The refinement must still
    reach the FP64 residual with no fallback to the FP64 matrix, and the
    solution must agree with the oracle's direct solve in the energy norm.
  * Shared copies: the same problem and preconditioner with every row and
    block read from its own copy and with bitwise-equal ones read from one
    copy, four at a time, give the same products and solves (bit for bit
    where the launch shapes agree) and match the oracle.
"""
import numpy as np
import pytest

import fcgen
import paper_1809_00828_amd as fc
from oracle import assemble, pcg, schwarz
from tests.gpu_common import energy, oracle_direct, oracle_system, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name", ["disk16_p2", "pois3d_p2", "elast3d_p2"])
def test_negative_eta_bar_is_diagonal_scaling(torch, name):
    print(f"[diag] {name}", flush=True)
    _, s = oracle_system(name)
    A = s["A"]
    S, fall = schwarz.compute_preconditioner(A, schwarz.select_blocks(
        s["elem_dofs"], s["eta"], -1.0))
    pb = fc.Problem.setup(oracle_system(name)[0])
    pc = fc.Precond(pb, eta_bar=-1.0)
    info = pc.info()
    assert info["n_blocks"] == 0
    assert info["n_fallback"] == fall.size
    r = np.random.default_rng(21).standard_normal(pb.n)
    z = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pc.apply_M(_dev(torch, r), z)
    torch.cuda.synchronize()
    ref = S @ r
    np.testing.assert_allclose(z.cpu().numpy(), ref, rtol=1e-13, atol=0.0)
    if name == "disk16_p2":
        # Jacobi on the alpha = 1e-10 disk needs ~1200 iterations and its
        # count moves by a few under rounding-level changes: z only
        return
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    res = fc.pcg_solve(pb, pc, b, x, tol=1e-8, check_every=8)
    torch.cuda.synchronize()
    _, io = pcg.pcg(A, s["b"], S, tol=1e-8)
    print(f"[diag] {name}: iters {res['iters']} (oracle {io['iters']})", flush=True)
    assert res["status"] == "OK", res
    assert abs(res["iters"] - io["iters"]) <= 2
    xr = oracle_direct(name)
    xo, _ = pcg.pcg(A, s["b"], S, tol=1e-8)
    # both iterates stop at the same rule: their errors against the direct
    # solution are of the same size
    assert energy(A, x.cpu().numpy() - xr) <= 2 * energy(A, xo - xr) + 1e-12 * energy(A, xr)


def test_refinement_on_uncut_cube(torch):
    """All rows of the row-mixed matrix are FP32 (no cell has eta_T < 1)."""
    d = fcgen.custom(3, 4, 2, "elasticity", 1e-8, shapes=[], clamp_zmin=True)
    s = assemble.assemble(d)
    assert np.all(s["eta"] == 1.0)
    A = s["A"]
    pb = fc.Problem.setup(d)
    pc = fc.Precond(pb, store=fc.STORE_F64 | fc.STORE_F32)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    np.testing.assert_allclose(b.cpu().numpy(), s["b"], rtol=1e-13,
                               atol=1e-13 * np.abs(s["b"]).max())
    tol = 1e-8
    x64 = torch.zeros_like(b)
    i64 = fc.pcg_solve(pb, pc, b, x64, tol=tol, stop="residual")
    x = torch.zeros_like(b)
    info = fc.pcg_solve(pb, pc, b, x, tol=tol, stop="residual", mode="ir_f32",
                        inner_tol=1e-4, maxit=200000)
    torch.cuda.synchronize()
    print(f"[ir uncut] iters {info['iters']} (fp64 {i64['iters']}), outer "
          f"{info['outer_iters']}, fallbacks {info['fallbacks']}", flush=True)
    assert info["status"] == "OK", info
    assert info["rel_res_true"] <= tol
    assert info["fallbacks"] == 0, info
    xr = np.linalg.solve(A.toarray(), s["b"])
    e64 = energy(A, x64.cpu().numpy() - xr) / energy(A, xr)
    e = energy(A, x.cpu().numpy() - xr) / energy(A, xr)
    assert e <= 10 * e64 + 1e-12


def test_shared_rows_give_the_same_products(torch, monkeypatch):
    """The same problem set up with the full matrix (FC_SPMV_SHARE=0) and
    with bitwise-equal rows kept once (FC_SPMV_SHARE=1): products and PCG
    solves agree bit for bit when both chose the same lanes per row (the
    set-up times the group width on each matrix), else to rounding."""
    d, s = oracle_system("elast3d_p2")
    monkeypatch.setenv("FC_SPMV_SHARE", "0")
    plain = fc.Problem.setup(d)
    monkeypatch.setenv("FC_SPMV_SHARE", "1")
    shared = fc.Problem.setup(d)
    ip, ish = plain.info(), shared.info()
    print(f"[share] rows {ish['shared_rows']} of {ish['n_dofs'] // 3}, values "
          f"{ish['shared_values']} of {ish['nnzb'] * 9}, row groups {ish['row_groups']}; "
          f"lanes {ip['spmv_group']} {ish['spmv_group']}", flush=True)
    assert 0 < ish["row_groups"] < ish["n_dofs"] // 3
    assert ip["shared_rows"] == 0 and ip["shared_values"] == 0
    assert 0 < ish["shared_rows"] < ish["n_dofs"] // 3
    same_group = ip["spmv_group"] == ish["spmv_group"]
    x = _dev(torch, np.random.default_rng(5).standard_normal(plain.n))
    y0 = torch.empty_like(x)
    y1 = torch.empty_like(x)
    plain.apply_A(x, y0)
    shared.apply_A(x, y1)
    torch.cuda.synchronize()
    a, b = y0.cpu().numpy(), y1.cpu().numpy()
    if same_group:
        assert a.tobytes() == b.tobytes()
    else:
        assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    ref = s["A"] @ x.cpu().numpy()
    assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max()
    res = []
    for pb in (plain, shared):
        pc = fc.Precond(pb)
        rhs = torch.empty(pb.n, dtype=torch.float64, device="cuda")
        pb.rhs(rhs)
        xs = torch.zeros_like(rhs)
        info = fc.pcg_solve(pb, pc, rhs, xs, tol=1e-10)
        torch.cuda.synchronize()
        res.append((info["iters"], xs.cpu().numpy()))
    # refinement on the row-mixed matrix: its FP32 rows read the FP32 copy
    # of the shared rows through the same offsets
    for pb in (plain, shared):
        pc = fc.Precond(pb, store=fc.STORE_F64 | fc.STORE_F32)
        rhs = torch.empty(pb.n, dtype=torch.float64, device="cuda")
        pb.rhs(rhs)
        xs = torch.zeros_like(rhs)
        info = fc.pcg_solve(pb, pc, rhs, xs, tol=1e-8, stop="residual", mode="ir_f32",
                            inner_tol=1e-4, maxit=200000)
        torch.cuda.synchronize()
        assert info["status"] == "OK" and info["fallbacks"] == 0, info
        res.append((info["iters"], xs.cpu().numpy()))
    for a, b in ((0, 1), (2, 3)):
        if same_group:
            assert res[a][0] == res[b][0]
            assert res[a][1].tobytes() == res[b][1].tobytes()
        else:
            assert abs(res[a][0] - res[b][0]) <= 2


def test_shared_block_inverses_give_the_same_products(torch, monkeypatch):
    """Block products reading bitwise-equal local inverses from one copy
    (FC_SCHWARZ_SHARE=1) against every block reading its own
    (FC_SCHWARZ_SHARE=0): z = S r and the PCG solve agree bit for bit, and
    z matches the oracle's S r.  Uncut 4^3-cell p = 3 elasticity (m = 192):
    its interior cells have equal element blocks."""
    d = fcgen.custom(3, 4, 3, "elasticity", 1e-8, shapes=[], clamp_zmin=True)
    s = assemble.assemble(d)
    pb = fc.Problem.setup(d)
    store = fc.STORE_F64 | fc.STORE_F32
    monkeypatch.setenv("FC_SCHWARZ_SHARE", "0")
    own = fc.Precond(pb, store=store)
    monkeypatch.setenv("FC_SCHWARZ_SHARE", "1")
    shared = fc.Precond(pb, store=store)
    io, ish = own.info(), shared.info()
    print(f"[share blocks] distinct {ish['shared_distinct_blocks']} (FP64), "
          f"{ish['shared_distinct_blocks32']} (FP32) of {ish['n_blocks']}", flush=True)
    assert io["shared_distinct_blocks"] == 0 and io["shared_distinct_blocks32"] == 0
    assert 0 < ish["shared_distinct_blocks"] < ish["n_blocks"]
    assert 0 < ish["shared_distinct_blocks32"] < ish["n_blocks"]
    # the FP64 products take the blocks with one copy four at a time
    assert ish["shared_distinct_blocks"] <= ish["block_groups"] < ish["n_blocks"]
    r = _dev(torch, np.random.default_rng(8).standard_normal(pb.n))
    z0 = torch.empty_like(r)
    z1 = torch.empty_like(r)
    own.apply_M(r, z0)
    shared.apply_M(r, z1)
    torch.cuda.synchronize()
    assert z0.cpu().numpy().tobytes() == z1.cpu().numpy().tobytes()
    S, _ = schwarz.compute_preconditioner(s["A"], schwarz.select_blocks(
        s["elem_dofs"], s["eta"], 1.0))
    ref = S @ r.cpu().numpy()
    assert np.linalg.norm(z1.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)
    # FP64 PCG and PCG with the FP32 copy of the inverses
    for kw in ({}, {"mode": "s_f32", "stop": "residual", "tol": 1e-8}):
        out = []
        for pc in (own, shared):
            b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
            pb.rhs(b)
            x = torch.zeros_like(b)
            info = fc.pcg_solve(pb, pc, b, x, **{"tol": 1e-10, **kw})
            torch.cuda.synchronize()
            assert info["status"] == "OK", info
            out.append((info["iters"], x.cpu().numpy().tobytes()))
        assert out[0] == out[1], kw
