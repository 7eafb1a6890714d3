"""Full-size checks on the benchmark workload: 3-D elasticity on 32^3 cells,
p = 3, 64 voids, 2,738,019 unknowns.  They run in the launch configuration
that bench.py times, on outputs the oracle can compute one by one.
- Sampled rows of y = A x against rows assembled from the oracle's element
  systems of the cells that touch each sampled node.
- Sampled local inverses P_B against the oracle's pseudo-inverse of A_B,
  assembled from the 27 cells around the block.
- z = S r at the block's interior unknowns, which belong to that block
  alone.
- The benchmark solve: true residual at or below the tolerance, and bitwise
  reproducible."""
import itertools

import numpy as np
import pytest

import fcgen
import paper_1809_00828_amd as fc
from oracle import assemble as ASM
from oracle import schwarz as SCH
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu

DESC = fcgen.porous_elasticity_3d(seed=0)
N, P = DESC["n"], DESC["p"]
N1 = P * N + 1


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lib(torch):
    print("[fullsize] host assembly + upload", flush=True)
    pb = fc.HostSystem(DESC).upload()
    pc = fc.Precond(pb)
    eta = pb.eta()
    return pb, pc, eta


_cache = {}


def element(cell):
    if cell not in _cache:
        Ke, _, _ = ASM.element_system(DESC, cell)
        _cache[cell] = (Ke, ASM.element_dofs(DESC, cell))
    return _cache[cell]


def local_rows(dofs, cells):
    """Rows of the assembled, clamped A for `dofs`, from the element
    systems of `cells` (which must hold every cell touching them)."""
    clamped = set(ASM.clamped_dofs(DESC).tolist())
    rows = {int(d): {} for d in dofs}
    for c in cells:
        Ke, ed = element(c)
        for a, da in enumerate(ed):
            da = int(da)
            if da not in rows:
                continue
            r = rows[da]
            for b, db in enumerate(ed):
                r[int(db)] = r.get(int(db), 0.0) + Ke[a, b]
    for d, r in rows.items():
        if d in clamped:
            rows[d] = {d: r[d]}
        else:
            for c in list(r):
                if c in clamped:
                    del r[c]
    return rows


def cells_of_node(g):
    """Cells whose closure contains lattice point g = (gx, gy, gz)."""
    ranges = []
    for gk in g:
        e = gk // P
        cand = {e, e - 1} if gk % P == 0 else {e}
        ranges.append(sorted(c for c in cand if 0 <= c < N))
    return list(itertools.product(*ranges))


def test_spmv_sampled_rows(torch, lib):
    pb, _, _ = lib
    rng = np.random.default_rng(31)
    x = rng.standard_normal(pb.n)
    y = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.apply_A(torch.as_tensor(x, device="cuda"), y)
    y = y.cpu().numpy()
    nodes = [tuple(int(v) for v in rng.integers(0, N1, size=3)) for _ in range(12)]
    nodes += [(0, 0, 0), (N1 - 1, N1 - 1, N1 - 1), (N1 // 2, N1 // 2, 0), (5, 7, N1 - 1)]
    for g in nodes:
        node = g[0] + N1 * (g[1] + N1 * g[2])
        dofs = [3 * node + c for c in range(3)]
        cells = [(cx, cy, cz) for (cx, cy, cz) in cells_of_node(g)]
        rows = local_rows(dofs, cells)
        for d in dofs:
            ref = sum(v * x[c] for c, v in rows[d].items())
            scale = sum(abs(v * x[c]) for c, v in rows[d].items())
            assert abs(y[d] - ref) <= 1e-13 * scale + 1e-300, (g, d, y[d], ref)


def _neighbourhood(cell):
    return [tuple(c + o for c, o in zip(cell, off))
            for off in itertools.product((-1, 0, 1), repeat=3)
            if all(0 <= c + o < N for c, o in zip(cell, off))]


def _pick_blocks(eta):
    """One uncut, one cut and (if any) one fully fictitious cell."""
    rng = np.random.default_rng(32)
    out = []
    for sel in (eta == 1.0, (eta > 0.0) & (eta < 1.0), eta == 0.0):
        idx = np.flatnonzero(sel)
        if idx.size:
            out.append(int(rng.choice(idx)))
    return out


def test_local_inverse_and_apply_sampled_blocks(torch, lib):
    pb, pc, eta = lib
    rng = np.random.default_rng(33)
    r = rng.standard_normal(pb.n)
    z = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pc.apply_M(torch.as_tensor(r, device="cuda"), z)
    z = z.cpu().numpy()
    for k in _pick_blocks(eta):
        cell = (k % N, (k // N) % N, k // (N * N))
        print(f"[fullsize] block {k} cell {cell} eta {eta[k]:.3f}", flush=True)
        _, ed = element(cell)
        rows = local_rows(ed, _neighbourhood(cell))
        AB = np.array([[rows[int(a)].get(int(b), 0.0) for b in ed] for a in ed])
        ref = SCH.pseudo_inverse(AB)
        got = pc.block_inverse(k)
        lam = np.linalg.eigvalsh(AB)
        kept = lam[lam > 1e-13 * lam.max()]
        kappa = kept.max() / kept.min()
        tol = 1e-15 * AB.shape[0] * kappa + 1e-13
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= tol, (k, err, kappa)
        # unknowns interior to the cell belong to this block only
        zr = ref @ r[ed]
        for a, d in enumerate(ed):
            node = int(d) // 3
            g = (node % N1, (node // N1) % N1, node // (N1 * N1))
            if all(gk % P != 0 for gk in g):
                bound = tol * np.linalg.norm(ref) * np.linalg.norm(r[ed]) + 1e-14 * abs(zr[a])
                assert abs(z[int(d)] - zr[a]) <= bound, (k, int(d), z[int(d)], zr[a])


def test_benchmark_solve_properties(torch, lib):
    """The solve bench.py times: residual stop at 1e-8 with timing events."""
    pb, pc, _ = lib
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    xs = []
    for _ in range(2):
        x = torch.zeros_like(b)
        info = fc.pcg_solve(pb, pc, b, x, tol=1e-8, stop="residual", timing=True)
        print(f"[fullsize] solve {info['iters']} iterations, rel res {info['rel_res_true']:.3e}",
              flush=True)
        assert info["status"] == "OK"
        assert info["rel_res_true"] <= 1e-8
        xs.append(x)
    assert torch.equal(xs[0], xs[1])
