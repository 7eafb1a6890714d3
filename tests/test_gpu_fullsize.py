"""Full-size checks on the benchmark workloads, in the launch configuration
that bench.py times, on outputs the oracle can compute one by one:
- 3-D elasticity on 32^3 cells, p = 3, 64 voids (2,738,019 unknowns);
- 3-D Poisson on 64^3 cells, p = 2, 64 voids (2,146,689 unknowns), the
  learned form's evaluation problem.
Checked are:
- sampled rows of y = A x against rows assembled from the oracle's element
  systems of the cells that touch each sampled node;
- sampled local inverses P_B against the oracle's pseudo-inverse of A_B,
  assembled from the 27 cells around the block;
- z = S r at the block's interior unknowns, which belong to that block
  alone;
- the plain solve: true residual at or below the tolerance, and bitwise
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

WORKLOADS = {
    "elastic32_p3": lambda: fcgen.porous_elasticity_3d(seed=0),
    "poisson64_p2": lambda: fcgen.porous_poisson_3d(100, n=64, p=2),
}


class Workload:
    def __init__(self, name):
        self.name = name
        self.desc = WORKLOADS[name]()
        self.n, self.p = self.desc["n"], self.desc["p"]
        self.n1 = self.p * self.n + 1
        self.bd = 3 if self.desc["pde"] == "elasticity" else 1
        self.cache = {}
        self.clamped = set(ASM.clamped_dofs(self.desc).tolist())

    def element(self, cell):
        if cell not in self.cache:
            Ke, _, _ = ASM.element_system(self.desc, cell)
            self.cache[cell] = (Ke, ASM.element_dofs(self.desc, cell))
        return self.cache[cell]

    def local_rows(self, dofs, cells):
        """Rows of the assembled, clamped A for `dofs`, from the element
        systems of `cells` (which must hold every cell touching them)."""
        rows = {int(d): {} for d in dofs}
        for c in cells:
            Ke, ed = self.element(c)
            for a, da in enumerate(ed):
                da = int(da)
                if da not in rows:
                    continue
                r = rows[da]
                for b, db in enumerate(ed):
                    r[int(db)] = r.get(int(db), 0.0) + Ke[a, b]
        for d, r in rows.items():
            if d in self.clamped:
                rows[d] = {d: r[d]}
            else:
                for c in list(r):
                    if c in self.clamped:
                        del r[c]
        return rows

    def cells_of_node(self, g):
        """Cells whose closure contains lattice point g = (gx, gy, gz)."""
        ranges = []
        for gk in g:
            e = gk // self.p
            cand = {e, e - 1} if gk % self.p == 0 else {e}
            ranges.append(sorted(c for c in cand if 0 <= c < self.n))
        return list(itertools.product(*ranges))

    def neighbourhood(self, cell):
        return [tuple(c + o for c, o in zip(cell, off))
                for off in itertools.product((-1, 0, 1), repeat=3)
                if all(0 <= c + o < self.n for c, o in zip(cell, off))]


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module", params=list(WORKLOADS))
def lib(request, torch):
    wl = Workload(request.param)
    print(f"[fullsize] {wl.name}: host assembly + upload", flush=True)
    pb = fc.HostSystem(wl.desc).upload()
    pc = fc.Precond(pb)
    return wl, pb, pc, pb.eta()


def test_spmv_sampled_rows(torch, lib):
    wl, pb, _, _ = lib
    rng = np.random.default_rng(31)
    x = rng.standard_normal(pb.n)
    y = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.apply_A(torch.as_tensor(x, device="cuda"), y)
    y = y.cpu().numpy()
    N1 = wl.n1
    nodes = [tuple(int(v) for v in rng.integers(0, N1, size=3)) for _ in range(12)]
    nodes += [(0, 0, 0), (N1 - 1, N1 - 1, N1 - 1), (N1 // 2, N1 // 2, 0), (5, 7, N1 - 1)]
    # rows interior to a cell along every direction (4 x 4 x 4 blocks each)
    nodes += [(1, 1, 1), (2, 1, 1), (49, 50, 52), (50, 50, 52), (N1 - 3, N1 - 2, N1 - 2)]
    for g in nodes:
        node = g[0] + N1 * (g[1] + N1 * g[2])
        dofs = [wl.bd * node + c for c in range(wl.bd)]
        rows = wl.local_rows(dofs, wl.cells_of_node(g))
        for d in dofs:
            ref = sum(v * x[c] for c, v in rows[d].items())
            scale = sum(abs(v * x[c]) for c, v in rows[d].items())
            assert abs(y[d] - ref) <= 1e-13 * scale + 1e-300, (wl.name, g, d, y[d], ref)


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
    wl, pb, pc, eta = lib
    rng = np.random.default_rng(33)
    r = rng.standard_normal(pb.n)
    z = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pc.apply_M(torch.as_tensor(r, device="cuda"), z)
    z = z.cpu().numpy()
    N, N1, P = wl.n, wl.n1, wl.p
    for k in _pick_blocks(eta):
        cell = (k % N, (k // N) % N, k // (N * N))
        print(f"[fullsize] {wl.name} block {k} cell {cell} eta {eta[k]:.3f}", flush=True)
        _, ed = wl.element(cell)
        rows = wl.local_rows(ed, wl.neighbourhood(cell))
        AB = np.array([[rows[int(a)].get(int(b), 0.0) for b in ed] for a in ed])
        ref = SCH.pseudo_inverse(AB)
        got = pc.block_inverse(k)
        lam = np.linalg.eigvalsh(AB)
        kept = lam[lam > 1e-13 * lam.max()]
        kappa = kept.max() / kept.min()
        tol = 1e-15 * AB.shape[0] * kappa + 1e-13
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= tol, (wl.name, k, err, kappa)
        # unknowns interior to the cell belong to this block only
        zr = ref @ r[ed]
        for a, d in enumerate(ed):
            node = int(d) // wl.bd
            g = (node % N1, (node // N1) % N1, node // (N1 * N1))
            if all(gk % P != 0 for gk in g):
                bound = tol * np.linalg.norm(ref) * np.linalg.norm(r[ed]) + 1e-14 * abs(zr[a])
                assert abs(z[int(d)] - zr[a]) <= bound, (wl.name, k, int(d), z[int(d)], zr[a])


def test_benchmark_solve_properties(torch, lib):
    """The solve bench.py times: residual stop at 1e-8 with timing events."""
    wl, pb, pc, _ = lib
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    xs = []
    for _ in range(2):
        x = torch.zeros_like(b)
        info = fc.pcg_solve(pb, pc, b, x, tol=1e-8, stop="residual", timing=True)
        print(f"[fullsize] {wl.name} solve {info['iters']} iterations, rel res "
              f"{info['rel_res_true']:.3e}", flush=True)
        assert info["status"] == "OK"
        assert info["rel_res_true"] <= 1e-8
        xs.append(x)
    assert torch.equal(xs[0], xs[1])
