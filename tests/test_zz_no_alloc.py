"""The allocation-free solve (fc_pcg_solve_noalloc) against fc_pcg_solve,
through the C ABI: two calls in a row on one GPU, the second on a smaller
problem, each giving bit for bit the iterate, iteration count and residual
of the allocating entry point on the same problem (the same kernels and
launch shapes, launched directly instead of from a captured graph); a
problem above the scratch maximum is rejected on the host."""
import numpy as np
import pytest

import fcgen
import paper_1809_00828_amd as fc
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _pair(torch, desc, tol, stop):
    pb = fc.Problem.setup(desc)
    pc = fc.Precond(pb)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x_ref = torch.zeros_like(b)
    ref = fc.pcg_solve(pb, pc, b, x_ref, tol=tol, stop=stop, check_every=16)
    # garbage in x: the entry point must start from x = 0 itself
    x = torch.full_like(b, 3.0)
    got = fc.pcg_solve_noalloc(pb, pc, b, x, tol=tol, stop=stop, check_every=16)
    torch.cuda.synchronize()
    return pb.n, ref, got, x_ref.cpu().numpy(), x.cpu().numpy()


def test_noalloc_matches_pcg_solve_twice(torch):
    # first the larger problem (3-D p = 3 elasticity, 6,591 unknowns), then
    # a smaller one (2-D disk, 1,089 unknowns): the second call reuses the
    # scratch the first one left behind
    cases = [(fcgen.porous_elasticity_3d(seed=4, n=4, p=3, n_voids=3, rmin=0.06, rmax=0.12),
              1e-10, "precond"),
             (fcgen.disk_poisson_2d(0), 1e-9, "residual")]
    sizes = []
    for desc, tol, stop in cases:
        n, ref, got, xr, xg = _pair(torch, desc, tol, stop)
        print(f"[noalloc] n {n}: iters {got['iters']} (allocating {ref['iters']}), "
              f"status {got['status']}, rel res {got['rel_res_true']:.3e}", flush=True)
        sizes.append(n)
        assert got["status"] == ref["status"] == "OK"
        assert got["iters"] == ref["iters"]
        assert got["rel_res_true"] == ref["rel_res_true"]
        assert xg.tobytes() == xr.tobytes()
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_problems_above_the_scratch(torch):
    # 2-D p = 1 Poisson on 800^2 cells: 641,601 unknowns > 2^19
    desc = fcgen.custom(2, 800, 1, "poisson", 1e-10, shapes=[])
    pb = fc.Problem.setup(desc)
    assert pb.n > (1 << 19)
    pc = fc.Precond(pb)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    with pytest.raises(fc.FcError) as ei:
        fc.pcg_solve_noalloc(pb, pc, b, x, tol=1e-8)
    assert ei.value.status == 7
    assert "scratch maximum" in str(ei.value)
