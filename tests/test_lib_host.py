"""CPU checks of the native library: it loads, exports every symbol the
C header declares, and its host assembler (written independently of the
oracle) reproduces the oracle's system.  No GPU call is made."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import fcgen
import paper_1809_00828_amd as fc
from oracle import assemble

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "fc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fc_[A-Za-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = fc.load()
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(fc.EXPORTS) == declared


def bsr_to_csr(e):
    bd = e["bsr_dim"]
    rp, col, val = e["rowptr"], e["col"], e["val"]
    nbr = len(rp) - 1
    rows = np.repeat(np.arange(nbr), np.diff(rp))
    R = rows[:, None, None] * bd + np.arange(bd)[None, :, None] + 0 * np.arange(bd)[None, None, :]
    Cc = col[:, None, None] * bd + np.arange(bd)[None, None, :] + 0 * np.arange(bd)[None, :, None]
    return sp.csr_matrix((val.ravel(), (R.ravel(), Cc.ravel())), shape=(nbr * bd, nbr * bd))


BIG_VOID = [{"centre": [0.5, 0.52, 0.48], "semi": [0.33, 0.33, 0.33]}]

CASES = {
    "disk2d_p2": lambda: fcgen.disk_poisson_2d(0),
    "disk2d_p4_seed3": lambda: fcgen.disk_poisson_2d(3, n=8, p=4),
    "elastic3d_p2": lambda: fcgen.porous_elasticity_3d(seed=2, n=3, p=2, n_voids=2,
                                                       rmin=0.1, rmax=0.15),
    "elastic3d_p3": lambda: fcgen.porous_elasticity_3d(seed=3, n=4, p=3, n_voids=3,
                                                       rmin=0.05, rmax=0.12),
    "poisson3d_p2": lambda: fcgen.porous_poisson_3d(seed=1, n=4, p=2, n_voids=3,
                                                    rmin=0.08, rmax=0.15),
    "ellipse_inclusions": lambda: fcgen.batch_poisson(seed=1, count=1, min_dofs=0,
                                                      max_dofs=3000)[0],
    # a void that holds eight cells entirely, their functions removed
    "elastic3d_discard_alpha0": lambda: fcgen.custom(
        3, 6, 2, "elasticity", 0.0, shapes=BIG_VOID, clamp_zmin=True, discard_fictitious=True),
    "poisson3d_discard": lambda: fcgen.custom(
        3, 6, 2, "poisson", 1e-12, shapes=BIG_VOID, discard_fictitious=True),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_host_assembly_matches_oracle(name):
    d = CASES[name]()
    o = assemble.assemble(d)
    e = fc.HostSystem(d).export()
    A = bsr_to_csr(e)
    scale = abs(o["A"]).max()
    assert abs(A - o["A"]).max() <= 1e-13 * scale
    assert abs(A - A.T).max() <= 1e-15 * scale
    np.testing.assert_allclose(e["rhs"], o["b"], rtol=0, atol=1e-13 * max(abs(o["b"]).max(), 1e-300))
    np.testing.assert_array_equal(e["elem_dofs"], o["elem_dofs"])
    np.testing.assert_allclose(e["eta"], o["eta"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(e["eta"] == 1.0, o["eta"] == 1.0)
    np.testing.assert_array_equal(e["eta"] == 0.0, o["eta"] == 0.0)


def test_host_assembly_rejects_bad_description():
    d = fcgen.custom(2, 4, 0, "poisson")
    with pytest.raises(fc.FcError) as ei:
        fc.HostSystem(d)
    assert ei.value.status == 1
