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


@pytest.mark.parametrize("desc", [
    lambda: fcgen.disk_poisson_2d(0),
    lambda: fcgen.porous_elasticity_3d(seed=3, n=4, p=2, n_voids=3, rmin=0.06, rmax=0.12),
    lambda: fcgen.custom(3, 4, 2, "elasticity", 1e-8, shapes=[], clamp_zmin=True),
])
def test_shared_rows_reproduce_every_row(desc):
    """Rows kept once by the library: every block row read through its
    offset gives back its own values bit for bit, and the number of kept
    rows equals the number of distinct value sequences (grouped here by
    their bytes, independently of the library's hashing)."""
    h = fc.HostSystem(desc())
    e = h.export()
    sh = h.share()
    rp, bd = e["rowptr"], e["bsr_dim"]
    val = e["val"].reshape(-1, bd * bd)
    distinct = set()
    for r in range(rp.size - 1):
        L = rp[r + 1] - rp[r]
        mine = val[rp[r]:rp[r + 1]]                           # [L, bd*bd], block-major
        got = sh["vals"][sh["ofs"][r]: sh["ofs"][r] + L * bd * bd].reshape(bd * bd, L).T
        assert got.tobytes() == mine.tobytes(), r
        distinct.add(mine.T.tobytes())
    assert sh["distinct_rows"] == len(distinct)
    assert sh["vals"].size == sum(len(b) // 8 for b in distinct)


def _box_shape(row, dim, n1, p):
    """Extent of a row node's columns per direction: a vertex function
    (index a multiple of p) meets the cells on both sides of its vertex, an
    interior function only its own cell."""
    shape = []
    for _ in range(dim):
        g = row % n1
        row //= n1
        shape.append(min(n1 - 1, g + p) - max(0, g - p) + 1 if g % p == 0 else p + 1)
    return tuple(shape)


@pytest.mark.parametrize("desc", [
    lambda: fcgen.disk_poisson_2d(0),
    lambda: fcgen.porous_elasticity_3d(seed=3, n=4, p=2, n_voids=3, rmin=0.06, rmax=0.12),
    lambda: fcgen.custom(3, 4, 3, "elasticity", 1e-8, shapes=[], clamp_zmin=True),
])
def test_row_groups_cover_every_row_once(desc):
    """The grouped products write exactly the rows their groups name: every
    block row must appear in exactly one group, and the rows of a group must
    have bitwise-equal values and one lattice box shape."""
    d = desc()
    h = fc.HostSystem(d)
    e = h.export()
    groups = h.row_groups()
    rp, bd = e["rowptr"], e["bsr_dim"]
    nr = rp.size - 1
    assert groups.shape[0] > 0 and groups.shape[1] == 4
    rows = groups[groups >= 0]
    np.testing.assert_array_equal(np.sort(rows), np.arange(nr))
    # -1 only pads the tail of a group
    for g in groups:
        k = int(np.sum(g >= 0))
        assert k >= 1 and np.all(g[:k] >= 0) and np.all(g[k:] == -1)
    assert np.any(np.sum(groups >= 0, axis=1) > 1)
    val = e["val"].reshape(-1, bd * bd)
    n1 = d["p"] * d["n"] + 1
    for g in groups:
        g = g[g >= 0]
        ref = val[rp[g[0]]:rp[g[0] + 1]].tobytes()
        shape = _box_shape(int(g[0]), d["dim"], n1, d["p"])
        for r in g[1:]:
            assert val[rp[r]:rp[r + 1]].tobytes() == ref
            assert _box_shape(int(r), d["dim"], n1, d["p"]) == shape
