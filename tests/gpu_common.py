"""Helpers shared by the GPU parity tests: seeded problems, the oracle's
reference objects, and conversions between the library's BSR export and
scipy matrices."""
import functools

import numpy as np
import pytest
import scipy.sparse as sp

import fcgen
from oracle import assemble, pcg, schwarz


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


PROBLEMS = {
    # 2-D Poisson on a disk, 16^2 cells, p = 2, alpha = 1e-10 (m = 9)
    "disk16_p2": lambda: fcgen.disk_poisson_2d(0),
    # same family with a ragged grid and p = 4 (m = 25)
    "disk7_p4": lambda: fcgen.disk_poisson_2d(5, n=7, p=4),
    # 3-D Poisson on a porous cube, p = 2 (m = 27)
    "pois3d_p2": lambda: fcgen.porous_poisson_3d(seed=1, n=5, p=2, n_voids=4,
                                                 rmin=0.06, rmax=0.14),
    # 3-D Poisson, p = 3 (m = 64, largest LDS eigen path)
    "pois3d_p3": lambda: fcgen.porous_poisson_3d(seed=2, n=4, p=3, n_voids=3,
                                                 rmin=0.08, rmax=0.15),
    # 3-D elasticity, p = 2 (m = 81, certified direct inverse)
    "elast3d_p2": lambda: fcgen.porous_elasticity_3d(seed=3, n=4, p=2, n_voids=3,
                                                     rmin=0.06, rmax=0.12),
    # 3-D elasticity, p = 3 (m = 192, the benchmark's block size)
    "elast3d_p3": lambda: fcgen.porous_elasticity_3d(seed=4, n=3, p=3, n_voids=3,
                                                     rmin=0.06, rmax=0.12),
}


@functools.lru_cache(maxsize=None)
def oracle_system(name):
    d = PROBLEMS[name]()
    s = assemble.assemble(d)
    return d, s


@functools.lru_cache(maxsize=None)
def oracle_precond(name, eta_bar=1.0, stabilize=True):
    _, s = oracle_system(name)
    blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], eta_bar)
    S, fall = schwarz.compute_preconditioner(s["A"], blocks, stabilize=stabilize)
    return S, fall, blocks


@functools.lru_cache(maxsize=None)
def oracle_direct(name):
    d, s = oracle_system(name)
    return pcg.direct_solve(s["A"], s["b"])


def energy(A, v):
    return float(np.sqrt(max(float(v @ (A @ v)), 0.0)))


def csr_to_bsr_arrays(A, bd):
    """Exact block-row layout of a scipy matrix on the lattice: every block
    (i, j) with any stored entry becomes one dense bd x bd block."""
    A = A.tocsr()
    n = A.shape[0]
    nb = n // bd
    coo = A.tocoo()
    keys = np.unique((coo.row // bd).astype(np.int64) * nb + coo.col // bd)
    brow = (keys // nb).astype(np.int32)
    bcol = (keys % nb).astype(np.int32)
    rowptr = np.zeros(nb + 1, np.int32)
    np.add.at(rowptr, brow + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    pos = {int(k): i for i, k in enumerate(keys)}
    val = np.zeros((len(keys), bd, bd))
    for r, c, v in zip(coo.row, coo.col, coo.data):
        val[pos[int((r // bd) * nb + c // bd)], r % bd, c % bd] += v
    return rowptr, bcol, val


@functools.lru_cache(maxsize=None)
def max_block_kappa(name, eta_bar=1.0):
    """Largest condition number (over kept eigenvalues) of the element
    blocks.  Above ~1e10 the smallest kept eigenpairs, and so the local
    pseudo-inverses, are fixed by FP64 data only to ~eps * kappa: two
    backward-stable eigensolvers (or two assemblers that differ by rounding)
    then give preconditioners whose PCG iteration counts differ by more
    than rounding."""
    _, s = oracle_system(name)
    _, _, blocks = oracle_precond(name, eta_bar)
    worst = 1.0
    for B in blocks:
        lam = np.linalg.eigvalsh(schwarz.extract_submatrix(s["A"], B))
        if lam.max() <= 0:
            continue
        kept = lam[lam > 1e-13 * lam.max()]
        worst = max(worst, kept.max() / kept.min())
    return worst


WELL_DETERMINED_KAPPA = 1e10
