"""How well the FP64 data fix the paper's preconditioner.

The local pseudo-inverses of Eqs. (9)-(11) are only as well determined as
the smallest kept eigenvalue of each block allows: a backward-stable
eigensolver returns 1/lambda_min with relative error ~ eps*kappa(A_B).
This test computes the oracle's preconditioner a second way -- a cyclic
Jacobi eigen-decomposition written here, the algorithm the GPU uses --
and checks that on a well-determined problem the two PCG runs agree to
rounding while on a block-kappa ~1e11 problem (alpha = 1e-10, p = 4) the
iteration counts to 1e-10 already differ by several iterations.  The GPU
parity tests use this to separate well- from ill-determined cases.
"""
import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp

from oracle import pcg, schwarz
from tests.gpu_common import max_block_kappa, oracle_precond, oracle_system


def _jacobi_eig(A):
    A = A.copy()
    m = A.shape[0]
    V = np.eye(m)
    for _ in range(40):
        rotated = False
        for p in range(m - 1):
            for q in range(p + 1, m):
                apq, app, aqq = A[p, q], A[p, p], A[q, q]
                if apq != 0 and abs(apq) > 2.220446049250313e-16 * np.sqrt(abs(app * aqq)):
                    tau = (aqq - app) / (2 * apq)
                    t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + np.sqrt(1 + tau * tau))
                    c = 1 / np.sqrt(1 + t * t)
                    s = t * c
                    ap, aq = A[p, :].copy(), A[q, :].copy()
                    A[p, :], A[q, :] = c * ap - s * aq, s * ap + c * aq
                    ap, aq = A[:, p].copy(), A[:, q].copy()
                    A[:, p], A[:, q] = c * ap - s * aq, s * ap + c * aq
                    vp, vq = V[:, p].copy(), V[:, q].copy()
                    V[:, p], V[:, q] = c * vp - s * vq, s * vp + c * vq
                    rotated = True
        if not rotated:
            break
    return np.diag(A).copy(), V


def _jacobi_S(A, blocks):
    n = A.shape[0]
    rows, cols, vals = [], [], []
    for B in blocks:
        lam, V = _jacobi_eig(schwarz.extract_submatrix(A, B))
        keep = lam > 1e-13 * lam.max()
        P = (V[:, keep] / lam[keep]) @ V[:, keep].T
        rows.append(np.repeat(B, B.size))
        cols.append(np.tile(B, B.size))
        vals.append(P.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def test_iteration_spread_between_eigensolvers():
    out = {}
    for name in ("pois3d_p2", "disk7_p4"):
        _, s = oracle_system(name)
        A, b = s["A"], s["b"]
        S0, _, blocks = oracle_precond(name)
        S1 = _jacobi_S(A, blocks)
        _, i0 = pcg.pcg(A, b, S0, tol=1e-10)
        _, i1 = pcg.pcg(A, b, S1, tol=1e-10)
        out[name] = (max_block_kappa(name), i0["iters"], i1["iters"])
    k, a, b = out["pois3d_p2"]
    assert k < 1e10 and abs(a - b) <= 1, out
    k, a, b = out["disk7_p4"]
    assert k > 1e11 and abs(a - b) >= 3, out


def _lapack_S(A, blocks, driver):
    n = A.shape[0]
    rows, cols, vals = [], [], []
    for B in blocks:
        lam, V = sl.eigh(schwarz.extract_submatrix(A, B), driver=driver)
        keep = lam > 1e-13 * lam.max()
        P = (V[:, keep] / lam[keep]) @ V[:, keep].T
        rows.append(np.repeat(B, B.size))
        cols.append(np.tile(B, B.size))
        vals.append(P.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def test_iteration_spread_at_benchmark_block_kappa():
    """3-D p = 3 elasticity at alpha = 1e-8 with thin cuts (largest block
    kappa 6.9e9, inside the 1e8-1e10 of the benchmark's cut blocks): two
    LAPACK drivers for the same eigenproblems (divide and conquer, and QL
    iteration) give preconditioners whose PCG iteration counts to the
    Eq. 12 tolerance 1e-10 differ by several percent (724 and 687 here),
    while the solutions both reach at 1e-13 agree to 1e-12 in the energy
    norm: at this kappa the count is decided by rounding, the solution by
    the data."""
    from tests.gpu_common import energy
    name = "elast3d_p3_thin"
    _, s = oracle_system(name)
    A, b = s["A"], s["b"]
    S0, _, blocks = oracle_precond(name)
    S1 = _lapack_S(A, blocks, "ev")
    _, i0 = pcg.pcg(A, b, S0, tol=1e-10)
    _, i1 = pcg.pcg(A, b, S1, tol=1e-10)
    x0, _ = pcg.pcg(A, b, S0, tol=1e-13)
    x1, _ = pcg.pcg(A, b, S1, tol=1e-13)
    k = max_block_kappa(name)
    assert 1e8 < k <= 1e10
    assert abs(i0["iters"] - i1["iters"]) >= 0.03 * i0["iters"], (i0["iters"], i1["iters"])
    assert energy(A, x1 - x0) <= 1e-12 * energy(A, x0)
