"""Preconditioned conjugate gradients and the paper's convergence measures.

PCG follows the standard preconditioned CG recurrences (Saad, cited in the
paper's Sec. 1 and 5) with x_0 = 0:

    r_0 = b,  z_0 = S r_0,  p_0 = z_0
    alpha = (r, z) / (p, A p);  x += alpha p;  r -= alpha A p
    z = S r;  beta = (r_new, z_new) / (r, z);  p = z + beta p

Stopping (Eq. 12): the relative preconditioned residual ||S r_i|| / ||S b||
<= tol, with S r_i taken from the recurrence ("precond"); or the relative
residual ||r_i|| / ||b|| <= tol ("residual").  The iteration count is the
number of products with A.  The energy error is Eq. (13).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla

OK, NOTCONV, BREAKDOWN = 0, 4, 5


def pcg(A, b, S, tol=1e-10, maxit=300000, stop="precond", x_ref=None,
        keep_directions=False):
    """Returns (x, info).  info holds iters, status, the history of both
    relative residuals and, when x_ref is given, of the energy error."""
    n = b.size
    x = np.zeros(n)
    r = b.copy()
    z = S @ r
    p = z.copy()
    rz = float(r @ z)
    z0 = float(np.linalg.norm(z))
    b0 = float(np.linalg.norm(b))
    hist_prec = [1.0 if z0 > 0 else 0.0]
    hist_res = [1.0 if b0 > 0 else 0.0]
    hist_err = []
    dirs = [p.copy()] if keep_directions else None
    if x_ref is not None:
        hist_err.append(energy_error(A, x_ref, x))
    status = NOTCONV
    it = 0

    def converged():
        val = hist_prec[-1] if stop == "precond" else hist_res[-1]
        return val <= tol

    if z0 == 0.0 or b0 == 0.0:
        return x, {"iters": 0, "status": OK, "prec": hist_prec,
                   "res": hist_res, "err": hist_err, "dirs": dirs}
    while it < maxit:
        q = A @ p
        pq = float(p @ q)
        it += 1
        if not (pq > 0.0) or not (rz > 0.0):
            status = BREAKDOWN
            break
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        z = S @ r
        rz_new = float(r @ z)
        hist_prec.append(float(np.linalg.norm(z)) / z0)
        hist_res.append(float(np.linalg.norm(r)) / b0)
        if x_ref is not None:
            hist_err.append(energy_error(A, x_ref, x))
        if not np.isfinite(rz_new):
            status = BREAKDOWN
            break
        if converged():
            status = OK
            break
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
        if keep_directions:
            dirs.append(p.copy())
    return x, {"iters": it, "status": status, "prec": hist_prec,
               "res": hist_res, "err": hist_err, "dirs": dirs}


def energy_norm(A, v):
    return float(np.sqrt(max(float(v @ (A @ v)), 0.0)))


def energy_error(A, x_ref, x):
    """Relative error in the energy norm, Eq. (13)."""
    return energy_norm(A, x_ref - x) / energy_norm(A, x_ref)


def direct_solve(A, b):
    """Reference solution: dense Cholesky for small systems, sparse LU
    otherwise (a stand-in for the direct solver used in the paper)."""
    n = b.size
    if n <= 6000:
        c = scipy.linalg.cho_factor(A.toarray())
        return scipy.linalg.cho_solve(c, b)
    return spla.spsolve(A.tocsc(), b)
