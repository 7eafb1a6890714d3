"""Training the learned coarse correction from solver-generated pairs.

Every numerical step runs in libfc: the solves (fc_pcg_solve), the pairs
taken from a running solve (fc_learned_snapshots) and the training
(fc_model_train).  This module only picks the snapshot iterations and
stacks the pairs of several problems into one device tensor.
"""
from __future__ import annotations

import time

import numpy as np

from . import _lib as L


def snapshot_iterations(k_total: int, count: int) -> list:
    """`count` distinct iterations spread evenly over [0, k_total)."""
    if k_total <= 0:
        return [0]
    pts = np.unique(np.linspace(0, k_total - 1, num=min(count, k_total)).round().astype(int))
    return [int(v) for v in pts]


def problem_pairs(desc, count, kind="e-Sr", tol=1e-8, x_tol=1e-12, log=None):
    """Pairs from one problem: solve tightly for x*, count the iterations
    the plain solve needs to `tol`, and take `count` snapshots spread over
    them.  Returns (xin [k,2,G^3], t [k,G^3], G, iterations)."""
    import torch
    t0 = time.perf_counter()
    pb = L.Problem.setup(desc)
    pc = L.Precond(pb)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    xs = torch.zeros_like(b)
    L.pcg_solve(pb, pc, b, xs, tol=x_tol, stop="residual", raise_on_error=True)
    xt = torch.zeros_like(b)
    info = L.pcg_solve(pb, pc, b, xt, tol=tol, stop="residual", raise_on_error=True)
    its = snapshot_iterations(info["iters"], count)
    G = pc.coarse_grid()
    nv = G ** 3
    xin = torch.zeros((len(its), 2, nv), dtype=torch.float32, device="cuda")
    tt = torch.zeros((len(its), nv), dtype=torch.float32, device="cuda")
    k = pc.snapshots(b, xs, its, xin, tt, kind=kind, tol=0.0)
    if log:
        log(f"pairs: {k} from a {pb.n}-unknown problem ({info['iters']} iterations to {tol:g}, "
            f"{time.perf_counter() - t0:.1f} s)")
    return xin[:k], tt[:k], G, info["iters"]


def training_set(descs, per_problem, kind="e-Sr", log=None):
    """Stacked pairs of several problems of one grid size."""
    import torch
    xs, ts, g0 = [], [], None
    for d in descs:
        xin, t, G, _ = problem_pairs(d, per_problem, kind=kind, log=log)
        if g0 is not None and G != g0:
            raise L.FcError(L.FC_E_ARG, "training problems must share the coarse grid")
        g0 = G
        xs.append(xin)
        ts.append(t)
    return torch.cat(xs).contiguous(), torch.cat(ts).contiguous(), g0


def train(model: L.Model, xin, t, G, epochs=20, batch=8, lr=1e-3):
    """Adam on the pairs (fc_model_train); returns the per-epoch loss."""
    n = xin.shape[0]
    x5 = xin.reshape(n, 2, G, G, G)
    t5 = t.reshape(n, 1, G, G, G)
    return model.train(x5, t5, epochs=epochs, batch=batch, lr=lr)
