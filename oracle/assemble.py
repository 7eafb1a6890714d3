"""Finite cell discretisation and assembly of A x = b (Sec. 2.1, Eq. 1; Eq. 2).

Weak forms, with the indicator alpha multiplying every volume term:

  scalar      a(u,v) = int alpha (grad u . grad v + u v),  l(v) = int alpha f v
  elasticity  a(u,v) = int alpha eps(v) : C : eps(u),       l(v) = int_{top} t . v

The elasticity tensor is written in Voigt notation (engineering shear) and
the element stiffness is the textbook sum over quadrature points of
B^T D B.  The face x_{d-1} = 1 carries the traction; when the description
asks for it, every function that is nonzero on x_{d-1} = 0 is clamped
strongly: its rows and columns are zeroed, the diagonal entry is kept and
its load entry is set to zero.  With discard_fictitious, every function
whose support lies only in cells without physical material (eta_T = 0) is
removed the same way: the preprocessing the paper applies to elements
completely outside the physical domain (Sec. 5.2), done in place so that
the numbering stays the lattice's.

Numbering.  Per direction the global 1-D index of local function a on cell
e is g = p*e + L(a) with L(0) = 0, L(1) = p, L(j) = j - 1; the node id is
g_0 + (pn+1)(g_1 + (pn+1) g_2), the unknown is ncomp*node + component, and
element-local functions are ordered a_0 + (p+1)(a_1 + (p+1) a_2).
"""
from __future__ import annotations

import itertools
import numpy as np
import scipy.sparse as sp

from . import basis, geometry


def ncomp_of(desc):
    return desc["dim"] if desc["pde"] == "elasticity" else 1


def n_nodes_1d(desc):
    return desc["p"] * desc["n"] + 1


def n_dofs(desc):
    return ncomp_of(desc) * n_nodes_1d(desc) ** desc["dim"]


def cells(desc):
    """All cells, first coordinate fastest."""
    n, d = desc["n"], desc["dim"]
    for idx in itertools.product(range(n), repeat=d):
        yield tuple(reversed(idx))


def cell_index(desc, cell):
    n = desc["n"]
    return sum(c * n ** k for k, c in enumerate(cell))


def local_to_global_1d(p, e, a):
    if a == 0:
        return p * e
    if a == 1:
        return p * e + p
    return p * e + a - 1


def element_dofs(desc, cell):
    """Global unknowns of the cell in element-local order."""
    p, d = desc["p"], desc["dim"]
    nc = ncomp_of(desc)
    n1 = n_nodes_1d(desc)
    dofs = []
    for loc in itertools.product(range(p + 1), repeat=d):
        a = tuple(reversed(loc))        # a_0 fastest
        node = 0
        stride = 1
        for k in range(d):
            node += local_to_global_1d(p, cell[k], a[k]) * stride
            stride *= n1
        for c in range(nc):
            dofs.append(nc * node + c)
    return np.array(dofs, dtype=np.int64)


def cell_quadrature(desc, cell):
    """Quadrature points, weights and alpha values of one cell, and eta_T.

    Every leaf of the integration tree gets a (p+1)^d Gauss rule and alpha is
    evaluated at each point.  eta_T (Eq. 8) is the physical fraction of the
    cell measured with the same points.
    """
    d, p = desc["dim"], desc["p"]
    h = 1.0 / desc["n"]
    lo = np.array(cell, dtype=np.float64) * h
    hi = lo + h
    pts, wts = [], []
    for blo, bhi, _state in geometry.leaf_boxes(desc, lo, hi):
        x, w = basis.tensor_rule(p + 1, blo, bhi)
        pts.append(x)
        wts.append(w)
    pts = np.concatenate(pts)
    wts = np.concatenate(wts)
    phys = geometry.is_physical(desc, pts)
    alpha = np.where(phys, 1.0, desc["alpha"])
    # fraction of the cell's quadrature weight at physical points; the ratio
    # is exactly 1.0 when every point is physical
    eta = float(np.sum(wts[phys]) / np.sum(wts))
    return pts, wts, alpha, eta


def element_basis(desc, cell, pts):
    """Tensor-product shape values (nq, nn) and physical gradients
    (nq, d, nn) at the points, element-local function order."""
    d, p = desc["dim"], desc["p"]
    h = 1.0 / desc["n"]
    lo = np.array(cell, dtype=np.float64) * h
    xi = 2.0 * (pts - lo) / h - 1.0
    V, D = [], []
    for k in range(d):
        v, dv = basis.shape_1d(p, xi[:, k])
        V.append(v)
        D.append(dv * (2.0 / h))
    nq = pts.shape[0]
    nn = (p + 1) ** d
    N = np.ones((nq, nn))
    G = np.ones((nq, d, nn))
    for j, loc in enumerate(itertools.product(range(p + 1), repeat=d)):
        a = tuple(reversed(loc))
        col = j
        for k in range(d):
            N[:, col] *= V[k][:, a[k]]
            for g in range(d):
                G[:, g, col] *= (D[k][:, a[k]] if g == k else V[k][:, a[k]])
    return N, G


def lame(desc):
    E, nu = desc["E"], desc["nu"]
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def voigt_D(desc):
    """Isotropic elasticity matrix, Voigt order (xx, yy[, zz], then shears)."""
    lam, mu = lame(desc)
    d = desc["dim"]
    if d == 2:   # plane strain: (xx, yy, xy)
        D = np.array([[lam + 2 * mu, lam, 0.0],
                      [lam, lam + 2 * mu, 0.0],
                      [0.0, 0.0, mu]])
    else:        # (xx, yy, zz, yz, xz, xy)
        D = np.zeros((6, 6))
        D[:3, :3] = lam
        D[np.arange(3), np.arange(3)] = lam + 2 * mu
        D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def strain_B(G, d):
    """Strain-displacement matrices (nq, nstrain, d*nn) from gradients."""
    nq, _, nn = G.shape
    if d == 2:
        B = np.zeros((nq, 3, 2 * nn))
        B[:, 0, 0::2] = G[:, 0]
        B[:, 1, 1::2] = G[:, 1]
        B[:, 2, 0::2] = G[:, 1]
        B[:, 2, 1::2] = G[:, 0]
    else:
        B = np.zeros((nq, 6, 3 * nn))
        B[:, 0, 0::3] = G[:, 0]
        B[:, 1, 1::3] = G[:, 1]
        B[:, 2, 2::3] = G[:, 2]
        B[:, 3, 1::3] = G[:, 2]      # gamma_yz = du_y/dz + du_z/dy
        B[:, 3, 2::3] = G[:, 1]
        B[:, 4, 0::3] = G[:, 2]      # gamma_xz
        B[:, 4, 2::3] = G[:, 0]
        B[:, 5, 0::3] = G[:, 1]      # gamma_xy
        B[:, 5, 1::3] = G[:, 0]
    return B


def load_f(desc, x):
    """Scalar load f(x) = sum_k amp_k cos(2 pi k.x + phase_k)."""
    f = np.zeros(x.shape[0])
    for m in desc["modes"]:
        k = np.asarray(m["k"], dtype=np.float64)
        f += m["amp"] * np.cos(2.0 * np.pi * (x @ k) + m["phase"])
    return f


def element_system(desc, cell, chunk=4096):
    """Element stiffness Ke, element volume load fe and eta_T of one cell."""
    d = desc["dim"]
    pts, wts, alpha, eta = cell_quadrature(desc, cell)
    wa = wts * alpha
    nn = (desc["p"] + 1) ** d
    if desc["pde"] == "poisson":
        Ke = np.zeros((nn, nn))
        fe = np.zeros(nn)
        for s in range(0, pts.shape[0], chunk):
            sl = slice(s, s + chunk)
            N, G = element_basis(desc, cell, pts[sl])
            w = wa[sl]
            Ke += N.T @ (w[:, None] * N)
            for g in range(d):
                Ke += G[:, g].T @ (w[:, None] * G[:, g])
            fe += N.T @ (w * load_f(desc, pts[sl]))
        return Ke, fe, eta
    D = voigt_D(desc)
    m = d * nn
    Ke = np.zeros((m, m))
    for s in range(0, pts.shape[0], chunk):
        sl = slice(s, s + chunk)
        _, G = element_basis(desc, cell, pts[sl])
        B = strain_B(G, d)
        DB = np.einsum("ij,qjm->qim", D, B) * wa[sl][:, None, None]
        # sum_q B_q^T D B_q w_q alpha_q as one product over (q, strain)
        Ke += B.reshape(-1, m).T @ DB.reshape(-1, m)
    return Ke, np.zeros(m), eta


def traction_load(desc, cell):
    """Load of the traction t on the face x_{d-1} = 1 for a top cell."""
    d, p = desc["dim"], desc["p"]
    nc = ncomp_of(desc)
    nn = (p + 1) ** d
    fe = np.zeros(nc * nn)
    if desc["pde"] != "elasticity" or cell[d - 1] != desc["n"] - 1:
        return fe
    t = np.asarray(desc["traction"], dtype=np.float64)
    if not np.any(t):
        return fe
    h = 1.0 / desc["n"]
    lo = np.array(cell, dtype=np.float64) * h
    flo = lo[: d - 1]
    fx, fw = basis.tensor_rule(p + 1, flo, flo + h)
    pts = np.concatenate([fx, np.ones((fx.shape[0], 1))], axis=1)
    N, _ = element_basis(desc, cell, pts)
    for c in range(nc):
        fe[c::nc] += t[c] * (N.T @ fw)
    return fe


def clamped_dofs(desc):
    """Unknowns of every function that is nonzero on x_{d-1} = 0."""
    if not desc.get("clamp_zmin"):
        return np.zeros(0, dtype=np.int64)
    d = desc["dim"]
    n1 = n_nodes_1d(desc)
    nc = ncomp_of(desc)
    plane = n1 ** (d - 1)
    nodes = np.arange(plane)           # g_{d-1} = 0 is the first plane
    return (nc * nodes[:, None] + np.arange(nc)[None, :]).ravel()


def assemble(desc, keep_cells=None, keep_elements=False):
    """Assemble the global system.

    Returns a dict with A (scipy CSR), b, eta (per cell, cell index order),
    elem_dofs (n_cells, m) and the list of cells; with keep_elements also
    Ke, the element stiffness matrices (n_cells, m, m) in cell order.
    """
    ndof = n_dofs(desc)
    rows, cols, vals = [], [], []
    b = np.zeros(ndof)
    cl = list(cells(desc))
    eta = np.zeros(len(cl))
    edofs = []
    kes = []
    for ci, cell in enumerate(cl):
        Ke, fe, et = element_system(desc, cell)
        if keep_elements:
            kes.append(Ke)
        fe = fe + traction_load(desc, cell)
        dofs = element_dofs(desc, cell)
        edofs.append(dofs)
        eta[ci] = et
        rows.append(np.repeat(dofs, dofs.size))
        cols.append(np.tile(dofs, dofs.size))
        vals.append(Ke.ravel())
        np.add.at(b, dofs, fe)
    A = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ndof, ndof)).tocsr()
    A.sum_duplicates()
    A, b = apply_clamp(desc, A, b)
    if desc.get("discard_fictitious"):
        A, b = remove_dofs(A, b, fictitious_dofs(np.array(edofs), eta, ndof))
    out = {"A": A, "b": b, "eta": eta, "elem_dofs": np.array(edofs), "cells": cl}
    if keep_elements:
        out["Ke"] = np.array(kes)
    return out


def fictitious_dofs(elem_dofs, eta, ndof):
    """Unknowns of the functions that touch no cell with eta_T > 0."""
    touch = np.zeros(ndof, dtype=bool)
    for c in np.flatnonzero(eta > 0.0):
        touch[elem_dofs[c]] = True
    return np.flatnonzero(~touch)


def apply_clamp(desc, A, b):
    return remove_dofs(A, b, clamped_dofs(desc))


def remove_dofs(A, b, cd):
    """Zero the rows and columns of the unknowns cd, keep their diagonal
    entries and set their load entries to zero."""
    if cd.size == 0:
        return A, b
    diag = A.diagonal()[cd].copy()
    keep = np.ones(A.shape[0])
    keep[cd] = 0.0
    K = sp.diags(keep)
    A = (K @ A @ K).tocsr()
    A = A + sp.csr_matrix((diag, (cd, cd)), shape=A.shape)
    A.sum_duplicates()
    A.eliminate_zeros()
    b = b.copy()
    b[cd] = 0.0
    return A.tocsr(), b
