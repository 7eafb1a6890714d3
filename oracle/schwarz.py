"""Additive Schwarz preconditioner of the paper (Sec. 3, Eq. 6; Algorithm 1).

    S = sum_B R_B^T (R_B A R_B^T)^+ R_B

Blocks are element-wise: one block per cell holding every function
supported on it (Sec. 3.1), selected when the cell's volume fraction eta_T
does not exceed the threshold eta_bar (Sec. 3.2, "Optimizing the number of
blocks").  Each local inverse is the stabilised pseudo-inverse of Eqs.
(9)-(11): eigen-decompose the symmetric block, keep the eigenpairs whose
eigenvalue exceeds eps * max(eigenvalue), and sum 1/lambda v v^T over them.
After all blocks are summed, every diagonal entry of S that is still zero
gets 1/A_ll (diagonal scaling of Algorithm 1).

The global S is assembled as a sparse matrix, exactly as the algorithm
prolongates each local inverse into S.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def select_blocks(elem_dofs, eta, eta_bar=1.0):
    """Element blocks of the cells whose eta_T <= eta_bar."""
    return [elem_dofs[i] for i in range(len(eta)) if eta[i] <= eta_bar]


def vertex_patch_blocks(desc, elem_dofs, eta, eta_bar=1.0):
    """Vertex-patch blocks: one per vertex of the cell grid (vertices in
    order of the first direction fastest), the union of the element blocks
    of the (up to 2^dim) cells that share the vertex, i.e. every function
    supported on those cells, in ascending unknown order.  A patch is kept
    when one of its cells has eta_T <= eta_bar.  Every element block lies
    inside the patch of each of its vertices, so the functions a cut cell
    makes nearly dependent stay together, as Sec. 3.1 asks of a block."""
    n, d = desc["n"], desc["dim"]
    blocks = []
    for vid in range((n + 1) ** d):
        vc = [(vid // (n + 1) ** k) % (n + 1) for k in range(d)]
        ranges = [range(max(0, c - 1), min(n - 1, c) + 1) for c in vc]
        cells = [sum(cc[k] * n ** k for k in range(d)) for cc in itertools.product(*ranges)]
        if min(eta[c] for c in cells) > eta_bar:
            continue
        blocks.append(np.unique(np.concatenate([elem_dofs[c] for c in cells])))
    return blocks


def extract_submatrix(A, B):
    """A_B = R_B A R_B^T: the assembled entries of A on the index set B."""
    return A[B][:, B].toarray()


def pseudo_inverse(AB, eps=1e-13, stabilize=True):
    """Stabilised local inverse of Eqs. (9)-(11).

    With stabilize=False the plain inverse sum over all eigenpairs is
    returned (the unstabilised S* of Sec. 5.2).  When no eigenvalue is
    positive the block contributes nothing.
    """
    lam, V = np.linalg.eigh(AB)
    if not stabilize:
        return (V / lam) @ V.T
    lmax = lam.max()
    if lmax <= 0.0:
        return np.zeros_like(AB)
    keep = lam > eps * lmax
    Vk = V[:, keep]
    return (Vk / lam[keep]) @ Vk.T


def compute_preconditioner(A, blocks, eps=1e-13, stabilize=True):
    """Algorithm 1: sum the prolongated local (pseudo-)inverses, then give
    every function with a zero diagonal entry of S the diagonal scaling
    1/A_ll (only where A_ll > 0, so that a function with no stiffness at
    all is left out instead of receiving an infinite entry)."""
    n = A.shape[0]
    rows, cols, vals = [], [], []
    for B in blocks:
        P = pseudo_inverse(extract_submatrix(A, B), eps, stabilize)
        rows.append(np.repeat(B, B.size))
        cols.append(np.tile(B, B.size))
        vals.append(P.ravel())
    if rows:
        S = sp.coo_matrix((np.concatenate(vals),
                           (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n)).tocsr()
        S.sum_duplicates()
    else:
        S = sp.csr_matrix((n, n))
    sdiag = S.diagonal()
    adiag = A.diagonal()
    fall = np.nonzero((sdiag == 0.0) & (adiag > 0.0))[0]
    if fall.size:
        S = S + sp.csr_matrix((1.0 / adiag[fall], (fall, fall)), shape=(n, n))
    return S.tocsr(), fall


def block_overlap(blocks, n):
    """Number of blocks each unknown belongs to."""
    count = np.zeros(n, dtype=np.int64)
    for B in blocks:
        count[B] += 1
    return count
