"""Element-by-element forms of the operator and of the preconditioner.

    A = sum_e R_e^T K_e R_e              (the assembly of the element
                                          stiffness matrices, Sec. 3.1)
    S = sum_B R_B^T P_B R_B + D_fall     (Eq. 6, with the diagonal scaling
                                          that Algorithm 1 gives functions
                                          no block reaches)

applied without forming a global matrix: gather the unknowns of each
element (block), multiply by its matrix, add the products back at the same
unknowns.  In this form the 32^3-cell benchmark problem fits a CPU's
memory with both A and S (two stacks of 32,768 dense 192 x 192 matrices,
about 19 GB) and a PCG iteration can be timed at full size.

Clamped unknowns are treated as ``assemble.remove_dofs`` treats them: their
rows and columns are zero except the diagonal, which keeps the operator's
own diagonal entry.
"""
from __future__ import annotations

import numpy as np


class ElementOperator:
    """y = sum_e R_e^T M_e R_e x (+ the clamped and extra diagonals).

    dofs: (E, m) global unknowns of each element, in the element's local
    order; mats: (E, m, m) element matrices; n: number of unknowns;
    clamped: unknowns whose rows and columns are removed (diagonal kept);
    diag_extra: optional length-n diagonal added to the product."""

    def __init__(self, dofs, mats, n, clamped=None, diag_extra=None):
        self.dofs = np.asarray(dofs, dtype=np.int64)
        self.mats = mats
        self.n = int(n)
        self.shape = (self.n, self.n)
        self.keep = None
        self.cdiag = None
        if clamped is not None and len(clamped):
            keep = np.ones(self.n)
            keep[clamped] = 0.0
            self.keep = keep
            d = np.bincount(self.dofs.ravel(),
                            weights=np.einsum("emm->em", mats).ravel(), minlength=self.n)
            self.cdiag = np.zeros(self.n)
            self.cdiag[clamped] = d[clamped]
        self.extra = None if diag_extra is None else np.asarray(diag_extra, dtype=np.float64)

    def __matmul__(self, x):
        v = x if self.keep is None else self.keep * x
        xe = v[self.dofs]
        ye = np.matmul(self.mats, xe[..., None])[..., 0]
        y = np.bincount(self.dofs.ravel(), weights=ye.ravel(), minlength=self.n)
        if self.keep is not None:
            y = self.keep * y + self.cdiag * x
        if self.extra is not None:
            y = y + self.extra * x
        return y

    def diagonal(self):
        d = np.bincount(self.dofs.ravel(), weights=np.einsum("emm->em", self.mats).ravel(),
                        minlength=self.n)
        if self.keep is not None:
            d = self.keep * d + self.cdiag
        if self.extra is not None:
            d = d + self.extra
        return d
