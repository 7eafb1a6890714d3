"""Integrated Legendre shape functions and Gauss-Legendre quadrature.

The paper names the integrated Legendre basis in the remark of Sec. 3.2 and
counts (p+1)^d functions per element for the full tensor-product space
(footnote in Sec. 3.2).  The normalisation used is the Szabo-Babuska one:

    N_0 = (1 - xi)/2,  N_1 = (1 + xi)/2,
    N_j = (P_j - P_{j-2}) / sqrt(2 (2j - 1)),   j = 2..p,

on the reference interval [-1, 1].
"""
from __future__ import annotations

import math
import numpy as np
from numpy.polynomial import legendre as L


def legendre_value(j: int, xi):
    c = np.zeros(j + 1)
    c[j] = 1.0
    return L.legval(xi, c)


def shape_1d(p: int, xi):
    """Values and xi-derivatives of the p+1 shape functions at points xi.

    Returns (N, dN) with shape (len(xi), p+1); column a is local function a
    (0 = left vertex, 1 = right vertex, j >= 2 = bubble j).
    """
    xi = np.asarray(xi, dtype=np.float64)
    N = np.zeros(xi.shape + (p + 1,))
    dN = np.zeros(xi.shape + (p + 1,))
    N[..., 0] = 0.5 * (1.0 - xi)
    N[..., 1] = 0.5 * (1.0 + xi)
    dN[..., 0] = -0.5
    dN[..., 1] = 0.5
    for j in range(2, p + 1):
        s = math.sqrt(2.0 * (2 * j - 1))
        N[..., j] = (legendre_value(j, xi) - legendre_value(j - 2, xi)) / s
        # d/dxi (P_j - P_{j-2}) = (2j-1) P_{j-1}
        dN[..., j] = (2 * j - 1) * legendre_value(j - 1, xi) / s
    return N, dN


def gauss(npts: int):
    """Gauss-Legendre points and weights on [-1, 1]."""
    return L.leggauss(npts)


def tensor_rule(npts: int, lo, hi):
    """Tensor Gauss rule on the box [lo, hi]: points (n, d) and weights."""
    g, w = gauss(npts)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = lo.size
    axes_x = [lo[k] + 0.5 * (g + 1.0) * (hi[k] - lo[k]) for k in range(d)]
    axes_w = [0.5 * (hi[k] - lo[k]) * w for k in range(d)]
    # point index = i_0 + npts*(i_1 + npts*i_2): first coordinate fastest
    grids = np.meshgrid(*axes_x, indexing="ij")
    wgrid = np.ones([npts] * d)
    for k in range(d):
        shape = [1] * d
        shape[k] = npts
        wgrid = wgrid * axes_w[k].reshape(shape)
    pts = np.stack([gk.transpose(list(range(d))[::-1]).ravel() for gk in grids],
                   axis=1)
    wts = wgrid.transpose(list(range(d))[::-1]).ravel()
    return pts, wts
