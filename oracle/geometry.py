"""Physical-domain indicator, exact box classification and octree leaves.

The finite cell method embeds the physical domain in a box and separates
physical from fictitious points by the indicator alpha: 1 inside the
physical domain, a small constant outside (Sec. 2.1, Eq. 1).  Cut cells are
integrated on an octree (quadtree in 2-D) of depth 3 relative to the cell
size, with Gauss points on the leaves (Sec. 5.1, problem setup).

Shapes are axis-aligned ellipsoids; a point x lies inside a shape when
sum(((x - c)/s)^2) <= 1.  For domain "voids" the physical domain is the box
minus the union of shapes, for "inclusions" it is the union of shapes.
"""
from __future__ import annotations

import numpy as np

PHYS, FICT, CUT = 0, 1, 2


def inside_any_shape(desc, x):
    """Boolean array: point inside at least one shape.  x has shape (n, d)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    hit = np.zeros(x.shape[0], dtype=bool)
    for s in desc["shapes"]:
        c = np.asarray(s["centre"])
        a = np.asarray(s["semi"])
        u = (x - c) / a
        hit |= np.sum(u * u, axis=1) <= 1.0
    return hit


def is_physical(desc, x):
    inside = inside_any_shape(desc, x)
    return ~inside if desc["domain"] == "voids" else inside


def alpha_at(desc, x):
    """Indicator alpha at points x (Eq. 1)."""
    return np.where(is_physical(desc, x), 1.0, desc["alpha"])


def _box_vs_shape(shape, lo, hi):
    """(entirely_inside, entirely_outside) of the box [lo, hi] w.r.t. one
    ellipsoid, decided exactly in coordinates scaled by the semi-axes."""
    c = np.asarray(shape["centre"])
    a = np.asarray(shape["semi"])
    ulo = (np.asarray(lo) - c) / a
    uhi = (np.asarray(hi) - c) / a
    nearest = np.clip(0.0, ulo, uhi)
    dmin2 = float(np.sum(nearest * nearest))
    dmax2 = float(np.sum(np.maximum(ulo * ulo, uhi * uhi)))
    return dmax2 <= 1.0, dmin2 > 1.0


def classify_box(desc, lo, hi):
    """PHYS, FICT or CUT for the box [lo, hi]."""
    in_some = False
    out_all = True
    for s in desc["shapes"]:
        inside, outside = _box_vs_shape(s, lo, hi)
        in_some |= inside
        out_all &= outside
    if desc["domain"] == "voids":
        if in_some:
            return FICT
        return PHYS if out_all else CUT
    if in_some:
        return PHYS
    return FICT if out_all else CUT


def leaf_boxes(desc, lo, hi, depth=None):
    """Leaves of the integration tree of the box [lo, hi].

    A cut box is bisected in every direction until the leaf edge is 2^-depth
    of the cell edge; uncut boxes stop at once.
    """
    if depth is None:
        depth = desc["quad_depth"]
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    state = classify_box(desc, lo, hi)
    if state != CUT or depth == 0:
        return [(lo, hi, state)]
    d = lo.size
    mid = 0.5 * (lo + hi)
    out = []
    for corner in range(2 ** d):
        clo = lo.copy()
        chi = hi.copy()
        for k in range(d):
            if (corner >> k) & 1:
                clo[k] = mid[k]
            else:
                chi[k] = mid[k]
        out.extend(leaf_boxes(desc, clo, chi, depth - 1))
    return out
