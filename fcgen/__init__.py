"""Seeded synthetic finite cell problem descriptions.

This module only draws random numbers and packs them into a plain problem
description (a dict of Python scalars and lists).  It contains none of the
method's arithmetic: no basis functions, quadrature, assembly or solver
steps.  Both the CPU oracle and the GPU library consume the same
description, so the two sides always see identical geometry and loads.

Description keys
----------------
dim          2 or 3
n            cells per direction of the embedding grid over [0,1]^dim
p            polynomial order of the integrated Legendre basis
pde          "poisson"  (scalar reaction-diffusion  -lap u + u = f)
             "elasticity" (linear elasticity, E and nu)
alpha        fictitious-domain indicator value outside the physical domain
quad_depth   octree/quadtree depth used for cut cells
domain       "voids"      physical = box minus the union of the shapes
             "inclusions" physical = union of the shapes
shapes       list of {"centre": [..], "semi": [..]} axis-aligned ellipsoids
             (a sphere has equal semi-axes)
modes        scalar load f(x) = sum_k amp_k cos(2 pi k.x + phase_k)
E, nu        elasticity constants
traction     traction vector applied on the face z = 1 (3-D elasticity)
clamp_zmin   clamp every function that is nonzero on z = 0
discard_fictitious
             (optional, default False) remove every function whose support
             lies only in cells without physical material
"""
from __future__ import annotations

import math
import numpy as np

__all__ = [
    "disk_poisson_2d", "porous_elasticity_3d", "porous_poisson_3d",
    "batch_poisson", "custom", "n_dofs", "unet_init",
]


def n_dofs(desc: dict) -> int:
    """Number of unknowns of the full tensor-product lattice."""
    ncomp = desc["dim"] if desc["pde"] == "elasticity" else 1
    return ncomp * (desc["p"] * desc["n"] + 1) ** desc["dim"]


def _fourier_modes(rng: np.random.Generator, dim: int, count: int = 8):
    modes = []
    for _ in range(count):
        k = rng.integers(1, 5, size=dim).tolist()
        amp = float(rng.standard_normal())
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        modes.append({"k": [int(v) for v in k], "amp": amp, "phase": phase})
    return modes


def custom(dim, n, p, pde="poisson", alpha=1e-10, shapes=(), domain="voids",
           modes=None, quad_depth=3, E=1.0, nu=0.3, traction=None,
           clamp_zmin=False, seed=0, discard_fictitious=False) -> dict:
    """A description with explicitly given geometry (used by tests)."""
    if modes is None:
        modes = _fourier_modes(np.random.default_rng(seed), dim)
    if traction is None:
        traction = [0.0] * dim
        if pde == "elasticity" and dim == 3:
            traction = [0.0, 0.0, -1.0]
    return {
        "dim": int(dim), "n": int(n), "p": int(p), "pde": pde,
        "alpha": float(alpha), "quad_depth": int(quad_depth),
        "domain": domain,
        "shapes": [{"centre": [float(c) for c in s["centre"]],
                    "semi": [float(a) for a in s["semi"]]} for s in shapes],
        "modes": modes, "E": float(E), "nu": float(nu),
        "traction": [float(t) for t in traction],
        "clamp_zmin": bool(clamp_zmin), "seed": int(seed),
        "discard_fictitious": bool(discard_fictitious),
    }


def disk_poisson_2d(seed: int = 0, n: int = 16, p: int = 2,
                    radius: float = 0.37, alpha: float = 1e-10) -> dict:
    """2-D Poisson on a disk immersed in [0,1]^2.

    The centre is (0.5, 0.5) plus a point drawn uniformly from the disk of
    radius 0.05; f is a sum of 8 Fourier modes with unit-normal amplitudes.
    """
    rng = np.random.default_rng(seed)
    rho = 0.05 * math.sqrt(rng.uniform())
    th = rng.uniform(0.0, 2.0 * math.pi)
    centre = [0.5 + rho * math.cos(th), 0.5 + rho * math.sin(th)]
    modes = _fourier_modes(rng, 2)
    return custom(2, n, p, "poisson", alpha,
                  shapes=[{"centre": centre, "semi": [radius, radius]}],
                  domain="inclusions", modes=modes, seed=seed)


def _spherical_voids(rng, count, rmin, rmax):
    voids = []
    while len(voids) < count:
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r, 1.0 - r, size=3)
        ok = True
        for v in voids:
            d = math.dist(c, v["centre"])
            if d <= r + v["semi"][0]:
                ok = False
                break
        if ok:
            voids.append({"centre": c.tolist(), "semi": [r, r, r]})
    return voids


def porous_elasticity_3d(seed: int = 0, n: int = 32, p: int = 3,
                         n_voids: int = 64, rmin: float = 0.02,
                         rmax: float = 0.06, alpha: float = 1e-8,
                         discard_fictitious: bool = False) -> dict:
    """3-D linear elasticity on the unit cube minus seeded spherical voids.

    Radii are uniform in [rmin, rmax]; centres are uniform in [r, 1-r]^3 so
    no void touches a face; a draw that overlaps an earlier void is redrawn.
    The face z = 0 is clamped and z = 1 carries the traction (0, 0, -1).
    """
    rng = np.random.default_rng(seed)
    voids = _spherical_voids(rng, n_voids, rmin, rmax)
    return custom(3, n, p, "elasticity", alpha, shapes=voids, domain="voids",
                  modes=[], E=1.0, nu=0.3, traction=[0.0, 0.0, -1.0],
                  clamp_zmin=True, seed=seed, discard_fictitious=discard_fictitious)


def porous_poisson_3d(seed: int = 0, n: int = 64, p: int = 2,
                      n_voids: int = 64, rmin: float = 0.02,
                      rmax: float = 0.06, alpha: float = 1e-10) -> dict:
    """Scalar -lap u + u = f on the porous cube of porous_elasticity_3d."""
    rng = np.random.default_rng(seed)
    voids = _spherical_voids(rng, n_voids, rmin, rmax)
    modes = _fourier_modes(rng, 3)
    return custom(3, n, p, "poisson", alpha, shapes=voids, domain="voids",
                  modes=modes, seed=seed)


def batch_poisson(seed: int = 0, count: int = 512, min_dofs: int = 50_000,
                  max_dofs: int = 200_000) -> list:
    """Uneven batch of 2-D/3-D Poisson problems with elliptical inclusions
    or voids.  Grid sizes are uniform in 8..128 (2-D) or 8..24 (3-D), p in
    1..4; a draw is repeated until its DOF count lies in the given range
    (pass min_dofs=0, max_dofs=None for the unconditioned generator)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        dim = 2 if rng.uniform() < 0.5 else 3
        n = int(rng.integers(8, 129)) if dim == 2 else int(rng.integers(8, 25))
        p = int(rng.integers(1, 5))
        nd = (p * n + 1) ** dim
        if nd < min_dofs or (max_dofs is not None and nd > max_dofs):
            continue
        k = int(rng.integers(1, 7))
        shapes = []
        tries = 0
        while len(shapes) < k and tries < 1000:
            tries += 1
            semi = rng.uniform(0.05, 0.25, size=dim)
            c = rng.uniform(0.2, 0.8, size=dim)
            rb = float(semi.max())
            if all(math.dist(c, s["centre"]) > rb + max(s["semi"])
                   for s in shapes):
                shapes.append({"centre": c.tolist(), "semi": semi.tolist()})
        domain = "inclusions" if rng.uniform() < 0.5 else "voids"
        modes = _fourier_modes(rng, dim)
        out.append(custom(dim, n, p, "poisson", 1e-10, shapes=shapes,
                          domain=domain, modes=modes,
                          seed=seed * 100003 + len(out)))
    return out


def unet_init(ch=(8, 16, 32, 32), in_ch=2, seed=0):
    """Seeded He-normal initial parameters of the coarse-correction U-Net
    (flat vector: per convolution W[co][ci][27] then b[co], layer order
    enc0a enc0b enc1a enc1b enc2a enc2b bota botb up2a up2b up1a up1b up0a
    up0b head), float32; biases start at zero."""
    c0, c1, c2, c3 = ch
    io = [(in_ch, c0), (c0, c0), (c0, c1), (c1, c1), (c1, c2), (c2, c2), (c2, c3), (c3, c3),
          (c3, c2), (c2, c2), (c2, c1), (c1, c1), (c1, c0), (c0, c0), (c0, 1)]
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in io:
        parts.append(rng.standard_normal(co * ci * 27) * math.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
