"""FP64 oracle of the learned coarse correction (test infrastructure only).

The correction adds a learned coarse component to the Schwarz apply inside
flexible CG, the kind of coarse level the paper's outlook names (Sec. 6)
for extending the additive Schwarz method.  Everything here is the plain
definition, for checking the GPU kernels:

Transfer between unknowns and the coarse grid (scalar, even n):
  * vertex unknowns are the functions whose lattice indices are all
    multiples of p; they form the (n+1)^d vertex grid (Q1 hats);
  * the coarse grid is every other vertex, (n/2+1)^d points;
  * prolongation P_c is trilinear interpolation from coarse to vertex
    grid, injected into the vertex unknowns (all others zero);
  * restriction of a residual is P_c^T; of an error, sampling at the
    coarse vertices.

Network (4 levels, widths c0..c3, ReLU, 'same' 3x3x3 convolutions with
zero padding, average pooling over the existing children, nearest
upsampling, additive skips):
  enc_l:  h = relu(conv_b(relu(conv_a(x))))          l = 0..2 (pool after)
  bottom: relu(conv_b(relu(conv_a(.))))
  dec_l:  h = relu(conv_a(up(h))) + s_l; h = relu(conv_b(h))   l = 2, 1, 0
  head:   conv(c0 -> 1)
Learned flexible CG (the coarse level itself is not in the paper; this is
the definition the GPU solver follows):
  * network input: channel 0 is P_c^T r scaled to unit RMS, channel 1 the
    coarse volume fraction (coarse_eta);
  * correction: z = S r + gamma P_c y with y the network output and
    gamma = (y . P_c^T r) / (y . A_c y), A_c = P_c^T A P_c the Galerkin
    coarse operator, gamma = 0 when the quotient is not positive finite;
  * flexible CG, truncated to m directions: the new direction is z_new
    made A-orthogonal to the last m directions,
    p = z_new - sum_j (z_new . A p_j) / (p_j . A p_j) p_j, since a
    preconditioner that changes from step to step (a network is nonlinear
    in r) breaks the short recurrence of CG; m = 1 is the Polak-Ribiere
    form beta = -(z_new . A p) / (p . A p);
  * training targets, at the coarse vertices, zero where the vertex
    function touches no physical material, scaled to unit RMS: the error
    e = x* - x_k minus the Schwarz apply z_k = S r_k, sampled (kind
    "e-Sr"); the error itself (kind "e"); or the coarse Galerkin
    projection of the error (kind "coarse"): the y minimising
    ||e - P_c y||_A over the material vertices, the solution of
    A_c y = P_c^T r there (r = A e), a plain function of the network's
    residual input.
Parameters are one flat vector: per convolution W[co][ci][27] then b[co],
in the order enc0a enc0b enc1a enc1b enc2a enc2b bota botb up2a up2b up1a
up1b up0a up0b head; the tap index is dz*9 + dy*3 + dx (offsets -1..1).
"""
from __future__ import annotations

import numpy as np

from .pcg import BREAKDOWN, NOTCONV, OK

LAYERS = ["enc0a", "enc0b", "enc1a", "enc1b", "enc2a", "enc2b", "bota", "botb",
          "up2a", "up2b", "up1a", "up1b", "up0a", "up0b", "head"]


def layer_shapes(ch, in_ch=2):
    c0, c1, c2, c3 = ch
    io = [(in_ch, c0), (c0, c0), (c0, c1), (c1, c1), (c1, c2), (c2, c2), (c2, c3), (c3, c3),
          (c3, c2), (c2, c2), (c2, c1), (c1, c1), (c1, c0), (c0, c0), (c0, 1)]
    return dict(zip(LAYERS, io))


def n_params(ch, in_ch=2):
    return sum(ci * co * 27 + co for ci, co in layer_shapes(ch, in_ch).values())


def unpack(theta, ch, in_ch=2):
    out = {}
    off = 0
    for name, (ci, co) in layer_shapes(ch, in_ch).items():
        w = theta[off: off + co * ci * 27].reshape(co, ci, 3, 3, 3)
        off += co * ci * 27
        b = theta[off: off + co]
        off += co
        out[name] = (w, b)
    assert off == theta.size
    return out


# ------------------------------------------------------------- layers
def conv3d(x, w, b):
    """x (B, Ci, D, H, W), w (Co, Ci, 3, 3, 3), b (Co): 'same' convolution."""
    B, Ci, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    y = np.zeros((B, w.shape[0], D, H, W))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                patch = xp[:, :, dz:dz + D, dy:dy + H, dx:dx + W]
                y += np.einsum("bcdhw,oc->bodhw", patch, w[:, :, dz, dy, dx])
    return y + b[None, :, None, None, None]


def conv3d_backward(x, w, gy):
    """Gradients of sum(gy * conv3d(x, w, b)) w.r.t. x, w, b."""
    B, Ci, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                patch = xp[:, :, dz:dz + D, dy:dy + H, dx:dx + W]
                gw[:, :, dz, dy, dx] = np.einsum("bodhw,bcdhw->oc", gy, patch)
                gxp[:, :, dz:dz + D, dy:dy + H, dx:dx + W] += np.einsum(
                    "bodhw,oc->bcdhw", gy, w[:, :, dz, dy, dx])
    gb = gy.sum(axis=(0, 2, 3, 4))
    return gxp[:, :, 1:-1, 1:-1, 1:-1], gw, gb


def pool(x):
    """Average over the existing children of every coarse voxel."""
    B, C, D, H, W = x.shape
    d, h, w = (D + 1) // 2, (H + 1) // 2, (W + 1) // 2
    s = np.zeros((B, C, d, h, w))
    cnt = np.zeros((d, h, w))
    for a in range(2):
        for bb in range(2):
            for c in range(2):
                sub = x[:, :, a::2, bb::2, c::2]
                s[:, :, :sub.shape[2], :sub.shape[3], :sub.shape[4]] += sub
                cnt[:sub.shape[2], :sub.shape[3], :sub.shape[4]] += 1
    return s / cnt


def pool_backward(gy, shape):
    B, C, D, H, W = shape
    d, h, w = gy.shape[2:]
    cnt = np.zeros((d, h, w))
    for a in range(2):
        for bb in range(2):
            for c in range(2):
                n0 = len(range(a, D, 2))
                n1 = len(range(bb, H, 2))
                n2 = len(range(c, W, 2))
                cnt[:n0, :n1, :n2] += 1
    g = gy / cnt
    gx = np.zeros(shape)
    for a in range(2):
        for bb in range(2):
            for c in range(2):
                n0 = len(range(a, D, 2))
                n1 = len(range(bb, H, 2))
                n2 = len(range(c, W, 2))
                gx[:, :, a::2, bb::2, c::2] = g[:, :, :n0, :n1, :n2]
    return gx


def upsample(x, size):
    """Nearest upsampling to the given fine size: y[i] = x[i // 2]."""
    D, H, W = size
    iz = np.arange(D) // 2
    iy = np.arange(H) // 2
    ix = np.arange(W) // 2
    return x[:, :, iz][:, :, :, iy][:, :, :, :, ix]


def upsample_backward(gy, coarse_shape):
    gx = np.zeros(coarse_shape)
    D, H, W = gy.shape[2:]
    for z in range(D):
        for y in range(H):
            for xx in range(W):
                gx[:, :, z // 2, y // 2, xx // 2] += gy[:, :, z, y, xx]
    return gx


def relu(x):
    return np.maximum(x, 0.0)


# ------------------------------------------------------------- network
def forward(theta, x, ch, in_ch=2):
    """U-Net output (B, 1, D, H, W) for input x (B, in_ch, D, H, W)."""
    return _run(theta, x, None, ch, in_ch)[0]


def loss_and_grad(theta, x, target, ch, in_ch=2):
    """Mean squared error over all output voxels and its gradient with
    respect to the flat parameter vector."""
    _, loss, grad = _run(theta, x, target, ch, in_ch)
    return loss, grad


def _run(theta, x, target, ch, in_ch):
    """Forward pass, and with a target also the backward pass, written
    level by level."""
    P = unpack(theta, ch, in_ch)

    def fconv(name, h, act=True):
        w, b = P[name]
        pre = conv3d(h, w, b)
        return (relu(pre) if act else pre), pre

    saved = {}
    h = x
    skips = []
    for lvl in range(3):
        a_in = h
        h1, p1 = fconv(f"enc{lvl}a", a_in)
        h2, p2 = fconv(f"enc{lvl}b", h1)
        saved[f"enc{lvl}"] = (a_in, p1, h1, p2)
        skips.append(h2)
        h = pool(h2)
    b_in = h
    b1, q1 = fconv("bota", b_in)
    b2, q2 = fconv("botb", b1)
    saved["bot"] = (b_in, q1, b1, q2)
    h = b2
    for lvl in (2, 1, 0):
        u = upsample(h, skips[lvl].shape[2:])
        a1, r1 = fconv(f"up{lvl}a", u)
        m = a1 + skips[lvl]
        a2, r2 = fconv(f"up{lvl}b", m)
        saved[f"up{lvl}"] = (h.shape, u, r1, m, r2)
        h = a2
    y, _ = fconv("head", h, act=False)
    if target is None:
        return y, None, None
    diff = y - target
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size
    grads = {}

    def bconv(name, h_in, pre, g_out, act=True):
        gpre = g_out * (pre > 0) if act else g_out
        gx, gw, gb = conv3d_backward(h_in, P[name][0], gpre)
        grads[name] = (gw, gb)
        return gx

    g = bconv("head", h, None, g, act=False)
    gskip = {}
    for lvl in (0, 1, 2):
        hshape, u, r1, m, r2 = saved[f"up{lvl}"]
        g = bconv(f"up{lvl}b", m, r2, g)
        gskip[lvl] = g.copy()
        g = bconv(f"up{lvl}a", u, r1, g)
        g = upsample_backward(g, hshape)
    b_in, q1, b1, q2 = saved["bot"]
    g = bconv("botb", b1, q2, g)
    g = bconv("bota", b_in, q1, g)
    for lvl in (2, 1, 0):
        a_in, p1, h1, p2 = saved[f"enc{lvl}"]
        g = pool_backward(g, skips[lvl].shape) + gskip[lvl]
        g = bconv(f"enc{lvl}b", h1, p2, g)
        g = bconv(f"enc{lvl}a", a_in, p1, g)
    flat = []
    for name in LAYERS:
        gw, gb = grads[name]
        flat.append(gw.ravel())
        flat.append(gb)
    return y, loss, np.concatenate(flat)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; t counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ transfers
def vertex_index(desc):
    """Unknown index of every vertex of the (n+1)^d vertex grid, shape
    (n+1,)*d with the last axis the first coordinate."""
    n, p, d = desc["n"], desc["p"], desc["dim"]
    n1 = p * n + 1
    g = np.arange(n + 1) * p
    if d == 2:
        return g[None, :] + n1 * g[:, None]
    return g[None, None, :] + n1 * (g[None, :, None] + n1 * g[:, None, None])


def prolong_1d(nc):
    """(2nc+1) x (nc+1) linear interpolation matrix."""
    P = np.zeros((2 * nc + 1, nc + 1))
    for i in range(nc + 1):
        P[2 * i, i] = 1.0
    for i in range(nc):
        P[2 * i + 1, i] = 0.5
        P[2 * i + 1, i + 1] = 0.5
    return P


def prolong(desc, wc):
    """Coarse vertex values (nc+1)^d -> unknown vector (vertex unknowns)."""
    n = desc["n"]
    P1 = prolong_1d(n // 2)
    if desc["dim"] == 2:
        fine = P1 @ wc @ P1.T
    else:
        fine = np.einsum("ia,jb,kc,abc->ijk", P1, P1, P1, wc)
    out = np.zeros((desc["p"] * n + 1) ** desc["dim"])
    out[vertex_index(desc).ravel()] = fine.ravel()
    return out


def restrict(desc, r):
    """Residual -> coarse vertex grid, the transpose of prolong."""
    n = desc["n"]
    P1 = prolong_1d(n // 2)
    fine = r[vertex_index(desc)]
    if desc["dim"] == 2:
        return P1.T @ fine @ P1
    return np.einsum("ia,jb,kc,ijk->abc", P1, P1, P1, fine)


def sample(desc, e):
    """Error -> its values at the coarse vertices."""
    return e[vertex_index(desc)][tuple([slice(None, None, 2)] * desc["dim"])]


def coarse_eta(desc, eta):
    """Volume fraction at the coarse vertices: mean over the coarse cells
    (2^d fine cells each, averaged) that touch the vertex."""
    n, d = desc["n"], desc["dim"]
    nc = n // 2
    shape = (n,) * d
    e = eta.reshape(shape)           # last axis = first coordinate
    if d == 3:
        cc = e.reshape(nc, 2, nc, 2, nc, 2).mean(axis=(1, 3, 5))
    else:
        cc = e.reshape(nc, 2, nc, 2).mean(axis=(1, 3))
    out = np.zeros((nc + 1,) * d)
    cnt = np.zeros((nc + 1,) * d)
    for off in np.ndindex(*(2,) * d):
        sl = tuple(slice(o, o + nc) for o in off)
        out[sl] += cc
        cnt[sl] += 1
    return out / cnt


def prolong_matrix(desc):
    """P_c as a sparse (unknowns x coarse vertices) matrix; coarse vertex
    (a, b, c) has column a + G (b + G c) with G = n/2 + 1."""
    import scipy.sparse as sp
    n, d = desc["n"], desc["dim"]
    P1 = sp.csr_matrix(prolong_1d(n // 2))
    if d == 2:
        Pv = sp.kron(P1, P1)                 # rows: vertex y*(n+1) + x
    else:
        Pv = sp.kron(sp.kron(P1, P1), P1)
    rows = vertex_index(desc).ravel()        # vertex (z, y, x) -> unknown
    nd = (desc["p"] * n + 1) ** d
    inj = sp.csr_matrix((np.ones(rows.size), (rows, np.arange(rows.size))),
                        shape=(nd, rows.size))
    return (inj @ Pv).tocsr()


def coarse_operator(desc, A):
    """Galerkin coarse operator A_c = P_c^T A P_c (dense)."""
    P = prolong_matrix(desc)
    return (P.T @ (A @ P)).toarray()


def vertex_mask(desc, eta):
    """1 at coarse vertices whose fine vertex function touches a cell with
    physical material (eta > 0), else 0."""
    n, d = desc["n"], desc["dim"]
    e = eta.reshape((n,) * d) > 0
    G = n // 2 + 1
    out = np.zeros((G,) * d)
    for idx in np.ndindex(*out.shape):
        sl = tuple(slice(max(2 * i - 1, 0), min(2 * i + 1, n)) for i in idx)
        out[idx] = 1.0 if e[sl].any() else 0.0
    return out


def unit_rms(v):
    nrm = float(np.sqrt(np.mean(v * v)))
    return v / nrm if nrm > 0 else np.zeros_like(v)


def network_input(desc, r, eta):
    """Channel 0: P_c^T r scaled to unit RMS; channel 1: coarse eta."""
    return np.stack([unit_rms(restrict(desc, r)), coarse_eta(desc, eta)])


def snapshot_target(desc, e, z, eta, kind="e-Sr"):
    """Training target at the coarse vertices: the error e (kind "e") or the
    error left after the Schwarz apply, e - S r (kind "e-Sr"), sampled,
    zero on purely fictitious vertices, scaled to unit RMS."""
    v = e - z if kind == "e-Sr" else e
    return unit_rms(sample(desc, v) * vertex_mask(desc, eta))


def coarse_projection(desc, A, r, eta):
    """Coarse Galerkin projection of the error behind the residual r: on the
    material vertices (vertex_mask) y solves A_c y = P_c^T r, elsewhere
    y = 0.  P_c y is then the A-orthogonal projection of e = A^{-1} r onto
    the span of the material coarse vertex functions."""
    m = vertex_mask(desc, eta).ravel() > 0
    Ac = coarse_operator(desc, A)
    rc = restrict(desc, r).ravel()
    y = np.zeros(rc.size)
    y[m] = np.linalg.solve(Ac[np.ix_(m, m)], rc[m])
    return y.reshape(vertex_mask(desc, eta).shape)


def coarse_projection_target(desc, A, r, eta):
    """Training target of kind "coarse": coarse_projection scaled to unit
    RMS."""
    return unit_rms(coarse_projection(desc, A, r, eta))


def fcg(A, b, S, P, Ac, correction, tol=1e-8, maxit=300000, m=1):
    """Flexible CG with the preconditioner z = S r + gamma P y,
    y = correction(r) on the coarse vertices and
    gamma = (y . P^T r) / (y . A_c y) the energy-optimal step along P y
    (zero when that is not a positive finite number).  Each new direction is
    made A-orthogonal to the last m directions (m = 1: the Polak-Ribiere
    form).  Residual stop ||r|| / ||b|| <= tol; x_0 = 0."""
    n = b.size
    x = np.zeros(n)
    r = b.copy()
    b0 = float(np.linalg.norm(b))
    gammas = []

    def precond(r):
        z = S @ r
        y = np.asarray(correction(r), dtype=np.float64).ravel()
        den = float(y @ (Ac @ y))
        num = float(y @ (P.T @ r))
        g = num / den if (den > 0 and np.isfinite(den) and np.isfinite(num)) else 0.0
        gammas.append(g)
        return z + g * (P @ y)

    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    res = [1.0 if b0 > 0 else 0.0]
    status = NOTCONV
    if b0 == 0.0:
        return x, {"iters": 0, "status": OK, "res": res, "gamma": gammas}
    kept = []          # (p_j, A p_j, p_j . A p_j) of the last m directions
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
        res.append(float(np.linalg.norm(r)) / b0)
        if res[-1] <= tol:
            status = OK
            break
        kept.append((p, q, pq))
        if len(kept) > m:
            kept.pop(0)
        z = precond(r)
        rz = float(r @ z)
        p = z.copy()
        for pj, qj, pqj in kept:
            p -= (float(z @ qj) / pqj) * pj
    return x, {"iters": it, "status": status, "res": res, "gamma": gammas}
