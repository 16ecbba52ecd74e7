"""FP64 oracle of the differentiable form: the loss
    L(theta, I_l, I_r) = sum over p in Omega of A_ref(p, d*(p))
with the selected disparities d* and the pixel set Omega held fixed, and its exact
gradient with respect to the warp plane theta = (a0, a1, a2) and both images.

TEST INFRASTRUCTURE ONLY (see oracle/stereo.py): used by tests, the smoke check and
the benchmark's CPU-baseline leg; never by the library.

The loss chains the paper's forward steps: the warp of Sec. II-A, the correlation
of Eq. 3-5 and the bilateral aggregation of Eq. 8-10.  The paper has no backward
pass; the gradient below is the chain rule of those definitions, written out term
by term:
  dL/dc(q, d)   = w(p, q) / Z(p)                 for every p in Omega with d*(p) = d
  dL/dw(p, q)   = (c(q, d*(p)) - A(p)) / Z(p)
  dw/dg(q)      = -2 w (g(q) - g(p)) / (255^2 gamma_r^2),   dw/dg(p) = -dw/dg(q)
  dc/dl_i       = (r_i - mu_r) / sqrt(S_ll S_rr) - c (l_i - mu_l) / S_ll
  dc/dr_i       = (l_i - mu_l) / sqrt(S_ll S_rr) - c (r_i - mu_r) / S_rr
  warped(u, v)  = I0 + f (I1 - I0),  x = u - s(u, v):
                  dW/dI0 = 1 - f, dW/dI1 = f, dW/ds = -(I1 - I0), ds/dtheta = (1, v, u)
Block reads are clamp-to-edge, so a clamped read sends its gradient to the edge
pixel it read.  Where either block std-dev is below sigma_min the correlation is the
constant 0 and contributes no gradient.
"""
from __future__ import annotations

import numpy as np

from . import stereo as S

CHUNK = 512  # Omega pixels per vectorised chunk (memory bound only)


def _omega(mask):
    vv, uu = np.nonzero(mask)
    return uu.astype(np.int64), vv.astype(np.int64)


def loss(left, right, plane, disp, mask, block_radius, agg_radius, gamma_d, gamma_r,
         sigma_min=1e-2) -> float:
    """Sum of aggregated reference costs at the frozen disparities over Omega."""
    Wp = S.warp(right, plane)
    pu, pv = _omega(mask)
    d = np.asarray(disp)[pv, pu].astype(np.int64)

    def cost_at(x, y, dd):
        return S.cost_entries(left, Wp, x, y, dd, block_radius, sigma_min)

    total = 0.0
    for i in range(0, pu.size, CHUNK):
        sl = slice(i, i + CHUNK)
        total += S.aggregate_entries(cost_at, left, pu[sl], pv[sl], d[sl], agg_radius,
                                     gamma_d, gamma_r).sum()
    return float(total)


def _block_positions(H, W, u, v, r):
    offs = np.arange(-r, r + 1)
    dy = np.repeat(offs, 2 * r + 1)
    dx = np.tile(offs, 2 * r + 1)
    return (np.clip(v[..., None] + dy, 0, H - 1), np.clip(u[..., None] + dx, 0, W - 1))


def grad(left, right, plane, disp, mask, block_radius, agg_radius, gamma_d, gamma_r,
         sigma_min=1e-2):
    """Returns (loss, grad_left [H][W], grad_right [H][W], grad_plane [3])."""
    L = np.asarray(left, np.float64)
    R = np.asarray(right, np.float64)
    H, W = L.shape
    Wp = S.warp(R, plane)
    pu, pv = _omega(mask)
    dsel = np.asarray(disp)[pv, pu].astype(np.int64)

    gL = np.zeros((H, W))
    gWp = np.zeros((H, W))
    total = 0.0
    kr = -2.0 / (255.0 ** 2 * gamma_r ** 2)
    for i in range(0, pu.size, CHUNK):
        u = pu[i:i + CHUNK]
        v = pv[i:i + CHUNK]
        d = dsel[i:i + CHUNK]
        w, qx, qy = S.bilateral_weights(L, u, v, agg_radius, gamma_d, gamma_r)
        Z = w.sum(-1)
        dq = np.broadcast_to(d[:, None], qx.shape)
        bl = S.block_values(L, qx, qy, block_radius)            # [P, m, n]
        br = S.block_values(Wp, qx - dq, qy, block_radius)
        c = S.zncc(bl, br, sigma_min)                           # [P, m]
        A = (w * c).sum(-1) / Z
        total += A.sum()

        # aggregation: w.r.t. the costs and w.r.t. the weights (guide = left image)
        dc = w / Z[:, None]
        dw = (c - A[:, None]) / Z[:, None]
        gq = dw * w * kr * (L[qy, qx] - L[v, u][:, None])       # zero on outside taps
        np.add.at(gL, (qy, qx), gq)
        np.add.at(gL, (v, u), -gq.sum(-1))

        # correlation: w.r.t. both blocks
        ml = bl.mean(-1, keepdims=True)
        mr = br.mean(-1, keepdims=True)
        el = bl - ml
        er = br - mr
        n = bl.shape[-1]
        sll = (el * el).sum(-1)
        srr = (er * er).sum(-1)
        ok = (np.sqrt(sll / n) >= sigma_min) & (np.sqrt(srr / n) >= sigma_min)
        den = np.sqrt(np.where(ok, sll * srr, 1.0))
        cc = np.where(ok, c, 0.0)[..., None]
        dl = er / den[..., None] - cc * el / np.where(ok, sll, 1.0)[..., None]
        dr = el / den[..., None] - cc * er / np.where(ok, srr, 1.0)[..., None]
        coef = np.where(ok, dc, 0.0)[..., None]
        ly, lx = _block_positions(H, W, qx, qy, block_radius)
        ry, rx = _block_positions(H, W, qx - dq, qy, block_radius)
        np.add.at(gL, (ly, lx), coef * dl)
        np.add.at(gWp, (ry, rx), coef * dr)

    # warp: linear interpolation along the row (transpose) and the shift derivative
    vv, uu = np.mgrid[0:H, 0:W]
    s = S.shift_field(plane, H, W)
    x = np.clip(uu - s, -2.0, W + 1.0)
    x0f = np.floor(x)
    f = x - x0f
    x0 = x0f.astype(np.int64)
    c0 = np.clip(x0, 0, W - 1)
    c1 = np.clip(x0 + 1, 0, W - 1)
    gR = np.zeros((H, W))
    np.add.at(gR, (vv, c0), gWp * (1.0 - f))
    np.add.at(gR, (vv, c1), gWp * f)
    dWds = -(R[vv, c1] - R[vv, c0])
    t = gWp * dWds
    gplane = np.array([t.sum(), (t * vv).sum(), (t * uu).sum()])
    return float(total), gL, gR, gplane
