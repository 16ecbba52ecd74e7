"""Pins of the oracle gradient: FP64 central differences of the oracle loss, and the
loss against the full-volume forward oracle.

The plane is chosen so that no warp sample position lies within 0.2 px of an
integer: linear interpolation has kinks at integers, and a difference quotient
across one would average two slopes.
"""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import stereo as S
from synth.road import RoadScene, make_pair

PLANE = (5.5, 0.004, 0.002, 0.0)


def _case(H=30, W=44, seed=11, r=2, rho=2, D=6):
    p = make_pair(RoadScene(H, W, 0.0, 5.5, n_bumps=1, bump_amp=0.5, noise_right=2.0,
                            dtype="f32"), seed)
    rng = np.random.default_rng(seed)
    disp = rng.integers(0, D, (H, W))
    mask = rng.random((H, W)) < 0.5
    return p.left.astype(np.float64), p.right.astype(np.float64), disp, mask, r, rho


def test_sample_positions_avoid_kinks():
    H, W = 30, 44
    s = S.shift_field(PLANE, H, W)
    v, u = np.mgrid[0:H, 0:W]
    frac = np.mod(u - s, 1.0)
    assert np.all((frac > 0.2) & (frac < 0.8))


def test_loss_matches_full_forward_volume():
    L, R, disp, mask, r, rho = _case()
    gd, gr = 2.0, 0.1
    Wp = S.warp(R, PLANE)
    CL, _ = S.cost_volumes(L, Wp, 6, r, 1e-2)
    AL = S.aggregate_volume(CL, L, rho, gd, gr)
    vv, uu = np.nonzero(mask)
    ref = AL[disp[vv, uu], vv, uu].sum()
    got = A.loss(L, R, PLANE, disp, mask, r, rho, gd, gr)
    assert abs(got - ref) < 1e-10


def test_plane_gradient_matches_central_differences():
    L, R, disp, mask, r, rho = _case()
    gd, gr = 2.0, 0.1
    loss, gL, gR, gp = A.grad(L, R, PLANE, disp, mask, r, rho, gd, gr)
    h = 1e-4
    for k in range(3):
        e = np.zeros(4)
        e[k] = h
        lp = A.loss(L, R, tuple(np.add(PLANE, e)), disp, mask, r, rho, gd, gr)
        lm = A.loss(L, R, tuple(np.subtract(PLANE, e)), disp, mask, r, rho, gd, gr)
        fd = (lp - lm) / (2 * h)
        assert abs(gp[k] - fd) <= 1e-5 * abs(fd) + 1e-7, (k, gp[k], fd)


@pytest.mark.parametrize("which", ["left", "right"])
def test_image_gradient_matches_central_differences(which):
    L, R, disp, mask, r, rho = _case()
    gd, gr = 2.0, 0.1
    _, gL, gR, _ = A.grad(L, R, PLANE, disp, mask, r, rho, gd, gr)
    g = gL if which == "left" else gR
    rng = np.random.default_rng(3)
    H, W = L.shape
    picks = [(int(rng.integers(H)), int(rng.integers(W))) for _ in range(10)]
    picks += [(0, 0), (H - 1, W - 1), (0, W // 2), (H // 2, 0)]   # clamped-read edges
    h = 1e-3
    scale = np.abs(g).max()
    for (y, x) in picks:
        Lp, Lm, Rp, Rm = L.copy(), L.copy(), R.copy(), R.copy()
        if which == "left":
            Lp[y, x] += h
            Lm[y, x] -= h
        else:
            Rp[y, x] += h
            Rm[y, x] -= h
        fd = (A.loss(Lp, Rp, PLANE, disp, mask, r, rho, gd, gr)
              - A.loss(Lm, Rm, PLANE, disp, mask, r, rho, gd, gr)) / (2 * h)
        assert abs(g[y, x] - fd) <= 1e-5 * abs(fd) + 1e-7 * scale, (which, y, x, g[y, x], fd)


def test_plane_gradient_wider_windows():
    L, R, disp, mask, r, rho = _case(H=26, W=40, seed=5, r=3, rho=4, D=5)
    gd, gr = 3.0, 0.1
    _, _, _, gp = A.grad(L, R, PLANE, disp, mask, r, rho, gd, gr)
    h = 1e-4
    for k in range(3):
        e = np.zeros(4)
        e[k] = h
        fd = (A.loss(L, R, tuple(np.add(PLANE, e)), disp, mask, r, rho, gd, gr)
              - A.loss(L, R, tuple(np.subtract(PLANE, e)), disp, mask, r, rho, gd, gr)) / (2 * h)
        assert abs(gp[k] - fd) <= 1e-5 * abs(fd) + 1e-7, (k, gp[k], fd)
