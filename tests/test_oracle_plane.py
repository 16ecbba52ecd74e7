"""Pins of the road-plane oracle (oracle/plane.py, Sec. II-A): exact recovery of a
noiseless plane, recovery under gross outliers, degenerate draws, the tie rule, the
least-squares refit and the roll angle."""
import numpy as np

from oracle import plane as PL


def _plane_map(H, W, a0, a1, a2):
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    return a0 + a1 * v + a2 * u


def _draws(rng, valid, K):
    idx = np.flatnonzero(valid.ravel())
    return np.stack([rng.choice(idx, 3, replace=False) for _ in range(K)])


def test_noiseless_plane_is_recovered_exactly():
    H, W = 40, 64
    d = _plane_map(H, W, 10.0, 0.15, -0.02)
    valid = np.ones((H, W), bool)
    rng = np.random.default_rng(0)
    plane, counts, best, inl = PL.ransac_plane(d, valid, _draws(rng, valid, 8), 0.1)
    assert np.allclose(plane, [10.0, 0.15, -0.02], atol=1e-10)
    assert inl.all() and counts.max() == H * W


def test_gross_outliers_are_rejected():
    H, W = 60, 80
    rng = np.random.default_rng(1)
    d = _plane_map(H, W, 5.0, 0.1, 0.01) + rng.normal(0.0, 0.05, (H, W))
    out = rng.random((H, W)) < 0.3
    d[out] = rng.uniform(0.0, 60.0, out.sum())
    valid = np.ones((H, W), bool)
    plane, counts, best, inl = PL.ransac_plane(d, valid, _draws(rng, valid, 64), 0.25)
    assert np.allclose(plane, [5.0, 0.1, 0.01], atol=0.05)
    # the refit's inliers are the plane's points (a few outliers fall near the plane)
    assert (inl & ~out).sum() >= 0.99 * (~out).sum() and (inl & out).sum() < 0.02 * out.sum()


def test_degenerate_draws_and_ties():
    H, W = 10, 10
    d = _plane_map(H, W, 1.0, 0.5, 0.25)
    valid = np.ones((H, W), bool)
    collinear = [0 * W + 0, 1 * W + 1, 2 * W + 2]     # on the diagonal u = v
    good = [0 * W + 0, 0 * W + 5, 7 * W + 3]
    plane, counts, best, _ = PL.ransac_plane(d, valid, np.array([collinear, good, good]), 0.1)
    assert counts[0] == -1 and counts[1] == counts[2] == H * W
    assert best == 1                                 # equal counts: the lowest index
    assert PL.plane_through_three([0, 1, 2], [0, 1, 2], [1, 2, 3]) is None
    # draws outside the image are degenerate; with no hypothesis left the plane is NaN
    plane, counts, best, inl = PL.ransac_plane(d, valid, np.array([[0, 5, H * W], [-1, 3, 40], good]), 0.1)
    assert list(counts) == [-1, -1, H * W] and best == 2
    plane, counts, best, inl = PL.ransac_plane(d, valid, np.array([collinear, [0, 1, H * W]]), 0.1)
    assert list(counts) == [-1, -1] and np.isnan(plane).all() and not inl.any()


def test_least_squares_refit_and_roll():
    # symmetric noise around a plane (+e and -e at mirrored points) leaves the fit unchanged
    u = np.array([0, 10, 0, 10, 0, 10, 0, 10], np.float64)
    v = np.array([0, 0, 8, 8, 0, 0, 8, 8], np.float64)
    e = np.array([0.3, -0.2, 0.1, 0.4, -0.3, 0.2, -0.1, -0.4])
    d = 2.0 + 0.5 * v - 0.25 * u + e
    assert np.allclose(PL.least_squares_plane(u, v, d), [2.0, 0.5, -0.25], atol=1e-12)
    gamma = 0.07
    a1 = 0.2
    assert abs(PL.roll_angle((3.0, a1, -np.tan(gamma) * a1)) - gamma) < 1e-12
