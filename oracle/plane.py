"""FP64 oracle of the road-plane estimation of Sec. II-A: the warp's plane fitted to
reliable correspondences by least squares inside RANSAC, and the roll angle.

TEST INFRASTRUCTURE ONLY (see oracle/stereo.py): used by tests and the benchmark's
CPU-baseline leg, never by the library.

Reading (Sec. II-A describes the method; the paper's correspondences come from ORB
matches on real images, which synthetic pairs do not need): the correspondences are
the pixels (u, v) with a valid disparity d (a previous frame's post-processed map,
or any disparity map with a validity mask); the model is the plane of disparities
d = a0 + a1 v + a2 u (Eq. 2 with the u-term of the roll-fitted plane of Sec. II-A);
RANSAC draws K hypotheses, each the plane through 3 of the points (the random draws
are an input, so the oracle and the kernels use the same ones), keeps the hypothesis
with the most inliers |d - a0 - a1 v - a2 u| <= threshold (ties to the lowest
hypothesis index; hypotheses whose 3 points do not determine a plane, or that draw
an index outside the image, score -1), and
refits that hypothesis's inliers by least squares.  The roll angle is
gamma = arctan(-a2 / a1) (Sec. II-A, with gamma_1 = a2 and gamma_2 = a1).
"""
from __future__ import annotations

import numpy as np


def plane_through_three(u, v, d):
    """The plane d = a0 + a1 v + a2 u through three points, or None when they do not
    determine one (collinear in (u, v))."""
    A = np.stack([np.ones(3), np.asarray(v, np.float64), np.asarray(u, np.float64)], axis=1)
    if abs(np.linalg.det(A)) < 1e-9:
        return None
    return np.linalg.solve(A, np.asarray(d, np.float64))


def inliers(plane, u, v, d, threshold):
    """|d - (a0 + a1 v + a2 u)| <= threshold."""
    a0, a1, a2 = plane
    return np.abs(np.asarray(d, np.float64) - (a0 + a1 * np.asarray(v, np.float64) +
                                               a2 * np.asarray(u, np.float64))) <= threshold


def least_squares_plane(u, v, d):
    """argmin sum (d - a0 - a1 v - a2 u)^2 (library least squares)."""
    A = np.stack([np.ones(len(u)), np.asarray(v, np.float64), np.asarray(u, np.float64)], axis=1)
    sol, *_ = np.linalg.lstsq(A, np.asarray(d, np.float64), rcond=None)
    return sol


def ransac_plane(disp, valid, samples, threshold):
    """RANSAC with least-squares refit over a disparity map.

    disp [H][W], valid [H][W] bool; samples [K][3] linear pixel indices (v * W + u).
    Returns (plane (a0, a1, a2), counts [K] (-1 for degenerate hypotheses), best index,
    inlier mask [H][W] of the best hypothesis)."""
    disp = np.asarray(disp, np.float64)
    H, W = disp.shape
    vv, uu = np.mgrid[0:H, 0:W]
    ok = np.asarray(valid, bool)
    pu, pv, pd = uu[ok], vv[ok], disp[ok]
    samples = np.asarray(samples, np.int64)
    counts = np.full(len(samples), -1, np.int64)
    planes = []
    for k, s in enumerate(samples):
        if np.any((s < 0) | (s >= H * W)):     # a draw outside the image: no hypothesis
            planes.append(None)
            continue
        sv, su = s // W, s % W
        pl = plane_through_three(su, sv, disp[sv, su])
        planes.append(pl)
        if pl is not None:
            counts[k] = int(inliers(pl, pu, pv, pd, threshold).sum())
    best = int(np.argmax(counts))          # first maximum: ties to the lowest index
    if planes[best] is None:               # every hypothesis degenerate
        return np.full(3, np.nan), counts, best, np.zeros_like(ok)
    inl = ok & inliers(planes[best], uu, vv, disp, threshold)
    plane = least_squares_plane(uu[inl], vv[inl], disp[inl])
    return plane, counts, best, inl


def roll_angle(plane) -> float:
    """gamma = arctan(-gamma_1 / gamma_2) for the plane d = gamma_0 + gamma_1 u + gamma_2 v."""
    a0, a1, a2 = plane
    return float(np.arctan(-a2 / a1))
