"""Reconstruction accuracy in millimetres, measured the way Sec. III measures it on
its 3-D printed models, here on the synthetic road's known bumps:

  1. around a bump, take a square region of the reconstructed point cloud;
  2. fit the ground plane n0 x + n1 y + n2 z + n3 = 0 through the 3-D points at the
     region's four corners (the road surface);
  3. take random 3-D points on the bump and their distances to that plane: the
     measured heights of the model above (or below) the road.

The same is done on the ground truth: the generator's disparities triangulated with
the same camera (Sec. II-D) give the true heights of the same pixels above the plane
through the true corners.  The accuracy is |measured - true| per sampled point.

Host-side analysis of the library's output (NumPy, FP64); not part of the GPU path.
"""
from __future__ import annotations

import numpy as np


def plane_through(points: np.ndarray) -> np.ndarray:
    """Least-squares plane through k >= 3 points [k, 3]: (n0, n1, n2, n3) with a unit
    normal (n0, n1, n2) and n . p + n3 = 0 (exact for coplanar points)."""
    p = np.asarray(points, np.float64)
    c = p.mean(axis=0)
    _, _, vt = np.linalg.svd(p - c)
    n = vt[-1]
    return np.array([n[0], n[1], n[2], -float(n @ c)])


def point_plane_distance(plane: np.ndarray, points: np.ndarray) -> np.ndarray:
    """Signed distance n . p + n3 of points [..., 3] to a plane with a unit normal."""
    return np.asarray(points, np.float64) @ plane[:3] + plane[3]


def triangulate(disp: np.ndarray, camera) -> np.ndarray:
    """Sec. II-D: z = f T / d, x = (u - u0) z / f, y = (v - v0) z / f (NaN for d <= 0)."""
    f, T, u0, v0 = (float(t) for t in camera)
    H, W = disp.shape
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    d = np.asarray(disp, np.float64)
    z = np.where(d > 0, f * T / np.where(d > 0, d, 1.0), np.nan)
    return np.stack([(u - u0) * z / f, (v - v0) * z / f, z], axis=-1)


def bump_study(xyz: np.ndarray, disp_gt: np.ndarray, camera, bumps, rng: np.random.Generator,
               sigma: float = 10.0, half: int = 30, n_points: int = 40, margin: int = 8) -> dict:
    """The Sec. III accuracy measurement on every bump whose region fits the image.

    xyz      reconstructed points [H][W][3] (NaN where invalid), metres
    disp_gt  the generator's disparity [H][W]; bumps: (u, v, amplitude) per bump
    Region: a (2 half + 1)^2 square centred on the bump (the bump's height there is
    below e^-9 of its peak at the corners).  Corners: the mean of the valid points of
    the 3 x 3 patch at each corner.  Points: n_points random valid pixels within
    sigma sqrt(2 ln 2) of the centre (the bump's upper half).  Returns per-point
    errors in mm and their summary."""
    gt = triangulate(disp_gt, camera)
    H, W = disp_gt.shape
    errs, heights, used = [], [], 0
    r_core = sigma * np.sqrt(2.0 * np.log(2.0))
    for (bu, bv, amp) in bumps:
        cu, cv = int(round(bu)), int(round(bv))
        if cu - half < margin or cv - half < margin or cu + half >= W - margin or cv + half >= H - margin:
            continue
        corners_m, corners_t = [], []
        for (du, dv) in ((-half, -half), (half, -half), (-half, half), (half, half)):
            pm = xyz[cv + dv - 1:cv + dv + 2, cu + du - 1:cu + du + 2].reshape(-1, 3)
            pt = gt[cv + dv - 1:cv + dv + 2, cu + du - 1:cu + du + 2].reshape(-1, 3)
            ok = np.isfinite(pm).all(axis=1)
            if not ok.any():
                break
            corners_m.append(pm[ok].mean(axis=0))
            corners_t.append(pt[ok].mean(axis=0))
        if len(corners_m) < 4:
            continue
        vv, uu = np.mgrid[cv - half:cv + half + 1, cu - half:cu + half + 1]
        core = ((uu - bu) ** 2 + (vv - bv) ** 2 <= r_core ** 2) & np.isfinite(xyz[vv, uu]).all(axis=-1)
        cand = np.flatnonzero(core)
        if cand.size == 0:
            continue
        pick = rng.choice(cand, size=min(n_points, cand.size), replace=False)
        pv, pu = vv.ravel()[pick], uu.ravel()[pick]
        hm = point_plane_distance(plane_through(np.array(corners_m)), xyz[pv, pu])
        ht = point_plane_distance(plane_through(np.array(corners_t)), gt[pv, pu])
        # the two normals may point opposite ways: compare heights with the true sign
        hm = hm * np.sign(hm @ ht) if np.any(hm * ht) else hm
        errs.append(np.abs(hm - ht) * 1e3)
        heights.append(np.abs(ht).max() * 1e3)
        used += 1
    if not errs:
        return {"bumps_used": 0}
    e = np.concatenate(errs)
    return {"bumps_used": used, "points": int(e.size), "mean_abs_err_mm": round(float(e.mean()), 3),
            "rms_err_mm": round(float(np.sqrt((e ** 2).mean())), 3), "max_err_mm": round(float(e.max()), 3),
            "bump_height_range_mm": [round(float(min(heights)), 2), round(float(max(heights)), 2)]}
