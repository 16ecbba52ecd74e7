"""The Sec. III accuracy measurement (paper_1807_07433_amd/accuracy.py) on the CPU:
plane through corner points, point-to-plane distances, the triangulation, and the
whole study against a reconstruction with planted, known height errors."""
import numpy as np

import synth
from paper_1807_07433_amd import accuracy as ACC


def test_plane_through_coplanar_corners_is_exact():
    rng = np.random.default_rng(1)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    c = -0.7
    a, b = np.cross(n, [1.0, 0, 0]), None
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    pts = np.array([x * a + y * b - c * n for x, y in ((-1, -1), (2, -1), (-1, 3), (2, 3))])
    pl = ACC.plane_through(pts)
    assert abs(np.linalg.norm(pl[:3]) - 1.0) < 1e-12
    assert np.abs(ACC.point_plane_distance(pl, pts)).max() < 1e-12
    # a point t along the normal is at distance t (up to the plane's orientation)
    q = pts[0] + 0.123 * n
    assert abs(abs(ACC.point_plane_distance(pl, q)) - 0.123) < 1e-12


def test_triangulation_closed_form():
    d = np.array([[10.0, 20.0], [40.0, -1.0]])
    xyz = ACC.triangulate(d, (700.0, 0.12, 0.5, 0.5))
    assert abs(xyz[0, 0, 2] - 700 * 0.12 / 10) < 1e-12
    assert abs(xyz[1, 0, 0] - (0 - 0.5) * xyz[1, 0, 2] / 700) < 1e-12
    assert np.isnan(xyz[1, 1]).all()


def test_study_measures_planted_height_errors():
    """A reconstruction equal to the ground truth has zero error; moving the sampled
    bump points by t along their region's plane normal gives an error of t."""
    case = synth.road1280_d64()
    cam = (case.camera.f, case.camera.baseline, case.camera.u0, case.camera.v0)
    gt = ACC.triangulate(case.pair.disp_gt, cam)
    bumps = case.pair.extra["bumps"]
    r = ACC.bump_study(gt, case.pair.disp_gt, cam, bumps, np.random.default_rng(0))
    assert r["bumps_used"] >= 6 and r["max_err_mm"] < 1e-6
    # bumps of +-3 px at these depths are centimetres high
    assert 5.0 < r["bump_height_range_mm"][1] < 500.0
    # shift every point inside each bump's core by 2 mm along the local ground normal
    moved = gt.copy()
    for (bu, bv, amp) in bumps:
        cu, cv = int(round(bu)), int(round(bv))
        if not (38 <= cu < 1280 - 38 and 38 <= cv < 720 - 38):
            continue
        corners = [gt[cv + dv - 1:cv + dv + 2, cu + du - 1:cu + du + 2].reshape(-1, 3).mean(0)
                   for du, dv in ((-30, -30), (30, -30), (-30, 30), (30, 30))]
        n = ACC.plane_through(np.array(corners))[:3]
        vv, uu = np.mgrid[cv - 30:cv + 31, cu - 30:cu + 31]
        core = (uu - bu) ** 2 + (vv - bv) ** 2 <= (10 * np.sqrt(2 * np.log(2))) ** 2
        moved[vv[core], uu[core]] += 0.002 * n
    r2 = ACC.bump_study(moved, case.pair.disp_gt, cam, bumps, np.random.default_rng(0))
    assert r2["bumps_used"] == r["bumps_used"]
    assert abs(r2["mean_abs_err_mm"] - 2.0) < 1e-6 and abs(r2["max_err_mm"] - 2.0) < 1e-6
