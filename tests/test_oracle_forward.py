"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Each test names the passage it pins.  None retypes the oracle's own formula: they
use library routines (np.corrcoef, scipy.ndimage), closed forms, invariances,
hand-built cases and a literal brute-force loop on tiny inputs.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import stereo as S

RNG = np.random.default_rng(12345)


# --------------------------------------------------------------------- warp (Sec. II-A)
def test_warp_moves_points_to_the_right():
    """Sec. II-A: the warp moves every point of row v to the right by the shift
    alpha0 + alpha1 v - delta."""
    R = np.zeros((3, 30))
    R[:, 10] = 100.0
    out = S.warp(R, (5.0, 0.0, 0.0, 2.0))  # s = 3
    assert np.argmax(out[1]) == 13 and out[1, 13] == 100.0


def test_warp_integer_shift_is_translation():
    R = RNG.integers(0, 256, (6, 40)).astype(np.uint8)
    out = S.warp(R, (9.0, 0.0, 0.0, 4.0))  # s = 5
    assert np.array_equal(out[:, 5:], R[:, :-5].astype(np.float64))
    assert np.array_equal(out[:, :5], np.repeat(R[:, :1], 5, axis=1).astype(np.float64))


def test_warp_zero_shift_is_identity():
    R = RNG.integers(0, 256, (5, 17)).astype(np.uint8)
    assert np.array_equal(S.warp(R, (3.0, 0.0, 0.0, 3.0)), R.astype(np.float64))


def test_warp_ramp_is_exact_for_fractional_rowwise_shift():
    """Linear interpolation reproduces a linear ramp exactly (reading: linear lerp)."""
    H, W = 8, 50
    R = np.tile(3.0 * np.arange(W) + 7.0, (H, 1))
    plane = (2.25, 0.3, 0.0, 0.0)
    out = S.warp(R, plane)
    v = np.arange(H)[:, None]
    u = np.arange(W)[None, :]
    x = u - (2.25 + 0.3 * v)
    ok = (x >= 0) & (x <= W - 1)
    assert np.allclose(out[ok], (3.0 * x + 7.0)[np.broadcast_to(ok, x.shape)], atol=1e-12)


def test_warp_flat_neighbours_exact():
    R = np.full((4, 12), 77.0)
    out = S.warp(R, (0.37, 0.11, 0.013, 0.0))
    assert np.all(out == 77.0)


# --------------------------------------------------------------------- ZNCC (Eq. 3-5)
def test_zncc_equals_pearson_correlation():
    bl = RNG.normal(size=(50, 49)) * 30 + 100
    br = 0.5 * bl + RNG.normal(size=(50, 49)) * 20
    c = S.zncc(bl, br, 1e-2)
    ref = np.array([np.corrcoef(bl[i], br[i])[0, 1] for i in range(50)])
    assert np.allclose(c, ref, atol=1e-13)


def test_zncc_identical_blocks_is_one_and_bounded():
    bl = RNG.integers(0, 256, (100, 81)).astype(np.float64)
    assert np.allclose(S.zncc(bl, bl, 1e-2), 1.0, atol=1e-14)
    br = RNG.integers(0, 256, (100, 81)).astype(np.float64)
    c = S.zncc(bl, br, 1e-2)
    assert np.all(np.abs(c) <= 1.0 + 1e-15)


def test_zncc_affine_invariance_and_symmetry():
    bl = RNG.normal(size=(20, 49)) * 25 + 120
    br = RNG.normal(size=(20, 49)) * 25 + 120
    c = S.zncc(bl, br, 1e-2)
    assert np.allclose(S.zncc(1.7 * bl - 40, br, 1e-2), c, atol=1e-13)
    assert np.allclose(S.zncc(bl, 0.3 * br + 9, 1e-2), c, atol=1e-13)
    assert np.allclose(S.zncc(-2.0 * bl + 5, br, 1e-2), -c, atol=1e-13)
    assert np.allclose(S.zncc(br, bl, 1e-2), c, atol=1e-14)


def test_zncc_flat_block_is_zero():
    bl = np.full((3, 49), 12.0)
    br = RNG.normal(size=(3, 49))
    assert np.all(S.zncc(bl, br, 1e-2) == 0.0)
    assert np.all(S.zncc(br, bl, 1e-2) == 0.0)


def test_cost_pairs_left_u_with_target_u_minus_d():
    """Eq. 3 pairs i_l(x, y) with i_r(x - d, y): a target that is the reference moved
    k pixels left correlates perfectly at d = k."""
    L = RNG.integers(0, 256, (20, 60)).astype(np.float64)
    k = 4
    T = np.empty_like(L)
    T[:, :-k] = L[:, k:]
    T[:, -k:] = L[:, -1:]
    CL, _ = S.cost_volumes(L, T, 8, 2, 1e-2)
    inner = CL[:, 3:-3, 3 + k:-3 - k]
    assert np.allclose(inner[k], 1.0, atol=1e-12)
    assert np.all(inner[np.arange(8) != k] < 0.999)


def test_target_volume_identity():
    """C_tar(u - d, v, d) = C_ref(u, v, d) (stated after Eq. 5)."""
    L = RNG.integers(0, 256, (11, 23)).astype(np.float64)
    T = RNG.integers(0, 256, (11, 23)).astype(np.float64)
    D = 6
    CL, CR = S.cost_volumes(L, T, D, 1, 1e-2)
    for d in range(D):
        assert np.array_equal(CR[d, :, :23 - d], CL[d, :, d:])


def test_cost_block_values_clamp_to_edge():
    img = np.arange(20, dtype=np.float64).reshape(4, 5)
    b = S.block_values(img, np.array([0]), np.array([0]), 1)[0]
    assert b.tolist() == [0, 0, 1, 0, 0, 1, 5, 5, 6]


# ------------------------------------------------------------ bilateral (Eq. 8-10)
def _brute_force_fbs(C, g, rho, gd, gr):
    D, H, W = C.shape
    A = np.zeros_like(C)
    for d in range(D):
        for v in range(H):
            for u in range(W):
                num = den = 0.0
                for y in range(v - rho, v + rho + 1):
                    for x in range(u - rho, u + rho + 1):
                        if 0 <= x < W and 0 <= y < H:
                            wd = math.exp(-((x - u) ** 2 + (y - v) ** 2) / gd ** 2)
                            wr = math.exp(-((g[y, x] - g[v, u]) / 255.0) ** 2 / gr ** 2)
                            num += wd * wr * C[d, y, x]
                            den += wd * wr
                A[d, v, u] = num / den
    return A


def test_bilateral_brute_force_tiny():
    C = RNG.uniform(-1, 1, (5, 7, 9))
    g = RNG.integers(0, 256, (7, 9)).astype(np.float64)
    A = S.aggregate_volume(C, g, 2, 1.5, 0.2)
    assert np.allclose(A, _brute_force_fbs(C, g, 2, 1.5, 0.2), atol=1e-14)


def test_bilateral_constant_slices_stay_constant():
    C = np.stack([np.full((9, 13), v) for v in (-0.5, 0.25, 0.9)])
    g = RNG.integers(0, 256, (9, 13))
    A = S.aggregate_volume(C, g, 3, 2.0, 0.1)
    for k, v in enumerate((-0.5, 0.25, 0.9)):
        assert np.allclose(A[k], v, atol=1e-15)


def test_bilateral_large_gamma_r_is_normalised_gaussian():
    """gamma_r -> inf leaves the spatial Gaussian of Eq. 9, renormalised at borders."""
    C = RNG.uniform(-1, 1, (3, 12, 15))
    g = RNG.integers(0, 256, (12, 15))
    rho, gd = 3, 2.0
    A = S.aggregate_volume(C, g, rho, gd, 1e9)
    off = np.arange(-rho, rho + 1)
    ker = np.exp(-(off[:, None] ** 2 + off[None, :] ** 2) / gd ** 2)
    ones = ndimage.correlate(np.ones((12, 15)), ker, mode="constant", cval=0.0)
    for d in range(3):
        ref = ndimage.correlate(C[d], ker, mode="constant", cval=0.0) / ones
        assert np.allclose(A[d], ref, atol=1e-12)


def test_bilateral_all_gammas_large_is_box_mean():
    C = RNG.uniform(-1, 1, (2, 10, 11))
    g = RNG.integers(0, 256, (10, 11))
    A = S.aggregate_volume(C, g, 2, 1e9, 1e9)
    ker = np.ones((5, 5))
    cnt = ndimage.correlate(np.ones((10, 11)), ker, mode="constant")
    for d in range(2):
        assert np.allclose(A[d], ndimage.correlate(C[d], ker, mode="constant") / cnt, atol=1e-12)


def test_bilateral_step_edge_does_not_bleed():
    H, W = 10, 20
    g = np.zeros((H, W))
    g[:, 10:] = 200.0
    C = np.zeros((1, H, W))
    C[0, :, 10:] = 1.0
    A = S.aggregate_volume(C, g, 4, 3.0, 0.05)
    assert np.all(A[0, :, :10] < 1e-12)
    assert np.all(A[0, :, 10:] > 1 - 1e-12)


def test_bilateral_range_scale_two_pixel_case():
    """Range term uses intensities/255: a neighbour 25.5 levels away with gamma_r = 0.1
    gets exp(-1) times the spatial weight."""
    C = np.array([[[0.0, 1.0]]])
    g = np.array([[100.0, 125.5]])
    A = S.aggregate_volume(C, g, 1, 2.0, 0.1)
    w = math.exp(-1 / 4.0) * math.exp(-1.0)
    assert abs(A[0, 0, 0] - w / (1 + w)) < 1e-14


def test_bilateral_commutes_with_transpose():
    C = RNG.uniform(-1, 1, (2, 8, 11))
    g = RNG.integers(0, 256, (8, 11)).astype(np.float64)
    A = S.aggregate_volume(C, g, 2, 1.7, 0.3)
    At = S.aggregate_volume(C.transpose(0, 2, 1).copy(), g.T.copy(), 2, 1.7, 0.3)
    assert np.allclose(A, At.transpose(0, 2, 1), atol=1e-14)


def test_aggregate_entries_matches_volume():
    L = RNG.integers(0, 256, (14, 19)).astype(np.float64)
    T = RNG.integers(0, 256, (14, 19)).astype(np.float64)
    CL, _ = S.cost_volumes(L, T, 5, 1, 1e-2)
    A = S.aggregate_volume(CL, L, 2, 2.0, 0.2)
    u = np.array([0, 5, 18, 7])
    v = np.array([0, 13, 6, 7])
    d = np.array([0, 4, 2, 1])
    got = S.aggregate_entries(lambda x, y, dd: S.cost_entries(L, T, x, y, dd, 1, 1e-2),
                              L, u, v, d, 2, 2.0, 0.2)
    assert np.allclose(got, A[d, v, u], atol=1e-14)


# ------------------------------------------------------------------ WTA, L-R, subpixel
def test_wta_hand_cases_and_ties():
    A = np.zeros((4, 1, 3))
    A[:, 0, 0] = [0.1, 0.5, 0.5, 0.2]   # tie -> lowest d
    A[:, 0, 1] = [0.9, 0.1, 0.2, 0.3]
    A[:, 0, 2] = [-0.3, -0.2, -0.1, 0.0]
    disp, best, second = S.wta(A)
    assert disp[0].tolist() == [1, 0, 3]
    assert best[0].tolist() == [0.5, 0.9, 0.0]
    assert second[0].tolist() == [0.5, 0.3, -0.1]


def test_lr_check_hand_cases():
    ref = np.array([[3, 3, 2, 2, 1, 1]])        # matches at x = -3, -2, 0, 1, 3, 4
    tar = np.array([[2, 2, 0, 1, 1, 0]])        # consistent where the match exists
    assert S.lr_check(ref, tar, 0)[0].tolist() == [False, False, True, True, True, True]
    bad = tar.copy()
    bad[0, 1] += 2                              # looked up by u = 3
    assert S.lr_check(ref, bad, 1)[0].tolist() == [False, False, True, False, True, True]
    off = tar.copy()
    off[0, 3] += 1                              # looked up by u = 4
    assert S.lr_check(ref, off, 1)[0].tolist() == [False, False, True, True, True, True]
    assert S.lr_check(ref, off, 0)[0].tolist() == [False, False, True, True, False, True]


def test_subpixel_recovers_quadratic_vertex():
    """Eq. 12 is the vertex of the parabola through the three costs."""
    D = 9
    d = np.arange(D, dtype=np.float64)
    for d0 in (3.0, 3.2, 4.49, 5.77, 1.51):
        for k, b in ((0.3, 0.5), (2.0, -1.0)):
            A = (-k * (d - d0) ** 2 + b)[:, None, None]
            disp, _, _ = S.wta(A)
            ds = S.subpixel(A, disp)
            assert abs(ds[0, 0] - d0) < 1e-12


def test_subpixel_invariant_to_affine_cost_map_and_unrefined_at_ends():
    A = RNG.uniform(-1, 1, (7, 4, 5))
    disp, _, _ = S.wta(A)
    ds = S.subpixel(A, disp)
    assert np.allclose(S.subpixel(3.0 * A - 0.4, disp), ds, atol=1e-12)
    ends = (disp == 0) | (disp == 6)
    assert np.array_equal(ds[ends], disp[ends].astype(np.float64))
    assert np.all(np.abs(ds - disp) <= 0.5 + 1e-12)


# --------------------------------------------------------- post-processing and 3-D
def test_postprocess_inverts_the_warp_map():
    """u - d_f is the target column that the warped column u - d_s displays."""
    H, W = 6, 400
    R = np.tile(np.arange(W, dtype=np.float64), (H, 1))   # column index as intensity
    plane = (120.0, 0.25, 0.02, 16.0)
    Wp = S.warp(R, plane)
    ds = RNG.integers(0, 32, (H, W)).astype(np.float64)
    df = S.postprocess(ds, plane)
    v, u = np.mgrid[0:H, 0:W]
    x = (u - ds).astype(np.int64)
    ok = (x >= 0) & (Wp[v, np.clip(x, 0, W - 1)] > 0) & (Wp[v, np.clip(x, 0, W - 1)] < W - 1)
    assert np.allclose((u - df)[ok], Wp[v, np.clip(x, 0, W - 1)][ok], atol=1e-9)


def test_triangulate_closed_form_and_nan():
    d = np.array([[10.0, 20.0, -1.0, 5.0]])
    valid = np.array([[True, True, True, False]])
    xyz = S.triangulate(d, valid, (700.0, 0.12, 1.5, 0.0))
    assert np.isclose(xyz[0, 0, 2], 700 * 0.12 / 10)
    assert np.isclose(xyz[0, 1, 0], (1 - 1.5) * (700 * 0.12 / 20) / 700)
    assert np.all(np.isnan(xyz[0, 2])) and np.all(np.isnan(xyz[0, 3]))


def test_planar_disparity_triangulates_to_a_plane():
    """Eq. 2: d = a0 + a1 v  =>  f T = (a0 + a1 v0) z + a1 f y for every point."""
    H, W = 40, 60
    a0, a1, f, T, u0, v0 = 12.0, 0.2, 700.0, 0.12, 29.5, 19.5
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    d = a0 + a1 * v
    xyz = S.triangulate(d, np.ones((H, W), bool), (f, T, u0, v0))
    res = (a0 + a1 * v0) * xyz[..., 2] + a1 * f * xyz[..., 1] - f * T
    assert np.max(np.abs(res)) < 1e-12


# ------------------------------------------------------------------ whole pipeline
def _integer_plane_pair(H=40, W=110, b=9, seed=5):
    import synth
    from synth.road import RoadScene, make_pair
    scene = RoadScene(H, W, 0.0, float(b), n_bumps=0, noise_right=0.0)
    return make_pair(scene, seed)


def test_noiseless_integer_plane_recovered_exactly():
    """With the true warp the residual disparity is delta at every interior pixel and
    every interior pixel passes the left-right check."""
    p = _integer_plane_pair()
    D, delta = 12, 6
    out = S.reconstruct(p.left, p.right, (9.0, 0.0, 0.0, float(delta)),
                        (700.0, 0.12, 54.5, 19.5), D, 2, 3, 2.0, 0.1)
    inner = (slice(6, -6), slice(6 + D, -6 - 9 - delta))
    assert np.all(out["disp_ref"][inner] == delta)
    assert np.all(out["valid"][inner])
    assert np.allclose(out["cost_ref"][delta][inner], 1.0, atol=1e-12)
    assert np.all(np.abs(out["disp_final"][inner] - 9.0) < 0.5)


@pytest.mark.slow
def test_fractional_plane_recovers_ground_truth():
    """Accuracy, not parity: on the 320x180 road the post-processed disparity tracks the
    generator's ground truth."""
    import synth
    c = synth.road320_d32()
    p = c.pair
    out = S.reconstruct(p.left, p.right, c.plane.as_tuple(),
                        (700.0, 0.12, 159.5, 89.5), c.params.D, 3, 4, 3.0, 0.1)
    m = out["valid"].copy()
    m[:8], m[-8:], m[:, :40], m[:, -8:] = False, False, False, False
    err = np.abs(out["disp_final"] - p.disp_gt)[m]
    assert m.mean() > 0.6
    assert np.median(err) < 0.25 and np.mean(err < 1.0) > 0.97
