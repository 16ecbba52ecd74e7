"""Pins of the restricted-search oracle (oracle/restricted.py, Sec. IV): facts it must
satisfy independently of its own code."""
import numpy as np

import synth
from oracle import restricted as RS
from oracle import stereo as S


def test_windows_are_centred_and_clamped_into_the_range():
    lo, width = RS.search_windows(np.array([[0, 1, 5, 9, 10, 11]]), 12, 2)
    assert width == 5
    # centred at 5 and 9 -> [3, 8), [7, 12); pushed inward at both ends
    assert lo.tolist() == [[0, 0, 3, 7, 7, 7]]
    lo, width = RS.search_windows(np.array([[3]]), 4, 9)   # wider than the range
    assert width == 4 and lo.tolist() == [[0]]


def test_windowed_wta_brute_force_ties_and_planted_outside_maximum():
    rng = np.random.default_rng(3)
    D, H, W = 11, 4, 5
    A = rng.integers(0, 4, (D, H, W)).astype(np.float64)   # many ties
    coarse = rng.integers(0, D, (H, W))
    lo, width = RS.search_windows(coarse, D, 2)
    got = RS.windowed_wta(A, lo, width)
    for v in range(H):
        for u in range(W):
            seg = [A[d, v, u] for d in range(lo[v, u], lo[v, u] + width)]
            best = max(seg)
            first = next(i for i, x in enumerate(seg) if x == best)
            assert got[v, u] == lo[v, u] + first
    # a larger value outside the window is never chosen
    A2 = A.copy()
    A2[0] = 100.0
    c2 = np.full((H, W), 8)
    lo2, w2 = RS.search_windows(c2, D, 1)
    assert np.all(RS.windowed_wta(A2, lo2, w2) >= 7)


def test_full_window_gives_the_full_method():
    """A radius covering the whole range reduces the restricted search to Sec. II-B."""
    case = synth.small_case(20, 48, 9, 2, 2, 5)
    p, prm = case.pair, case.params
    cam = (700.0, 0.12, 23.5, 9.5)
    full = S.reconstruct(p.left, p.right, case.plane.as_tuple(), cam, prm.D, prm.block_radius, prm.agg_radius,
                         prm.gamma_d, prm.gamma_r, prm.lr_threshold, prm.sigma_min)
    res = RS.reconstruct_restricted(p.left, p.right, case.plane.as_tuple(), prm.D, prm.block_radius,
                                    prm.agg_radius, prm.gamma_d, prm.gamma_r, prm.lr_threshold, prm.sigma_min,
                                    radius=prm.D)
    for k in ("disp_ref", "disp_tar", "valid", "disp_sub"):
        assert np.array_equal(res[k], full[k]), k


def test_agrees_wherever_the_full_winner_is_inside_the_window():
    """For any calculated disparities, a pixel whose full winner lies in its window gets
    that winner (the windowed maximum of the same values)."""
    case = synth.small_case(24, 60, 16, 3, 2, 6)
    p, prm = case.pair, case.params
    res = RS.reconstruct_restricted(p.left, p.right, case.plane.as_tuple(), prm.D, prm.block_radius,
                                    prm.agg_radius, prm.gamma_d, prm.gamma_r, prm.lr_threshold, prm.sigma_min,
                                    radius=3)
    full_d = S.wta(res["agg_ref"])[0]
    inside = (full_d >= res["lo_ref"]) & (full_d < res["lo_ref"] + res["width"])
    assert inside.mean() > 0.5
    assert np.array_equal(res["disp_ref"][inside], full_d[inside])
    # the calculated disparity is the unaggregated volume's first argmax
    assert np.array_equal(res["coarse_ref"], np.argmax(res["cost_ref"], axis=0))


def test_subpixel_only_at_a_discrete_maximum():
    """Eq. 12 through a maximum equals the full method's; next to a larger neighbour the
    winner stays unrefined."""
    A = np.zeros((7, 1, 3))
    A[:, 0, 0] = [0, 1, 3, 2, 0, 0, 0]     # maximum at 2
    A[:, 0, 1] = [0, 1, 2, 5, 4, 0, 0]     # window winner 2, neighbour 3 larger
    A[:, 0, 2] = [9, 8, 7, 6, 5, 4, 3]     # winner 3 inside a descending slope
    d = np.array([[2, 2, 3]])
    got = RS.subpixel_at_maximum(A, d)
    with np.errstate(divide="ignore", invalid="ignore"):  # the slope pixel's Eq. 12 divides by 0
        full = S.subpixel(A, d)
    assert got[0, 0] == full[0, 0] and abs(got[0, 0] - (2 + (1 - 2) / (2 + 4 - 12))) < 1e-12
    assert got[0, 1] == 2.0 and got[0, 2] == 3.0
