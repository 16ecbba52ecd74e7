"""GPU parity of the restricted search (Sec. IV): rsv_cost_argmax, and the target
argmax and the reference selection aggregated only in each pixel's window, against
oracle/restricted.py; the full-range identity; and, at 1280x720, agreement with the
full method wherever its winner lies inside the window.

Bars (tests/parity.py): calculated disparities as integer maps (near-ties of the
unaggregated cost); where a pixel's calculated disparity agrees with the oracle's
(same window), its restricted winner >= 99.9 % identical, every mismatch a near-tie of
the oracle's values in that window; subpixel and validity as for the full method."""
import numpy as np
import pytest
import torch

import synth
from oracle import restricted as RS
from oracle import stereo as S
from tests import parity as P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _camera(case):
    c = case.camera
    return (c.f, c.baseline, c.u0, c.v0)


CASES = [
    # H, W, D, block_radius, agg_radius, seed, radius
    (37, 150, 31, 3, 4, 31, 3),
    (70, 201, 64, 3, 5, 32, 4),
    (45, 133, 40, 2, 2, 33, 8),
    (29, 97, 17, 1, 1, 34, 0),
    (24, 70, 9, 4, 3, 35, 2),
]


@pytest.mark.parametrize("H,W,D,r,rho,seed,radius", CASES)
def test_restricted_against_oracle(rsv_gpu, H, W, D, r, rho, seed, radius):
    rsv = rsv_gpu
    case = synth.small_case(H, W, D, r, rho, seed)
    p, prm = case.pair, case.params
    _say(f"[restricted] H={H} W={W} D={D} r={r} rho={rho} seed={seed} radius={radius}")
    ref = RS.reconstruct_restricted(p.left, p.right, case.plane.as_tuple(), D, r, rho, prm.gamma_d, prm.gamma_r,
                                    prm.lr_threshold, prm.sigma_min, radius)
    out = rsv.reconstruct_restricted(_gpu(p.left), _gpu(p.right), case.plane, _camera(case), prm, radius)
    torch.cuda.synchronize()
    v, u = np.mgrid[0:H, 0:W]
    CL, CR, AL, AR = ref["cost_ref"], ref["cost_tar"], ref["agg_ref"], ref["agg_tar"]
    cc = {}
    for tag, C in (("coarse_ref", CL), ("coarse_tar", CR)):
        g = P.to_np(out[tag]).astype(np.int64)
        P.check_disparity(tag, g, ref[tag], C[g, v, u], C.max(0))
        cc[tag] = g == ref[tag]
    width = ref["width"]
    for tag, A, lo, m in (("disp_ref", AL, ref["lo_ref"], cc["coarse_ref"]),
                          ("disp_tar", AR, ref["lo_tar"], cc["coarse_tar"])):
        g = P.to_np(out[tag]).astype(np.int64)
        inside = (g >= lo) & (g < lo + width)
        assert inside[m].all(), f"{tag}: a winner outside its window"
        best = A[ref[tag], v, u]
        frac, nmis = P.check_disparity(tag, g[m], ref[tag][m], A[g, v, u][m], best[m])
        _say(f"  {tag}: {nmis} mismatches where the windows agree ({int((~m).sum())} pixels with another "
             f"calculated disparity, near-ties of the raw cost)")
    dref = P.to_np(out["disp_ref"]).astype(np.int64)
    dtar = P.to_np(out["disp_tar"]).astype(np.int64)
    agree = (dref == ref["disp_ref"]) & cc["coarse_ref"]
    dm = np.clip(ref["disp_ref"] - 1, 0, D - 1)
    dp = np.clip(ref["disp_ref"] + 1, 0, D - 1)
    am, a0, ap = AL[dm, v, u], AL[ref["disp_ref"], v, u], AL[dp, v, u]
    # whether Eq. 12 applies (a discrete maximum) is decided from float values on the
    # GPU: pixels whose neighbour is within a near-tie of the winner are not compared
    near = (np.abs(am - a0) <= P.TIE) | (np.abs(ap - a0) <= P.TIE)
    at_max = (am <= a0) & (ap <= a0)
    inner = agree & (ref["disp_ref"] > 0) & (ref["disp_ref"] < D - 1) & ~near
    P.check_subpixel("disp_sub", P.to_np(out["disp_sub"]), ref["disp_sub"], inner & at_max,
                     np.where(inner & at_max, 2 * am + 2 * ap - 4 * a0, -1.0), 2.5e-6)
    flat = inner & ~at_max
    assert np.array_equal(P.to_np(out["disp_sub"])[flat], ref["disp_sub"][flat].astype(np.float32))
    _say(f"  disp_sub: {int((inner & ~at_max).sum())} window-edge winners left unrefined, {int((agree & near).sum())} "
         f"near-tie neighbours not compared")
    P.check_subpixel_range("disp_sub", P.to_np(out["disp_sub"]), dref)
    x = np.clip(u - ref["disp_ref"], 0, W - 1)
    m = agree & ((dtar == ref["disp_tar"]) & cc["coarse_tar"])[v, x]
    assert np.array_equal(P.to_np(out["valid"]).astype(bool)[m], ref["valid"][m])


@pytest.mark.parametrize("H,W,D,r,rho,seed", [(40, 150, 48, 3, 5, 41), (33, 90, 20, 2, 3, 42)])
def test_full_range_window_equals_full_method_bitwise(rsv_gpu, H, W, D, r, rho, seed):
    """radius >= D - 1: every window is the whole range, and the restricted kernels
    produce the fused full path's outputs bit for bit."""
    rsv = rsv_gpu
    case = synth.small_case(H, W, D, r, rho, seed)
    L, R = _gpu(case.pair.left), _gpu(case.pair.right)
    _say(f"[restricted] full-range window H={H} W={W} D={D}")
    full = rsv.reconstruct(L, R, case.plane, _camera(case), case.params, tar_volume=False, ref_volume=False)
    res = rsv.reconstruct_restricted(L, R, case.plane, _camera(case), case.params, D)
    for k in ("disp_ref", "disp_tar", "disp_sub", "valid", "disp_final"):
        assert torch.equal(res[k].nan_to_num(), full[k].nan_to_num()), k


@pytest.mark.parametrize("H,W,D,r,rho,seed,radius", CASES)
def test_two_view_launch_equals_two_launches(rsv_gpu, H, W, D, r, rho, seed, radius):
    """rsv_aggregate_restricted_views + rsv_lr_check give the outputs of
    rsv_aggregate_restricted_argmax followed by rsv_aggregate_restricted_select, bit
    for bit (u8 left image; and float32 images)."""
    rsv = rsv_gpu
    case = synth.small_case(H, W, D, r, rho, seed)
    prm = case.params
    for L, R in ((_gpu(case.pair.left), _gpu(case.pair.right)),
                 (_gpu(case.pair.left.astype(np.float32)), _gpu(case.pair.right.astype(np.float32)))):
        _say(f"[restricted] two-view launch H={H} W={W} D={D} radius={radius} {L.dtype}")
        wp = rsv.warp(R, case.plane)
        cref, ctar = rsv.joint_views(rsv.cost_volume_joint(L, wp, prm), W)
        cc_ref, cc_tar = rsv.cost_argmax(cref), rsv.cost_argmax(ctar)
        dtar = rsv.aggregate_restricted_argmax(ctar, wp, prm, cc_tar, radius)
        sel = rsv.aggregate_restricted_select(cref, L, prm, cc_ref, radius, dtar)
        vw = rsv.aggregate_restricted_views(cref, ctar, L, wp, prm, cc_ref, cc_tar, radius)
        assert torch.equal(vw["disp_tar"], dtar)
        for k in ("disp_ref", "disp_sub"):
            assert torch.equal(vw[k], sel[k]), k
        assert torch.equal(rsv.lr_check(vw["disp_ref"], vw["disp_tar"], prm.lr_threshold), sel["valid"])


@pytest.mark.parametrize("H,W,D,seed", [(1, 1, 1, 1), (9, 33, 17, 2), (37, 150, 31, 3), (20, 70, 64, 4)])
def test_calculated_disparities_of_both_views_in_one_pass(rsv_gpu, H, W, D, seed):
    """rsv_cost_argmax_views equals two rsv_cost_argmax calls bit for bit, on the
    joint volume's views and on two dense volumes; with ties (a flat volume) and NaN."""
    rsv = rsv_gpu
    case = synth.small_case(max(H, 7), max(W, 7), D, 3, 2, seed)
    L, R = _gpu(case.pair.left), _gpu(case.pair.right)
    wp = rsv.warp(R, case.plane)
    jref, jtar = rsv.joint_views(rsv.cost_volume_joint(L, wp, case.params), L.shape[1])
    rng = np.random.default_rng(seed)
    dense = torch.from_numpy(rng.standard_normal((2, D, H, W)).astype(np.float32)).cuda()
    dense[0, :, 0, :] = 0.25                      # a row of ties
    dense[1, D // 2, :, 0] = float("nan")         # NaN ranks below every number
    _say(f"[restricted] calculated disparities of both views H={H} W={W} D={D}")
    for a, b in ((jref, jtar), (dense[0], dense[1])):
        cr, ct = rsv.cost_argmax_views(a, b)
        assert torch.equal(cr, rsv.cost_argmax(a)) and torch.equal(ct, rsv.cost_argmax(b))


def test_road1280_d64_agrees_with_full_inside_windows(rsv_gpu):
    """1280x720, D = 64: wherever the full method's winner lies inside the pixel's
    window, the restricted winner is the same (the window's values are the same
    floats), and then so are Eq. 12 and, where the looked-up target pixel also agrees,
    Eq. 11.  Also reports the agreement with the full method per radius."""
    rsv = rsv_gpu
    case = synth.road1280_d64()
    L, R = _gpu(case.pair.left), _gpu(case.pair.right)
    prm = case.params
    H, W = case.pair.left.shape
    full = rsv.reconstruct(L, R, case.plane, _camera(case), prm, tar_volume=False, ref_volume=False)
    fd, ft = full["disp_ref"], full["disp_tar"]
    for radius in (2, 4, 8):
        res = rsv.reconstruct_restricted(L, R, case.plane, _camera(case), prm, radius)
        width = min(2 * radius + 1, prm.D)
        ok = {}
        for tag, fm, cc in (("disp_ref", fd, res["coarse_ref"]), ("disp_tar", ft, res["coarse_tar"])):
            lo = (cc - radius).clamp(0, prm.D - width)
            inside = (fm >= lo) & (fm < lo + width)
            same = res[tag] == fm
            assert bool(same[inside].all()), f"{tag}: differs from the full winner inside its window"
            ok[tag] = inside
            _say(f"  radius {radius}: {tag} {float(same.float().mean()) * 100:.3f} % equal to the full method "
                 f"({float(inside.float().mean()) * 100:.3f} % of full winners inside the window)")
        m = ok["disp_ref"]
        assert torch.equal(res["disp_sub"][m], full["disp_sub"][m])
        x = (torch.arange(W, device="cuda")[None, :] - fd).clamp(0, W - 1)
        mv = m & torch.gather(ok["disp_tar"], 1, x.long())
        assert torch.equal(res["valid"][mv], full["valid"][mv])
