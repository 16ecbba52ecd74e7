"""Full-frame GPU parity against the FP64 oracle.

* road320_d32 (320x180 uint8, D = 32, NCC 7x7, bilateral 9x9): the oracle runs the
  whole frame in the test, and every entry of every stage is compared: warped image,
  both cost volumes, both aggregated volumes, both integer maps, validity, subpixel
  and the post-processed disparity and 3-D points; the fused forms must equal the
  volume path bit for bit.
* road1280_d64 (1280x720 uint8, D = 64, NCC 7x7, bilateral 11x11), in the form the
  benchmark times (joint cost volume, target argmax, selection folded into the
  reference aggregation): every pixel of disp_ref, disp_tar, valid and disp_sub
  against the oracle's maps, which tests/golden/make_oracle_maps.py writes from
  oracle/ and synth/ only.  Integer mismatches are re-checked with oracle columns
  computed in the test (each must be a near-tie).

Bars (tests/parity.py): >= 99.9 % identical integer disparities, every mismatch an
oracle near-tie (within 1e-5 of the best); subpixel within 1e-3 px where the integer
disparity agrees and |den| >= 1e-2 (6 e / |den| below, e the measured aggregation
error); validity identical wherever the pixel and the column it looks up agree.
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import stereo as S
from tests import parity as P
from tests.golden.make_oracle_maps import pair_digest
from tests.test_gpu_parity import _agg_columns, _camera, _check_selection, _gpu, _say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_road320_d32_every_entry(rsv_gpu):
    rsv = rsv_gpu
    case = synth.road320_d32()
    p, prm = case.pair, case.params
    H, W = p.left.shape
    _say(f"[full 320] {W}x{H} D={prm.D}: FP64 oracle on the whole frame")
    ref = S.reconstruct(p.left, p.right, case.plane.as_tuple(), _camera(case), prm.D, prm.block_radius,
                        prm.agg_radius, prm.gamma_d, prm.gamma_r, prm.lr_threshold, prm.sigma_min)
    L, R = _gpu(p.left), _gpu(p.right)
    _say("  GPU plain path, both volumes written")
    out = rsv.reconstruct(L, R, case.plane, _camera(case), prm, want_top2=True)
    torch.cuda.synchronize()
    e = {}
    for k, tol in (("warped", P.COST_TOL), ("cost_ref", P.COST_TOL), ("cost_tar", P.COST_TOL),
                   ("agg_ref", P.AGG_TOL), ("agg_tar", P.AGG_TOL)):
        e[k] = P.check_close(k, P.to_np(out[k]), ref[k], tol)
    _say("  max |err| (every entry): " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    agg_err = max(e["agg_ref"], e["agg_tar"], 1e-7)
    _check_selection("road320", out, ref, ref["agg_ref"], ref["agg_tar"], agg_err)
    dref = P.to_np(out["disp_ref"])
    dtar = P.to_np(out["disp_tar"])
    _say(f"  integer mismatches: disp_ref {int((dref != ref['disp_ref']).sum())}, "
         f"disp_tar {int((dtar != ref['disp_tar']).sum())} of {H * W}")
    top2 = P.to_np(out["top2"])
    P.check_close("best", top2[0], ref["best"], P.AGG_TOL)
    P.check_close("second", top2[1], ref["second"], P.AGG_TOL)
    _say("  post-processing and 3-D points on the GPU's subpixel map")
    df_ref = S.postprocess(P.to_np(out["disp_sub"]).astype(np.float64), case.plane.as_tuple())
    P.check_close("disp_final", P.to_np(out["disp_final"]), df_ref, 1e-4)
    xyz_ref = S.triangulate(df_ref, P.to_np(out["valid"]).astype(bool), _camera(case))
    xyz = P.to_np(out["xyz"])
    assert np.array_equal(np.isnan(xyz), np.isnan(xyz_ref))
    ok = ~np.isnan(xyz_ref)
    assert np.allclose(xyz[ok], xyz_ref[ok], rtol=1e-5, atol=1e-6)
    _say("  fused forms (target argmax; selection folded in) == volume path, bit for bit")
    for kw in (dict(tar_volume=False), dict(tar_volume=False, ref_volume=False)):
        f = rsv.reconstruct(L, R, case.plane, _camera(case), prm, **kw)
        for k in ("disp_ref", "disp_tar", "disp_sub", "valid", "disp_final", "xyz"):
            assert torch.equal(f[k].nan_to_num(), out[k].nan_to_num()), (kw, k)


def _near_tie(tag, gpu_d, ref_d, cols, idx):
    """Mismatching pixels idx: the oracle columns must agree with the stored oracle map
    and put the GPU's choice within P.TIE of the best."""
    best = cols.max(1)
    at = cols[np.arange(idx.size), gpu_d]
    assert np.array_equal(cols.argmax(1), ref_d), f"{tag}: oracle columns disagree with the stored maps"
    gap = best - at
    _say(f"  {tag}: {idx.size} mismatches, largest oracle gap {gap.max(initial=0.0):.2e}")
    assert np.all(gap <= P.TIE), f"{tag}: mismatch with oracle gap {gap.max():.3e} > {P.TIE}"


def test_road1280_d64_every_pixel(rsv_gpu):
    rsv = rsv_gpu
    case = synth.road1280_d64()
    p, prm = case.pair, case.params
    H, W = p.left.shape
    D = prm.D
    path = os.path.join(GOLDEN, "road1280_d64_oracle_maps.npz")
    g = np.load(path)
    assert tuple(g["shape"]) == (H, W, D)
    assert str(g["pair_sha256"]) == pair_digest(p.left, p.right), \
        "stored oracle maps belong to another pair: rerun tests/golden/make_oracle_maps.py"
    ref_d = g["disp_ref"].astype(np.int64)
    ref_t = g["disp_tar"].astype(np.int64)
    ref_valid = np.unpackbits(g["valid"])[:H * W].reshape(H, W).astype(bool)
    ref_sub = g["disp_sub"].astype(np.float64)
    den = g["den"].astype(np.float64)

    L, R = _gpu(p.left), _gpu(p.right)
    _say(f"[full 1280] {W}x{H} D={D}: GPU path as timed (joint volume, target argmax, folded selection)")
    out = rsv.reconstruct(L, R, case.plane, _camera(case), prm, tar_volume=False, ref_volume=False)
    torch.cuda.synchronize()
    assert out["agg_ref"] is None
    gd = P.to_np(out["disp_ref"]).astype(np.int64)
    gt = P.to_np(out["disp_tar"]).astype(np.int64)
    gvalid = P.to_np(out["valid"]).astype(bool)
    gsub = P.to_np(out["disp_sub"])

    Wp = S.warp(p.right, case.plane.as_tuple())

    def cl(x, y, d):
        return S.cost_entries(p.left, Wp, x, y, d, prm.block_radius, prm.sigma_min)

    def cr(x, y, d):
        return S.cost_entries(p.left, Wp, x + d, y, d, prm.block_radius, prm.sigma_min)

    for tag, gm, rm, cost_at, guide in (("disp_ref", gd, ref_d, cl, p.left), ("disp_tar", gt, ref_t, cr, Wp)):
        same = gm == rm
        frac = float(same.mean())
        _say(f"  {tag}: {frac * 100:.4f} % of {H * W} pixels identical")
        assert frac >= 0.999, f"{tag}: only {frac:.5f} identical"
        vv, uu = np.nonzero(~same)
        if vv.size:
            cols = _agg_columns(cost_at, guide, uu, vv, D, prm)
            _near_tie(tag, gm[vv, uu], rm[vv, uu], cols, vv)
        else:
            _say(f"  {tag}: 0 mismatches")

    # aggregation error of this build, measured on sampled entries of the volume path
    rng = np.random.default_rng(5)
    n = 1500
    u, v, d = rng.integers(0, W, n), rng.integers(0, H, n), rng.integers(0, D, n)
    jref, _ = rsv.joint_views(rsv.cost_volume_joint(L, rsv.warp(R, case.plane), prm), W)
    aref = rsv.aggregate(jref, L, prm)
    gi = (torch.from_numpy(d).cuda(), torch.from_numpy(v).cuda(), torch.from_numpy(u).cuda())
    a = S.aggregate_entries(cl, p.left, u, v, d, prm.agg_radius, prm.gamma_d, prm.gamma_r)
    agg_err = max(P.check_close("agg_ref (sampled)", P.to_np(aref[gi]), a, P.AGG_TOL), 1e-7)
    del aref, jref

    vv, uu = np.mgrid[0:H, 0:W]
    agree = gd == ref_d
    x = np.clip(uu - ref_d, 0, W - 1)
    m = agree & (gt == ref_t)[vv, x]
    bad_valid = int((gvalid[m] != ref_valid[m]).sum())
    _say(f"  valid: {int(m.sum())} pixels where both lookups agree, {bad_valid} differ; "
         f"{int(gvalid.sum())} valid on the GPU, {int(ref_valid.sum())} in the oracle")
    assert bad_valid == 0
    inner = agree & (ref_d > 0) & (ref_d < D - 1)
    worst, n_small = P.check_subpixel("disp_sub", gsub, ref_sub, inner, np.where(inner, den, -1.0), agg_err)
    _say(f"  disp_sub: worst |err| {worst:.2e} px over {int(inner.sum())} pixels; "
         f"{n_small} small-denominator pixels (|den| < {P.DEN_EXEMPT}) held to 6e/|den| with e = {agg_err:.1e}")
    edge = agree & ~((ref_d > 0) & (ref_d < D - 1))
    assert np.array_equal(gsub[edge], ref_sub[edge].astype(np.float32))
    P.check_subpixel_range("disp_sub (whole frame)", gsub, gd)


def test_road1280_d64_reconstruction_accuracy_mm(rsv_gpu):
    """Sec. III's accuracy measurement on the GPU's 3-D points of the 1280x720 road
    (accuracy.bump_study): every bump region in the image is measured, and the mean
    height error stays at the millimetre level (the oracle's own maps give 2.8 mm)."""
    from paper_1807_07433_amd import accuracy as ACC
    rsv = rsv_gpu
    case = synth.road1280_d64()
    out = rsv.reconstruct(_gpu(case.pair.left), _gpu(case.pair.right), case.plane, _camera(case), case.params,
                          tar_volume=False, ref_volume=False)
    r = ACC.bump_study(P.to_np(out["xyz"]).astype(np.float64), case.pair.disp_gt, _camera(case),
                       case.pair.extra["bumps"], np.random.default_rng(0))
    _say(f"[accuracy] {r}")
    assert r["bumps_used"] >= 6
    assert r["mean_abs_err_mm"] < 4.0
