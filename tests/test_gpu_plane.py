"""GPU parity of the road-plane estimation (rsv_plane_ransac, Sec. II-A) against the
FP64 oracle (oracle/plane.py) on the same seeded maps and draws.

Bars: inlier counts identical per hypothesis except for pixels whose oracle residual
lies within 1e-9 of the threshold (the two sides solve the 3-point planes in different
rounding orders); the best hypothesis and its count identical; the refitted plane
within 1e-9 relative (FP64 least squares on both sides, different summation orders);
degenerate and out-of-range draws score -1 on both; with no hypothesis left the plane
is NaN on both.  At 1280x720 (the road's ground truth plus a roll term, noise,
outliers and holes) the same bars, and the plane recovered from the GPU's own
reconstruction of the synthetic road is the road's plane.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import plane as PL
from tests.test_gpu_parity import _camera, _gpu, _say

pytestmark = pytest.mark.gpu

NEAR = 1e-9


def _near_threshold(disp, valid, samples, threshold):
    """Per hypothesis, the valid pixels whose oracle residual is within NEAR of the
    threshold (either side may count them)."""
    H, W = disp.shape
    d = disp.astype(np.float64)
    vv, uu = np.mgrid[0:H, 0:W]
    ok = valid.astype(bool)
    near = np.zeros(len(samples), np.int64)
    for k, s in enumerate(samples.astype(np.int64)):
        if np.any((s < 0) | (s >= H * W)):
            continue
        sv, su = s // W, s % W
        pl = PL.plane_through_three(su, sv, d[sv, su])
        if pl is None:
            continue
        r = np.abs(d[ok] - (pl[0] + pl[1] * vv[ok] + pl[2] * uu[ok]))
        near[k] = int((np.abs(r - threshold) <= NEAR).sum())
    return near


def _run(rsv, disp, valid, samples, threshold):
    out = rsv.plane_ransac(_gpu(disp), _gpu(valid), _gpu(samples), threshold)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _compare(tag, rsv, disp, valid, samples, threshold):
    g = _run(rsv, disp, valid, samples, threshold)
    plane, counts, best, inl = PL.ransac_plane(disp.astype(np.float64), valid.astype(bool), samples, threshold)
    near = _near_threshold(disp, valid, samples, threshold)
    diff = np.abs(g["counts"].astype(np.int64) - counts)
    _say(f"  {tag}: K={len(samples)} best {best} ({counts[best]} inliers), "
         f"{int((diff > 0).sum())} hypotheses with different counts, {int(near.sum())} near-threshold pixels")
    assert np.array_equal(g["counts"] < 0, counts < 0), f"{tag}: degenerate hypotheses differ"
    assert np.all(diff <= near), f"{tag}: count differences beyond the near-threshold pixels"
    if near.sum() == 0:
        assert np.array_equal(g["counts"], counts)
        assert int(g["best"][0]) == best
    assert counts[int(g["best"][0])] >= counts.max() - near.max()
    if counts[best] < 0:
        assert np.isnan(g["plane"]).all()
        return g, plane
    if near[best] == 0 and int(g["best"][0]) == best:
        assert int(g["best"][1]) == int(inl.sum())
        scale = np.array([max(abs(plane[0]), 1.0), max(abs(plane[1]), 1e-3), max(abs(plane[2]), 1e-3)])
        err = np.abs(g["plane"] - plane) / scale
        _say(f"  {tag}: plane {g['plane']} vs oracle {plane}, worst relative error {err.max():.1e}")
        assert err.max() < 1e-9
    return g, plane


@pytest.mark.parametrize("H,W,K,seed", [(37, 101, 7, 1), (120, 200, 64, 2), (64, 64, 300, 3), (3, 700, 40, 4)])
def test_plane_ransac_matches_oracle(rsv_gpu, H, W, K, seed):
    """Ragged sizes (blocks of 1024 pixels with a tail, K beyond one block of 256
    hypotheses), with a collinear draw, an out-of-range draw and a repeated draw."""
    disp, valid, samples = synth.plane_fit_input(H, W, seed, n_draws=K)
    samples = samples.copy()
    samples[0] = [0, 1, 2]                        # three pixels of row 0: collinear
    if K > 3:
        samples[3] = [0, 5, H * W]                # outside the image
    if K > 6:
        samples[6] = samples[2]                   # a repeat: equal counts
    _say(f"[plane] {W}x{H} K={K} seed={seed}")
    g, _ = _compare(f"{W}x{H}", rsv_gpu, disp, valid, samples, 0.25)
    assert g["counts"][0] == -1
    if K > 6:
        assert g["counts"][6] == g["counts"][2]


def test_plane_ransac_ties_and_degenerate(rsv_gpu):
    H, W = 10, 10
    v, u = np.mgrid[0:H, 0:W]
    disp = (1.0 + 0.5 * v + 0.25 * u).astype(np.float32)
    valid = np.ones((H, W), np.uint8)
    collinear, good = [0, 11, 22], [0, 5, 73]
    _say("[plane] ties to the lowest hypothesis; degenerate draws")
    g = _run(rsv_gpu, disp, valid, np.array([collinear, good, good], np.int32), 0.1)
    assert list(g["counts"]) == [-1, H * W, H * W] and list(g["best"]) == [1, H * W]
    assert np.allclose(g["plane"], [1.0, 0.5, 0.25], atol=1e-12)
    g = _run(rsv_gpu, disp, valid, np.array([collinear, [0, 1, H * W], [-1, 2, 3]], np.int32), 0.1)
    assert list(g["counts"]) == [-1, -1, -1] and np.isnan(g["plane"]).all()
    # a single row: every draw is collinear
    disp1, valid1, s1 = synth.plane_fit_input(1, 1500, 5, n_draws=16)
    g = _run(rsv_gpu, disp1, valid1, s1, 0.25)
    assert (g["counts"] == -1).all() and np.isnan(g["plane"]).all()


def test_plane_ransac_road1280(rsv_gpu):
    """The 1280x720 road's ground-truth disparities (plane 0.15 v + 10 with bumps) plus
    a roll term -0.004 u, N(0, 0.1) noise, 20 % outliers and 10 % holes, 512 draws."""
    case = synth.road1280_d64()
    disp, valid, samples = synth.plane_fit_input(720, 1280, 11, plane=(0.0, 0.0, -0.004), noise=0.1,
                                                 outliers=0.2, holes=0.1, n_draws=512, base=case.pair.disp_gt)
    _say("[plane] 1280x720, K=512")
    g, plane = _compare("road1280", rsv_gpu, disp, valid, samples, 0.5)
    assert np.allclose(g["plane"], [10.0, 0.15, -0.004], atol=[0.05, 2e-4, 2e-4])
    gamma = PL.roll_angle(g["plane"])
    _say(f"  roll {gamma:.5f} rad (the map's: {np.arctan(0.004 / 0.15):.5f})")
    assert abs(gamma - np.arctan(0.004 / 0.15)) < 2e-3


def test_plane_from_gpu_reconstruction_road1280(rsv_gpu):
    """Property at full size: RANSAC over the GPU's post-processed disparities of the
    synthetic road (valid pixels only) recovers the road's plane d = 0.15 v + 10 with no
    roll; the bumps and mismatches are the outliers."""
    rsv = rsv_gpu
    case = synth.road1280_d64()
    out = rsv.reconstruct(_gpu(case.pair.left), _gpu(case.pair.right), case.plane, _camera(case), case.params,
                          tar_volume=False, ref_volume=False)
    valid = out["valid"].cpu().numpy()
    samples = synth.ransac_draws(valid, 512, np.random.default_rng(3))
    res = rsv.plane_ransac(out["disp_final"].contiguous(), out["valid"].contiguous(), _gpu(samples), 0.5)
    torch.cuda.synchronize()
    pl = res["plane"].cpu().numpy()
    _say(f"[plane] from the GPU reconstruction: {pl}, {int(res['best'][1])} inliers of {int(valid.sum())} valid")
    assert np.allclose(pl, [10.0, 0.15, 0.0], atol=[0.05, 2e-4, 2e-4])
    assert abs(PL.roll_angle(pl)) < 2e-3
