"""Comparison rules shared by the GPU parity tests (no arithmetic of the method).

Tolerances (written here once, used by every parity test):
  * warped image and cost volumes: |gpu - oracle| <= 1e-4 on every entry;
  * aggregated volumes: <= 1e-4 on every entry;
  * integer disparities: >= 99.9 % identical, and every mismatch must be a near-tie in
    the oracle: the oracle's value at the GPU's d lies within TIE of its best;
  * subpixel disparity: <= 1e-3 px where the integer disparity agrees and the parabola's
    denominator |2a(d-1) + 2a(d+1) - 4a(d)| >= 1e-2; below that Eq. 12 amplifies an error
    e of the aggregated values to at most 6 e / |den|, which is the bound used there;
  * valid mask: identical wherever the pixel and the column it looks up agree on d.
"""
import numpy as np

COST_TOL = 1e-4
AGG_TOL = 1e-4
TIE = 1e-5
SUB_TOL = 1e-3
DEN_EXEMPT = 1e-2


def to_np(t):
    return t.detach().cpu().numpy()


def check_close(name, gpu, ref, tol):
    gpu = np.asarray(gpu, np.float64)
    err = np.abs(gpu - ref)
    worst = float(err.max()) if err.size else 0.0
    assert np.all(np.isfinite(gpu)), f"{name}: non-finite GPU values"
    assert worst <= tol, f"{name}: max |gpu - oracle| = {worst:.3e} > {tol:.1e}"
    return worst


def check_disparity(name, gpu_d, ref_d, ref_vals_at_gpu_d, ref_best, min_agree=0.999):
    """gpu_d, ref_d: integer maps; ref_vals_at_gpu_d: the oracle's aggregated value at the
    GPU's chosen d for each pixel; ref_best: the oracle's best value."""
    gpu_d = np.asarray(gpu_d)
    ref_d = np.asarray(ref_d)
    same = gpu_d == ref_d
    frac = float(same.mean()) if same.size else 1.0
    assert frac >= min_agree, f"{name}: only {frac:.5f} of integer disparities agree"
    gap = np.abs(np.asarray(ref_best) - np.asarray(ref_vals_at_gpu_d))[~same]
    assert np.all(gap <= TIE), f"{name}: mismatch with oracle gap {gap.max():.3e} > {TIE}"
    return frac, int((~same).sum())


def check_subpixel(name, gpu_sub, ref_sub, agree, den, agg_err=AGG_TOL):
    """<= SUB_TOL wherever |den| >= DEN_EXEMPT.  Where |den| is smaller, Eq. 12 amplifies
    an error e in the aggregated values to at most 6 e / |den| (first-order bound with
    the offset in [-1/2, 1/2]); such pixels must meet max(SUB_TOL, 6 agg_err / |den|)."""
    gpu_sub = np.asarray(gpu_sub, np.float64)
    den = np.abs(np.asarray(den, np.float64))
    err = np.abs(gpu_sub - ref_sub)
    normal = agree & (den >= DEN_EXEMPT)
    small = agree & (den < DEN_EXEMPT)
    worst = float(err[normal].max()) if normal.any() else 0.0
    assert worst <= SUB_TOL, f"{name}: subpixel error {worst:.3e} > {SUB_TOL}"
    if small.any():
        bound = np.maximum(SUB_TOL, 6.0 * agg_err / np.maximum(den[small], 1e-30))
        bad = err[small] > bound
        assert not bad.any(), f"{name}: {bad.sum()} small-denominator pixels beyond 6e/|den|"
    return worst, int(small.sum())


def check_subpixel_range(name, gpu_sub, gpu_disp):
    """Eq. 12 at a discrete maximum puts the parabola's vertex within half a pixel of
    the winner, at every pixel and at any size: the refined map is finite and
    |d_s - d| <= 1/2."""
    sub = np.asarray(gpu_sub, np.float64)
    d = np.asarray(gpu_disp, np.float64)
    assert np.isfinite(sub).all(), f"{name}: {int((~np.isfinite(sub)).sum())} non-finite values"
    off = np.abs(sub - d)
    assert off.max(initial=0.0) <= 0.5, f"{name}: |d_s - d| reaches {off.max():.6g}"
