"""FP64 oracle of restricted-search aggregation, the paper's proposed speed-up
(Sec. IV, future work): bilateral filtering only on the disparities around an
already calculated disparity, instead of on the whole cost volume.

TEST INFRASTRUCTURE ONLY (see oracle/stereo.py): used by tests and the benchmark's
CPU-baseline leg, never by the library.

Reading (Sec. IV states the idea only):
  * the calculated disparity of a pixel is the winner-take-all of its unaggregated
    correlation, c(p, d) of Eq. 3-5, with the WTA rule of Sec. II-B.3 (highest value,
    ties to the lowest d); for the target view, of the target volume;
  * the search window of a pixel is width = min(2 radius + 1, D) consecutive
    disparities centred on it, moved inward where it would leave [0, D);
  * the aggregated cost of Eq. 8-10 is evaluated only in the window (plus d - 1 and
    d + 1 of the winner, for Eq. 12), so wherever it is evaluated it equals the full
    method's value; the winner is the first maximum inside the window;
  * the left-right check (Eq. 11), Eq. 12 on the reference values and the
    post-processing are those of the full method, applied to the restricted winners;
    Eq. 12 fits a parabola through a discrete maximum, so a winner at a window edge
    whose neighbour just outside the window is larger stays unrefined (the full
    method's winner is the maximum of the whole range and never meets this case).
"""
from __future__ import annotations

import numpy as np

from . import stereo as S


def search_windows(coarse: np.ndarray, D: int, radius: int):
    """First disparity and width of each pixel's window: width = min(2 radius + 1, D),
    lo = clip(coarse - radius, 0, D - width)."""
    width = min(2 * int(radius) + 1, int(D))
    lo = np.clip(np.asarray(coarse, np.int64) - int(radius), 0, int(D) - width)
    return lo, width


def windowed_wta(A: np.ndarray, lo: np.ndarray, width: int) -> np.ndarray:
    """Winner-take-all inside each pixel's window [lo, lo + width): the first maximum
    of A over those d (Sec. II-B.3's rule restricted to the window)."""
    D, H, W = A.shape
    d = np.arange(D)[:, None, None]
    inside = (d >= lo[None]) & (d < lo[None] + width)
    masked = np.where(inside, A, -np.inf)
    return np.argmax(masked, axis=0).astype(np.int64)


def subpixel_at_maximum(A: np.ndarray, disp: np.ndarray) -> np.ndarray:
    """Eq. 12 (S.subpixel) where the winner is a maximum of its two neighbours; the
    winner itself where a neighbour is larger."""
    D, H, W = A.shape
    v, u = np.mgrid[0:H, 0:W]
    c0 = A[disp, v, u]
    higher = (A[np.clip(disp - 1, 0, D - 1), v, u] > c0) | (A[np.clip(disp + 1, 0, D - 1), v, u] > c0)
    with np.errstate(divide="ignore", invalid="ignore"):   # Eq. 12's value is discarded there
        fit = S.subpixel(A, disp)
    return np.where(higher, disp.astype(np.float64), fit)


def reconstruct_restricted(left, right, plane, D, block_radius, agg_radius, gamma_d, gamma_r,
                           lr_threshold, sigma_min, radius):
    """Warp -> both cost volumes -> calculated (unaggregated WTA) disparities -> the
    aggregation in each pixel's window -> windowed WTA on both volumes -> Eq. 11 ->
    Eq. 12 -> post-processing.  The aggregated volumes are computed in full here (the
    values inside the windows are the same numbers); returns every stage."""
    Wp = S.warp(right, plane)
    CL, CR = S.cost_volumes(left, Wp, D, block_radius, sigma_min)
    coarse_ref = S.wta(CL)[0]
    coarse_tar = S.wta(CR)[0]
    AL = S.aggregate_volume(CL, left, agg_radius, gamma_d, gamma_r)
    AR = S.aggregate_volume(CR, Wp, agg_radius, gamma_d, gamma_r)
    lo_ref, width = search_windows(coarse_ref, D, radius)
    lo_tar, _ = search_windows(coarse_tar, D, radius)
    dref = windowed_wta(AL, lo_ref, width)
    dtar = windowed_wta(AR, lo_tar, width)
    valid = S.lr_check(dref, dtar, lr_threshold)
    dsub = subpixel_at_maximum(AL, dref)
    dfin = S.postprocess(dsub, plane)
    return dict(warped=Wp, cost_ref=CL, cost_tar=CR, coarse_ref=coarse_ref, coarse_tar=coarse_tar,
                agg_ref=AL, agg_tar=AR, lo_ref=lo_ref, lo_tar=lo_tar, width=width, disp_ref=dref,
                disp_tar=dtar, valid=valid, disp_sub=dsub, disp_final=dfin)
