"""FP64 oracle of the dense stereo path (forward).

TEST INFRASTRUCTURE ONLY.  This module is a plain, slow, obviously correct CPU
implementation used to check the HIP library.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the library never does.  It
shares no code with the HIP path.

Every function follows a passage of the paper (Fan et al., "Real-Time Stereo
Vision for Road Surface 3-D Reconstruction", arXiv 1807.07433):

  warp               Sec. II-A, last paragraph (row v of the target shifted right by
                     alpha0 + alpha1*v - delta), with the v-d plane of Eq. 2.
  zncc, cost_*       Sec. II-B.1, Eq. 3-5 (zero-mean normalised cross-correlation of
                     (2*rho_b+1)^2 blocks) and the reference/target volume identity
                     stated right after Eq. 5.
  bilateral_*,       Sec. II-B.2, Eq. 8-10 (bilateral cost aggregation).
  aggregate_*
  wta                Sec. II-B.3 (winner-take-all on both aggregated volumes).
  lr_check           Sec. II-B.4, Eq. 11 (left-right consistency / uniqueness).
  subpixel           Sec. II-B.4, Eq. 12 (parabola through three costs).
  postprocess,       Sec. II-C (add the plane shift back) and Sec. II-D (3-D points).
  triangulate

Readings where the paper is silent (each is listed with its reason in the design
notes): linear interpolation along the row with clamp-to-edge for the warp,
written I0 + f*(I1 - I0); a third plane term a2*u (road roll); clamp-to-edge block
reads; correlation defined as 0 when either block's std-dev is below sigma_min;
bilateral taps outside the image skipped and the weights renormalised; range term
on intensities scaled by 1/255 with guide = left image for the reference volume and
the warped target for the target volume; WTA takes the highest correlation with
ties going to the lowest d; the left-right test accepts |difference| <= threshold;
the parabola uses the aggregated reference costs and is skipped at d = 0 and D-1.
"""
from __future__ import annotations

import numpy as np

ROW_CHUNK = 64  # rows processed at once by the full-image drivers (memory bound only)


# ----------------------------------------------------------------------------- warp
def shift_field(plane, height: int, width: int) -> np.ndarray:
    """s(u, v) = a0 + a1*v + a2*u - delta, in pixels (Eq. 2 plus a roll term)."""
    a0, a1, a2, delta = (float(t) for t in plane)
    v, u = np.mgrid[0:height, 0:width].astype(np.float64)
    return a0 + a1 * v + a2 * u - delta


def sample_row_linear(img: np.ndarray, v: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Linear interpolation of image rows v at real columns x, clamp-to-edge."""
    H, W = img.shape
    x = np.clip(x, -2.0, W + 1.0)          # keeps floor() finite; does not change values
    x0 = np.floor(x)
    f = x - x0
    x0 = x0.astype(np.int64)
    i0 = img[v, np.clip(x0, 0, W - 1)].astype(np.float64)
    i1 = img[v, np.clip(x0 + 1, 0, W - 1)].astype(np.float64)
    return i0 + f * (i1 - i0)


def warp(right: np.ndarray, plane) -> np.ndarray:
    """Perspective transformation of the target (right) image into the reference view.

    Each point of row v moves s(u, v) pixels to the right, i.e. the warped image at
    column u shows the target at column u - s(u, v) (Sec. II-A).
    """
    H, W = right.shape
    v, u = np.mgrid[0:H, 0:W]
    s = shift_field(plane, H, W)
    return sample_row_linear(right.astype(np.float64), v, u - s)


# ----------------------------------------------------------------------------- ZNCC
def block_values(img: np.ndarray, u: np.ndarray, v: np.ndarray, r: int) -> np.ndarray:
    """Clamp-to-edge (2r+1)^2 block around each (u, v); returns [..., n] in row-major
    (dy, dx) order."""
    H, W = img.shape
    img = img.astype(np.float64)
    u = np.asarray(u, np.int64)[..., None]
    v = np.asarray(v, np.int64)[..., None]
    offs = np.arange(-r, r + 1)
    dy = np.repeat(offs, 2 * r + 1)
    dx = np.tile(offs, 2 * r + 1)
    return img[np.clip(v + dy, 0, H - 1), np.clip(u + dx, 0, W - 1)]


def zncc(bl: np.ndarray, br: np.ndarray, sigma_min: float) -> np.ndarray:
    """Eq. 3-5: c = (sum l*r - n mu_l mu_r) / (n sigma_l sigma_r), population sigmas.

    Written in the algebraically identical centred form sum (l-mu_l)(r-mu_r) / n, so a
    constant block has sigma exactly 0.  c = 0 when either sigma < sigma_min (the
    paper leaves sigma = 0 undefined).
    """
    n = bl.shape[-1]
    dl = bl - bl.mean(axis=-1, keepdims=True)
    dr = br - br.mean(axis=-1, keepdims=True)
    sl = np.sqrt((dl * dl).sum(axis=-1) / n)
    sr = np.sqrt((dr * dr).sum(axis=-1) / n)
    cov = (dl * dr).sum(axis=-1) / n
    ok = (sl >= sigma_min) & (sr >= sigma_min)
    out = np.zeros(cov.shape, np.float64)
    out[ok] = cov[ok] / (sl[ok] * sr[ok])
    return out


def cost_entries(left, warped, u, v, d, r: int, sigma_min: float) -> np.ndarray:
    """Correlation of the left block centred at (u, v) with the warped-target block
    centred at (u - d, v): one entry c(u, v, d) of Eq. 3 for each index triple."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    d = np.asarray(d, np.int64)
    return zncc(block_values(left, u, v, r), block_values(warped, u - d, v, r), sigma_min)


def cost_volumes(left, warped, D: int, r: int, sigma_min: float):
    """Reference volume C_L[d][v][u] = c(u, v, d) and target volume
    C_R[d][v][x] = c(x + d, v, d) (the identity stated after Eq. 5); where x + d
    leaves the image the same correlation is taken with clamped left reads."""
    H, W = left.shape
    CL = np.empty((D, H, W), np.float64)
    CR = np.empty((D, H, W), np.float64)
    for v0 in range(0, H, ROW_CHUNK):
        v1 = min(H, v0 + ROW_CHUNK)
        vv, uu = np.mgrid[v0:v1, 0:W]
        for d in range(D):
            CL[d, v0:v1] = cost_entries(left, warped, uu, vv, d, r, sigma_min)
            CR[d, v0:v1] = cost_entries(left, warped, uu + d, vv, d, r, sigma_min)
    return CL, CR


# ------------------------------------------------------------------- bilateral (FBS)
def bilateral_weights(guide, u, v, rho: int, gamma_d: float, gamma_r: float):
    """Eq. 9-10 for every tap of the (2rho+1)^2 window around each (u, v).

    Returns (w, qx, qy), each [..., m].  Taps outside the image get w = 0 (their
    indices are clamped only so they can be gathered safely).  Intensities enter the
    range term divided by 255.
    """
    H, W = guide.shape
    g = guide.astype(np.float64)
    u = np.asarray(u, np.int64)[..., None]
    v = np.asarray(v, np.int64)[..., None]
    offs = np.arange(-rho, rho + 1)
    dy = np.repeat(offs, 2 * rho + 1)
    dx = np.tile(offs, 2 * rho + 1)
    qx = u + dx
    qy = v + dy
    inside = (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
    qxc = np.clip(qx, 0, W - 1)
    qyc = np.clip(qy, 0, H - 1)
    w_d = np.exp(-((qx - u) ** 2 + (qy - v) ** 2) / gamma_d ** 2)
    diff = (g[qyc, qxc] - g[np.clip(v, 0, H - 1), np.clip(u, 0, W - 1)]) / 255.0
    w_r = np.exp(-(diff ** 2) / gamma_r ** 2)
    w = np.where(inside, w_d * w_r, 0.0)
    return w, qxc, qyc


def aggregate_volume(C: np.ndarray, guide, rho: int, gamma_d: float, gamma_r: float):
    """Eq. 8 on every (u, v, d): weighted mean of the costs in the window."""
    D, H, W = C.shape
    A = np.empty_like(C, dtype=np.float64)
    for v0 in range(0, H, max(1, ROW_CHUNK // 4)):
        v1 = min(H, v0 + max(1, ROW_CHUNK // 4))
        vv, uu = np.mgrid[v0:v1, 0:W]
        w, qx, qy = bilateral_weights(guide, uu, vv, rho, gamma_d, gamma_r)
        z = w.sum(axis=-1)
        acc = np.zeros((D, v1 - v0, W))
        for k in range(w.shape[-1]):
            acc += w[None, :, :, k] * C[:, qy[:, :, k], qx[:, :, k]]
        A[:, v0:v1] = acc / z[None]
    return A


def aggregate_entries(cost_at, guide, u, v, d, rho: int, gamma_d: float, gamma_r: float):
    """Eq. 8 at sampled (u, v, d) triples.  cost_at(x, y, d) returns raw costs for
    index arrays; it is called once for all window taps of all samples."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    d = np.asarray(d, np.int64)
    w, qx, qy = bilateral_weights(guide, u, v, rho, gamma_d, gamma_r)
    c = cost_at(qx, qy, np.broadcast_to(d[..., None], qx.shape))
    return (w * c).sum(axis=-1) / w.sum(axis=-1)


# -------------------------------------------------------- selection and refinement
def wta(A: np.ndarray):
    """Winner-take-all: highest correlation over d; ties go to the lowest d
    (first occurrence).  Also returns the best and second-best values."""
    disp = np.argmax(A, axis=0)
    part = np.sort(A, axis=0)
    best = part[-1]
    second = part[-2] if A.shape[0] > 1 else np.full_like(best, -np.inf)
    return disp.astype(np.int64), best, second


def lr_check(disp_ref: np.ndarray, disp_tar: np.ndarray, tau: int) -> np.ndarray:
    """Eq. 11: l_ref(u, v) must equal l_tar(u - l_ref(u, v), v) within tau pixels;
    a match falling left of the image is invalid."""
    H, W = disp_ref.shape
    v, u = np.mgrid[0:H, 0:W]
    x = u - disp_ref
    inside = x >= 0
    look = disp_tar[v, np.clip(x, 0, W - 1)]
    return inside & (np.abs(disp_ref - look) <= tau)


def subpixel(A: np.ndarray, disp: np.ndarray) -> np.ndarray:
    """Eq. 12: d_s = d + (c(d-1) - c(d+1)) / (2c(d-1) + 2c(d+1) - 4c(d)); unrefined
    at the ends of the search range."""
    D, H, W = A.shape
    v, u = np.mgrid[0:H, 0:W]
    inner = (disp > 0) & (disp < D - 1)
    dm = np.clip(disp - 1, 0, D - 1)
    dp = np.clip(disp + 1, 0, D - 1)
    cm, c0, cp = A[dm, v, u], A[disp, v, u], A[dp, v, u]
    out = disp.astype(np.float64).copy()
    den = 2 * cm + 2 * cp - 4 * c0
    out[inner] = disp[inner] + (cm[inner] - cp[inner]) / den[inner]
    return out


def postprocess(disp_sub: np.ndarray, plane) -> np.ndarray:
    """Sec. II-C: add the warp shift back.  With the roll term the shift is taken
    at the matched target column: d_f = d_s + s(u - d_s, v)."""
    a0, a1, a2, delta = (float(t) for t in plane)
    H, W = disp_sub.shape
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    return disp_sub + (a0 + a1 * v + a2 * (u - disp_sub) - delta)


def triangulate(disp_final: np.ndarray, valid: np.ndarray, camera) -> np.ndarray:
    """Sec. II-D: z = f*T/d, x = (u-u0) z/f, y = (v-v0) z/f in the left camera frame;
    NaN where the match is invalid or d <= 0."""
    f, T, u0, v0 = (float(t) for t in camera)
    H, W = disp_final.shape
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    ok = valid & (disp_final > 0)
    z = np.where(ok, f * T / np.where(ok, disp_final, 1.0), np.nan)
    xyz = np.stack([(u - u0) * z / f, (v - v0) * z / f, z], axis=-1)
    xyz[~ok] = np.nan
    return xyz


# ----------------------------------------------------------------- whole pipeline
def reconstruct(left, right, plane, camera, D, block_radius, agg_radius, gamma_d,
                gamma_r, lr_threshold=1, sigma_min=1e-2):
    """Fig. 1 pipeline: warp -> both cost volumes -> aggregation -> WTA -> L-R check
    -> subpixel -> post-processing -> 3-D points.  Returns a dict of every stage."""
    Wp = warp(right, plane)
    CL, CR = cost_volumes(left, Wp, D, block_radius, sigma_min)
    AL = aggregate_volume(CL, left, agg_radius, gamma_d, gamma_r)
    AR = aggregate_volume(CR, Wp, agg_radius, gamma_d, gamma_r)
    dref, best, second = wta(AL)
    dtar, _, _ = wta(AR)
    valid = lr_check(dref, dtar, lr_threshold)
    dsub = subpixel(AL, dref)
    dfin = postprocess(dsub, plane)
    xyz = triangulate(dfin, valid, camera)
    return dict(warped=Wp, cost_ref=CL, cost_tar=CR, agg_ref=AL, agg_tar=AR,
                disp_ref=dref, disp_tar=dtar, best=best, second=second, valid=valid,
                disp_sub=dsub, disp_final=dfin, xyz=xyz)
