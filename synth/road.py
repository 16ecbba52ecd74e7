"""Seeded synthetic rectified road pairs.

These pairs stand in for the paper's ZED road datasets (Sec. III), which are not
public.  The generator holds none of the stereo method's arithmetic: it draws a
fractal texture, a road-plane disparity field with Gaussian bumps, and forms the
right image by inverse mapping with Keys cubic interpolation (deliberately not the
linear interpolation the method's warp uses).

Geometry (Sec. II-A): rows are rectified, the left image is the reference, and a
left pixel (u, v) appears in the right image at column u - d(u, v).  The road
disparity is d(u, v) = a*v + b + sum_k A_k exp(-|(u,v) - c_k|^2 / (2 s^2)), the
linear v-d model of Eq. 2 plus bumps and dips.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class RoadScene:
    """Parameters of one synthetic road pair."""
    height: int
    width: int
    plane_a: float            # disparity slope along v (alpha_1 of Eq. 2)
    plane_b: float            # disparity offset (alpha_0 of Eq. 2)
    n_bumps: int = 3
    bump_amp: float = 2.0     # |A_k| in pixels of disparity
    bump_sigma: float = 10.0  # spatial sigma of each bump, pixels
    noise_left: float = 0.0   # std of additive Gaussian noise, grey levels
    noise_right: float = 2.0
    gain_jitter: float = 0.0  # per-image gain drawn from U[1-g, 1+g]
    offset_jitter: float = 0.0  # per-image offset drawn from U[-o, o]
    texture_std: float = 32.0
    texture_mean: float = 128.0
    dtype: str = "u8"         # "u8" (rint + clip) or "f32"


@dataclass
class RoadPair:
    left: np.ndarray          # [H][W] uint8 or float32
    right: np.ndarray         # [H][W] uint8 or float32
    disp_gt: np.ndarray       # [H][W] float64, left-view disparity
    scene: RoadScene
    seed: int
    extra: dict = field(default_factory=dict)


def fractal_texture(rng: np.random.Generator, height: int, width: int,
                    mean: float, std: float) -> np.ndarray:
    """White Gaussian noise shaped to a 1/f amplitude spectrum (DC removed), drawn on
    an FFT-friendly canvas and cropped to height x width."""
    from scipy import fft as sfft
    hh, ww = sfft.next_fast_len(height, real=True), sfft.next_fast_len(width, real=True)
    white = rng.standard_normal((hh, ww))
    spec = sfft.rfft2(white)
    fy = np.fft.fftfreq(hh)[:, None]
    fx = np.fft.rfftfreq(ww)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    amp = np.zeros_like(f)
    amp[f > 0] = 1.0 / f[f > 0]
    tex = sfft.irfft2(spec * amp, s=(hh, ww))[:height, :width]
    tex = (tex - tex.mean()) / tex.std()
    return mean + std * tex


def _keys_cubic_row(row: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Keys (a = -0.5) cubic interpolation of a 1-D signal at real positions x."""
    n = row.shape[0]
    x0 = np.floor(x).astype(np.int64)
    t = x - x0
    a = -0.5

    def k(s):
        s = np.abs(s)
        return np.where(s <= 1, (a + 2) * s**3 - (a + 3) * s**2 + 1,
                        np.where(s < 2, a * s**3 - 5 * a * s**2 + 8 * a * s - 4 * a, 0.0))

    out = np.zeros_like(x, dtype=np.float64)
    for off in (-1, 0, 1, 2):
        idx = np.clip(x0 + off, 0, n - 1)
        out += row[idx] * k(t - off)
    return out


def disparity_field(scene: RoadScene, rng: np.random.Generator):
    """Draw bump centres/signs; return a callable d(u, v) and the bump list."""
    cu = rng.uniform(0, scene.width, scene.n_bumps)
    cv = rng.uniform(0, scene.height, scene.n_bumps)
    sgn = rng.choice([-1.0, 1.0], scene.n_bumps)
    amps = sgn * scene.bump_amp
    two_s2 = 2.0 * scene.bump_sigma ** 2
    reach = 6.0 * scene.bump_sigma  # beyond 6 sigma a bump adds < 2e-8 of its amplitude

    def d(u, v):
        """u, v: [H][W] arrays whose rows share one v value (image grids)."""
        u = np.asarray(u, np.float64)
        v = np.asarray(v, np.float64)
        out = scene.plane_a * v + scene.plane_b
        rows = v[:, 0]
        for k in range(scene.n_bumps):
            r0 = int(np.searchsorted(rows, cv[k] - reach))
            r1 = int(np.searchsorted(rows, cv[k] + reach))
            if r1 <= r0:
                continue
            ub, vb = u[r0:r1], v[r0:r1]
            near = np.abs(ub - cu[k]) < reach
            out[r0:r1][near] += amps[k] * np.exp(-((ub[near] - cu[k]) ** 2 + (vb[near] - cv[k]) ** 2)
                                                 / two_s2)
        return out

    return d, list(zip(cu.tolist(), cv.tolist(), amps.tolist()))


def make_pair(scene: RoadScene, seed: int) -> RoadPair:
    """Render one rectified pair (left = reference, right = target)."""
    rng = np.random.default_rng(seed)
    H, W = scene.height, scene.width
    dfun, bumps = disparity_field(scene, rng)
    max_d = abs(scene.plane_a) * H + abs(scene.plane_b) + scene.bump_amp + 1.0
    margin = int(np.ceil(max_d)) + 16
    canvas_w = W + margin
    tex = fractal_texture(rng, H, canvas_w, scene.texture_mean, scene.texture_std)

    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    d_gt = dfun(uu, vv)

    # Right pixel x shows the scene point whose left column u solves u - d(u, v) = x.
    # |dd/du| <= bump_amp / (bump_sigma * sqrt(e)) (0.18 here) < 1, so the iteration
    # contracts; 15 steps leave an error below 0.18^15 * bump_amp < 1e-10 px.
    xs = uu
    u_star = xs + dfun(xs, vv)
    for _ in range(15):
        u_star = xs + dfun(u_star, vv)
    right = np.empty((H, W), np.float64)
    for v in range(H):
        right[v] = _keys_cubic_row(tex[v], u_star[v])
    left = tex[:, :W].copy()

    def photometric(img, noise_std):
        g = 1.0 + (rng.uniform(-scene.gain_jitter, scene.gain_jitter) if scene.gain_jitter else 0.0)
        o = rng.uniform(-scene.offset_jitter, scene.offset_jitter) if scene.offset_jitter else 0.0
        out = g * img + o
        if noise_std > 0:
            out = out + rng.normal(0.0, noise_std, img.shape)
        return out

    left = photometric(left, scene.noise_left)
    right = photometric(right, scene.noise_right)
    if scene.dtype == "u8":
        left = np.clip(np.rint(left), 0, 255).astype(np.uint8)
        right = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    elif scene.dtype == "f32":
        left = np.clip(left, 0, 255).astype(np.float32)
        right = np.clip(right, 0, 255).astype(np.float32)
    else:
        raise ValueError(f"unknown dtype {scene.dtype!r}")
    return RoadPair(left, right, d_gt, scene, seed, {"bumps": bumps})


def with_dtype(scene: RoadScene, dtype: str) -> RoadScene:
    return dataclasses.replace(scene, dtype=dtype)
