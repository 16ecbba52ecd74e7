"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the
benchmark.  Nothing here computes any step of the stereo method: this module only
draws images, ground-truth disparities and the method's parameter values.

Workloads (sizes in pixels, D = residual disparity search range):
  road320_d32      one 320x180 uint8 pair, plane d = 0.1 v + 4, 3 bumps of +-2 px,
                   right-image noise N(0, 2); NCC 7x7, D = 32, bilateral 9x9.
  road1280_d64     one 1280x720 uint8 pair, plane d = 0.15 v + 10, 12 bumps of +-3 px;
                   NCC 7x7, D = 64, bilateral 11x11, baseline 0.12 m, f = 700 px.
  road1920_d128    one 1920x1080 uint8 pair, plane d = 0.2 v + 15, 20 bumps, noise N(0, 3)
                   and +-10 % gain / offset on both images; NCC 9x9, D = 128, bilateral 13x13.
  batch64_mixed    64 pairs, sizes from {640x360, 1280x720, 1920x1080}, D from {32, 64, 128};
                   NCC 7x7, bilateral 11x11.
  diff8_road1280   8 float32 pairs of the road1280_d64 kind with a perturbed starting plane.
  plane_fit_input  a disparity map for the road-plane fit: a plane with a roll term plus
                   N(0, noise), a fraction of gross outliers, invalid holes, and the RANSAC
                   draws (3 distinct valid pixels each).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from .road import RoadPair, RoadScene, make_pair, fractal_texture, with_dtype  # noqa: F401


@dataclass(frozen=True)
class MethodParams:
    """Parameter values of the stereo method (Sec. II); plain data only."""
    D: int                    # residual disparity search range
    block_radius: int         # NCC block radius (block width 2r+1)
    agg_radius: int           # bilateral window radius
    gamma_d: float            # spatial parameter of the bilateral weight
    gamma_r: float            # range parameter (intensities scaled to [0, 1])
    lr_threshold: int = 1     # left-right consistency tolerance, pixels
    sigma_min: float = 1e-2   # block std-dev below which the correlation is defined as 0


@dataclass(frozen=True)
class Camera:
    f: float = 700.0          # focal length, pixels
    baseline: float = 0.12    # metres
    u0: float | None = None   # principal point; None = image centre
    v0: float | None = None


@dataclass(frozen=True)
class Plane:
    """Warp plane s(u, v) = a0 + a1*v + a2*u - delta (pixels)."""
    a0: float
    a1: float
    a2: float
    delta: float

    def as_tuple(self):
        return (self.a0, self.a1, self.a2, self.delta)


@dataclass
class Case:
    name: str
    pair: RoadPair
    params: MethodParams
    plane: Plane
    camera: Camera


def _case(name, scene, params, seed, camera=None):
    pair = make_pair(scene, seed)
    plane = Plane(scene.plane_b, scene.plane_a, 0.0, float(params.D // 2))
    cam = camera or Camera()
    cam = replace(cam, u0=(scene.width - 1) / 2.0 if cam.u0 is None else cam.u0,
                  v0=(scene.height - 1) / 2.0 if cam.v0 is None else cam.v0)
    return Case(name, pair, params, plane, cam)


SCENE_320 = RoadScene(180, 320, 0.1, 4.0, n_bumps=3, bump_amp=2.0, noise_right=2.0)
PARAMS_320 = MethodParams(D=32, block_radius=3, agg_radius=4, gamma_d=3.0, gamma_r=0.1)

SCENE_1280 = RoadScene(720, 1280, 0.15, 10.0, n_bumps=12, bump_amp=3.0, noise_right=2.0)
PARAMS_1280 = MethodParams(D=64, block_radius=3, agg_radius=5, gamma_d=4.0, gamma_r=0.1)

SCENE_1920 = RoadScene(1080, 1920, 0.2, 15.0, n_bumps=20, bump_amp=3.0, noise_left=3.0,
                       noise_right=3.0, gain_jitter=0.1, offset_jitter=25.5)
PARAMS_1920 = MethodParams(D=128, block_radius=4, agg_radius=6, gamma_d=5.0, gamma_r=0.1)

BATCH_SIZES = ((360, 640), (720, 1280), (1080, 1920))
BATCH_DS = (32, 64, 128)


def road320_d32(index: int = 0) -> Case:
    return _case("road320_d32", SCENE_320, PARAMS_320, 1000 + index)


def road1280_d64(index: int = 0, dtype: str = "u8") -> Case:
    return _case("road1280_d64", with_dtype(SCENE_1280, dtype), PARAMS_1280, 2000 + index)


def road1920_d128(index: int = 0) -> Case:
    return _case("road1920_d128", SCENE_1920, PARAMS_1920, 3000 + index)


def _batch_case(args):
    i, scene, params = args
    return _case(f"batch64_mixed[{i}]", scene, params, 4000 + i)


def batch64_mixed(n_pairs: int = 64, sizes=BATCH_SIZES, ds=BATCH_DS, workers: int = 0) -> list[Case]:
    """Uneven batch: every pair has its own size, D, plane and bumps.  Each pair is
    seeded on its own, so `workers` > 1 (a process pool) gives the same pairs."""
    rng = np.random.default_rng(4000)
    jobs = []
    for i in range(n_pairs):
        h, w = sizes[rng.integers(len(sizes))]
        D = int(ds[rng.integers(len(ds))])
        a = float(rng.uniform(0.1, 0.2))
        b = float(rng.uniform(4.0, 15.0))
        nb = int(rng.integers(3, 21))
        scene = RoadScene(h, w, a, b, n_bumps=nb, bump_amp=3.0, noise_right=2.0)
        params = MethodParams(D=D, block_radius=3, agg_radius=5, gamma_d=4.0, gamma_r=0.1)
        jobs.append((i, scene, params))
    if workers and workers > 1:
        import concurrent.futures as cf
        with cf.ProcessPoolExecutor(workers) as ex:
            return list(ex.map(_batch_case, jobs))
    return [_batch_case(j) for j in jobs]


def diff8_road1280(n_pairs: int = 8) -> tuple[list[Case], list[Plane]]:
    """Float32 pairs plus a perturbed starting plane per pair (|shift change| <= 0.4 px)."""
    cases = [_case("diff8_road1280", with_dtype(SCENE_1280, "f32"), PARAMS_1280, 5000 + i)
             for i in range(n_pairs)]
    rng = np.random.default_rng(5999)
    starts = []
    for c in cases:
        H, W = c.pair.scene.height, c.pair.scene.width
        # split a 0.4 px budget over the three plane terms at the image extremes
        da0 = rng.uniform(-0.15, 0.15)
        da1 = rng.uniform(-0.15, 0.15) / H
        da2 = rng.uniform(-0.1, 0.1) / W
        p = c.plane
        starts.append(Plane(p.a0 + da0, p.a1 + da1, p.a2 + da2, p.delta))
    return cases, starts


def small_case(height: int, width: int, D: int, block_radius: int, agg_radius: int,
               seed: int, plane_a: float = 0.05, plane_b: float = 3.0, n_bumps: int = 2,
               gamma_d: float = 3.0, gamma_r: float = 0.1, dtype: str = "u8",
               noise_right: float = 2.0) -> Case:
    """A small pair for tests whose sizes span several tiles and a ragged tail."""
    scene = RoadScene(height, width, plane_a, plane_b, n_bumps=n_bumps, bump_amp=1.5,
                      noise_right=noise_right, dtype=dtype)
    params = MethodParams(D=D, block_radius=block_radius, agg_radius=agg_radius,
                          gamma_d=gamma_d, gamma_r=gamma_r)
    return _case(f"small_{height}x{width}_d{D}", scene, params, seed)


def ransac_draws(valid: np.ndarray, n_draws: int, rng: np.random.Generator) -> np.ndarray:
    """n_draws x 3 linear indices (v * W + u) of distinct valid pixels, int32."""
    idx = np.flatnonzero(np.asarray(valid).ravel())
    return np.stack([idx[rng.choice(idx.size, 3, replace=False)] for _ in range(n_draws)]).astype(np.int32)


def plane_fit_input(height: int, width: int, seed: int, plane=(10.0, 0.15, -0.004), noise: float = 0.05,
                    outliers: float = 0.3, holes: float = 0.1, n_draws: int = 256,
                    base: np.ndarray | None = None):
    """(disp float32 [H][W], valid uint8 [H][W], draws int32 [K][3]) for the road-plane
    fit: base (0 if None) + a0 + a1 v + a2 u + N(0, noise); a fraction `outliers` of the
    pixels replaced by U(0, max); a fraction `holes` marked invalid."""
    rng = np.random.default_rng(seed)
    v, u = np.mgrid[0:height, 0:width].astype(np.float64)
    d = plane[0] + plane[1] * v + plane[2] * u + rng.normal(0.0, noise, (height, width))
    if base is not None:
        d = d + base
    out = rng.random((height, width)) < outliers
    d[out] = rng.uniform(0.0, float(d.max()), int(out.sum()))
    valid = rng.random((height, width)) >= holes
    return d.astype(np.float32), valid.astype(np.uint8), ransac_draws(valid, n_draws, rng)
