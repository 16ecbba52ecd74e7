"""Writes the FP64 oracle's full-frame selection maps of a synthetic workload to
tests/golden/<workload>_oracle_maps.npz, for the GPU tests that compare every pixel.

    python tests/golden/make_oracle_maps.py [road1280_d64] [--workers N]

Calls only oracle/ (the FP64 reference) and synth/ (the seeded inputs).  The frame is
cut into row bands; each band is run through the oracle's whole forward path on the
band plus a halo of block_radius + agg_radius rows on each side, with the warp plane
re-based to the band's first row (the shift depends on v), and only the band's own
rows are kept.  Every stage of the path reads at most block_radius rows (the NCC
blocks) and then agg_radius rows (the bilateral window) away from a pixel, and the
warp, the WTA, the left-right check and Eq. 12 never look across rows, so a kept row
sees exactly what it sees in the whole frame: clamp-to-edge reads happen only at the
frame's own top and bottom, which are never cut.

Stored per pixel: disp_ref, disp_tar (uint16), valid (bits), disp_sub (float32, the
oracle's Eq. 12 in float64 rounded once) and den = 2a(d-1) + 2a(d+1) - 4a(d) on the
aggregated reference volume (float32; 0 where Eq. 12 does not apply), plus the sha256
of the input pair so a test can tell that the file belongs to the pair it generates.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import stereo as S  # noqa: E402

WORKLOADS = {"road1280_d64": synth.road1280_d64, "road320_d32": synth.road320_d32,
             "road1920_d128": synth.road1920_d128}
BAND = 24


def pair_digest(left: np.ndarray, right: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in (left, right):
        a = np.ascontiguousarray(a)
        h.update(str((a.dtype.str, a.shape)).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _band(args):
    name, v0, v1 = args
    case = WORKLOADS[name]()
    p, prm = case.pair, case.params
    H = p.left.shape[0]
    halo = prm.block_radius + prm.agg_radius
    s0, s1 = max(0, v0 - halo), min(H, v1 + halo)
    a0, a1, a2, delta = case.plane.as_tuple()
    plane = (a0 + a1 * s0, a1, a2, delta)          # row s0 of the band is row 0 here
    L, R = p.left[s0:s1], p.right[s0:s1]
    Wp = S.warp(R, plane)
    CL, CR = S.cost_volumes(L, Wp, prm.D, prm.block_radius, prm.sigma_min)
    AL = S.aggregate_volume(CL, L, prm.agg_radius, prm.gamma_d, prm.gamma_r)
    AR = S.aggregate_volume(CR, Wp, prm.agg_radius, prm.gamma_d, prm.gamma_r)
    del CL, CR
    dref, _, _ = S.wta(AL)
    dtar, _, _ = S.wta(AR)
    valid = S.lr_check(dref, dtar, prm.lr_threshold)
    dsub = S.subpixel(AL, dref)
    D = prm.D
    d = dref.astype(np.int64)
    inner = (d > 0) & (d < D - 1)
    vv, uu = np.mgrid[0:AL.shape[1], 0:AL.shape[2]]
    am = AL[np.clip(d - 1, 0, D - 1), vv, uu]
    a0v = AL[d, vv, uu]
    ap = AL[np.clip(d + 1, 0, D - 1), vv, uu]
    den = np.where(inner, 2 * am + 2 * ap - 4 * a0v, 0.0)
    k0, k1 = v0 - s0, v1 - s0
    return v0, dict(disp_ref=dref[k0:k1], disp_tar=dtar[k0:k1], valid=valid[k0:k1],
                    disp_sub=dsub[k0:k1], den=den[k0:k1])


def make(name: str, workers: int) -> str:
    case = WORKLOADS[name]()
    H, W = case.pair.left.shape
    bands = [(name, v, min(H, v + BAND)) for v in range(0, H, BAND)]
    maps = {k: [None] * len(bands) for k in ("disp_ref", "disp_tar", "valid", "disp_sub", "den")}
    t0 = time.time()
    with ProcessPoolExecutor(workers) as ex:
        for v0, out in ex.map(_band, bands):
            for k in maps:
                maps[k][v0 // BAND] = out[k]
            print(f"  rows {v0}..{v0 + BAND - 1} done ({time.time() - t0:.0f} s)", flush=True)
    full = {k: np.concatenate(v, axis=0) for k, v in maps.items()}
    path = os.path.join(HERE, f"{name}_oracle_maps.npz")
    np.savez_compressed(path, disp_ref=full["disp_ref"].astype(np.uint16),
                        disp_tar=full["disp_tar"].astype(np.uint16),
                        valid=np.packbits(full["valid"].astype(bool), axis=None),
                        disp_sub=full["disp_sub"].astype(np.float32), den=full["den"].astype(np.float32),
                        shape=np.array([H, W, case.params.D]),
                        pair_sha256=np.array(pair_digest(case.pair.left, case.pair.right)))
    print(f"wrote {path} ({os.path.getsize(path) / 1e6:.1f} MB, {time.time() - t0:.0f} s)")
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", default=["road1280_d64"])
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    a = ap.parse_args()
    for name in a.workloads:
        make(name, a.workers)


if __name__ == "__main__":
    main()
