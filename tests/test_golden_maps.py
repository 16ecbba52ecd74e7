"""The stored oracle maps (tests/golden/make_oracle_maps.py) on the CPU: the banded
computation the script uses gives the whole-frame oracle's maps, and the committed
file belongs to the pair the generator draws today."""
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import synth
from oracle import stereo as S
from tests.golden import make_oracle_maps as M

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_banded_oracle_equals_whole_frame():
    """road320_d32: bands of 24 rows with a halo of block_radius + agg_radius rows and the
    plane re-based per band give the whole-frame maps (the subpixel map to FP64 rounding
    of the re-based plane)."""
    case = synth.road320_d32()
    p, prm = case.pair, case.params
    H = p.left.shape[0]
    bands = [("road320_d32", v, min(H, v + M.BAND)) for v in range(0, H, M.BAND)]
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        res = dict(ex.map(M._band, bands))
    ref = S.reconstruct(p.left, p.right, case.plane.as_tuple(), (700.0, 0.12, 0.0, 0.0), prm.D,
                        prm.block_radius, prm.agg_radius, prm.gamma_d, prm.gamma_r, prm.lr_threshold,
                        prm.sigma_min)
    full = {k: np.concatenate([res[v][k] for v in sorted(res)], 0)
            for k in ("disp_ref", "disp_tar", "valid", "disp_sub")}
    for k in ("disp_ref", "disp_tar", "valid"):
        assert np.array_equal(full[k], ref[k]), k
    assert np.abs(full["disp_sub"] - ref["disp_sub"]).max() < 1e-9


def test_stored_maps_belong_to_the_generated_pair():
    path = os.path.join(GOLDEN, "road1280_d64_oracle_maps.npz")
    g = np.load(path)
    case = synth.road1280_d64()
    H, W = case.pair.left.shape
    assert tuple(g["shape"]) == (H, W, case.params.D)
    assert str(g["pair_sha256"]) == M.pair_digest(case.pair.left, case.pair.right)
    d = g["disp_ref"]
    assert d.shape == (H, W) and int(d.max()) < case.params.D
