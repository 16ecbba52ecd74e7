"""Seeded generator: determinism and that the pair really has the stated geometry."""
import numpy as np

import synth
from synth.road import RoadScene, make_pair


def test_seed_determinism():
    a = synth.road320_d32()
    b = synth.road320_d32()
    assert np.array_equal(a.pair.left, b.pair.left)
    assert np.array_equal(a.pair.right, b.pair.right)
    c = synth.road320_d32(index=1)
    assert not np.array_equal(a.pair.left, c.pair.left)


def test_shapes_and_dtypes():
    c = synth.road320_d32()
    assert c.pair.left.shape == (180, 320) and c.pair.left.dtype == np.uint8
    assert c.pair.right.shape == (180, 320) and c.pair.right.dtype == np.uint8
    assert c.params.D == 32 and c.plane.delta == 16


def test_right_image_is_inverse_warp_of_left():
    """R(u - d_gt(u, v), v) matches L(u, v) best at the ground-truth disparity: the
    residual is minimal there and far below that of a half-pixel offset."""
    scene = RoadScene(60, 200, 0.1, 6.0, n_bumps=2, bump_amp=2.0, noise_right=0.0, dtype="f32")
    p = make_pair(scene, 7)
    H, W = p.left.shape

    def rms(off):
        e = []
        for v in range(H):
            x = np.arange(40, W - 10) - p.disp_gt[v, 40:W - 10] + off
            r = np.interp(x, np.arange(W), p.right[v].astype(np.float64))
            e.append(r - p.left[v, 40:W - 10])
        return np.sqrt(np.mean(np.concatenate(e) ** 2))

    r0 = rms(0.0)
    assert r0 < rms(-0.15) and r0 < rms(0.15)
    assert r0 < 0.5 * rms(-0.5) and r0 < 0.5 * rms(0.5)


def test_integer_plane_is_exact_shift():
    scene = RoadScene(20, 90, 0.0, 7.0, n_bumps=0, noise_right=0.0, dtype="f32")
    p = make_pair(scene, 3)
    assert np.allclose(p.right[:, :80], p.left[:, 7:87], atol=1e-4)


def test_gain_offset_scene_does_not_saturate_much():
    scene = synth.SCENE_1920
    small = RoadScene(270, 480, scene.plane_a, scene.plane_b, n_bumps=5, bump_amp=3.0,
                      noise_left=3.0, noise_right=3.0, gain_jitter=0.1, offset_jitter=25.5)
    p = make_pair(small, 3000)
    for img in (p.left, p.right):
        assert np.mean((img == 0) | (img == 255)) < 0.01


def test_batch_draw_is_uneven():
    cases = synth.batch64_mixed(n_pairs=12, sizes=((36, 64), (72, 128)), ds=(32, 64))
    assert len({c.pair.left.shape for c in cases}) > 1
    assert len({c.params.D for c in cases}) > 1
