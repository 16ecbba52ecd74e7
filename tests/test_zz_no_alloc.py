"""rsv_cost_adjoint_noalloc, the adjoint's entry point for callers that cannot
allocate: called through the C ABI twice in a row (the second call on a smaller
pair, so it reuses the library's static workspace left by the first) and compared
with rsv_cost_adjoint on the same inputs and a caller-owned workspace.  Both calls
sum float atomics in an unspecified order, so the comparison allows float rounding:
image gradients |a - b| <= 1e-5 |b| + 1e-6 max|b| elementwise, plane terms and loss
to 1e-6 relative."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1807_07433_amd import _lib, ops
from synth.road import RoadScene, make_pair

pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(lib, H, W, D, r, rho, seed, plane):
    print(f"[no-alloc adjoint] H={H} W={W} D={D} r={r} rho={rho} seed={seed}", flush=True)
    p = make_pair(RoadScene(H, W, 0.0, plane[0], n_bumps=2, bump_amp=1.0, noise_right=2.0, dtype="f32"),
                  seed)
    rng = np.random.default_rng(seed)
    disp = _gpu(rng.integers(0, D, (H, W)).astype(np.int32))
    mask = _gpu((rng.random((H, W)) < 0.7).astype(np.uint8))
    prm = ops.StereoParams(D=D, block_radius=r, agg_radius=rho, gamma_d=3.0, gamma_r=0.1)
    L, R = _gpu(p.left), _gpu(p.right)
    cref, _ = ops.joint_views(ops.cost_volume_joint(L, ops.warp(R, plane), prm), W)
    ref = ops.cost_adjoint(L, R, plane, prm, cref, disp, mask)

    gl = torch.full((H, W), float("nan"), device="cuda")
    gr = torch.full((H, W), float("nan"), device="cuda")
    gp = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    loss = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
    cp = ops._params(prm)
    st = lib.rsv_cost_adjoint_noalloc(ops.image(L, "left"), ops.image(R, "right"), ops._plane(plane),
                                      C.byref(cp), cref.data_ptr(), cref.stride(0), cref.stride(1),
                                      disp.data_ptr(), mask.data_ptr(), gl.data_ptr(), gr.data_ptr(),
                                      gp.data_ptr(), loss.data_ptr(), ops._stream(L.device))
    assert st == 0, lib.rsv_status_string(st)
    torch.cuda.synchronize()
    for name, a, b in (("grad_left", gl, ref[0]), ("grad_right", gr, ref[1])):
        err = (a - b).abs()
        bound = 1e-5 * b.abs() + 1e-6 * b.abs().max()
        print(f"  {name}: max|diff| {float(err.max()):.3e}  scale {float(b.abs().max()):.3e}", flush=True)
        assert bool(torch.isfinite(a).all())
        assert bool((err <= bound).all()), name
    torch.testing.assert_close(gp, ref[2], rtol=1e-6, atol=0.0)
    torch.testing.assert_close(loss, ref[3], rtol=1e-6, atol=0.0)


def test_noalloc_adjoint_matches_workspace_form_twice(rsv_gpu):
    lib = _lib.load()
    _run(lib, 96, 160, 24, 3, 5, 41, (9.0, 0.02, 0.003, 12.0))
    _run(lib, 40, 72, 10, 2, 3, 42, (4.5, -0.01, 0.002, 5.0))


def test_noalloc_adjoint_rejects_frames_beyond_its_workspace(rsv_gpu):
    lib = _lib.load()
    W = 2048
    H = _lib.RSV_ADJOINT_NOALLOC_MAX_PIXELS // W + 1
    prm = ops._params(ops.StereoParams(D=16))
    fake = 0x1000
    img = _lib.Image(fake, _lib.RSV_F32, H, W, W)
    st = lib.rsv_cost_adjoint_noalloc(img, img, _lib.Plane(1.0, 0.0, 0.0, 0.0), C.byref(prm), fake,
                                      16 * H * W, W, fake, fake, fake, fake, fake, fake, None)
    assert st == -2
