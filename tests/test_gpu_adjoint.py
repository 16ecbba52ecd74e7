"""GPU parity of the differentiable form: rsv_cost_adjoint against the FP64 oracle
gradient (itself pinned to central differences in test_oracle_adjoint.py), the loss
against the oracle loss, and the plane refinement on the 8-pair 1280x720 workload.

Tolerance: the GPU computes in FP32 with float atomics.  Image gradients are held
elementwise to |g_gpu - g_ref| <= 1e-3 * |g_ref| + 2e-5 * max|g_ref| (every pixel,
the clamped border pixels included, which also get their own report); the three
plane terms to |g_gpu - g_ref| <= 1e-3 * |g_ref| + 1e-6 * max|g_ref|.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as OA
from synth.road import RoadScene, make_pair

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(tag, gpu, ref, rtol=1e-3, atol=2e-5, border=0):
    gpu = np.asarray(gpu, np.float64)
    scale = np.abs(ref).max()
    err = np.abs(gpu - ref)
    bound = rtol * np.abs(ref) + atol * scale
    worst = float((err / bound).max())
    _say(f"  {tag}: max|err| {err.max():.3e}  scale {scale:.3e}  worst err/bound {worst:.3f}")
    if border:
        edge = np.ones(ref.shape, bool)
        edge[border:-border, border:-border] = False
        rel = err[edge] / np.maximum(np.abs(ref[edge]), 1e-30)
        big = np.abs(ref[edge]) >= 1e-3 * scale
        _say(f"  {tag} border ({border} px): max|err| {err[edge].max():.3e}  "
             f"max rel err where |g| >= 1e-3 max: {rel[big].max() if big.any() else 0.0:.3e}")
    assert worst <= 1.0, f"{tag}: elementwise error exceeds {rtol}*|g| + {atol}*max|g| (x{worst:.2f})"


CASES = [
    # H, W, D, r, rho, seed, plane
    (30, 44, 6, 2, 2, 11, (5.5, 0.004, 0.002, 0.0)),
    (41, 77, 12, 3, 4, 12, (7.3, 0.011, -0.003, 3.0)),
    (26, 53, 9, 1, 6, 13, (2.6, -0.02, 0.004, 1.0)),
]


@pytest.mark.parametrize("H,W,D,r,rho,seed,plane", CASES)
def test_adjoint_matches_oracle_gradient(rsv_gpu, H, W, D, r, rho, seed, plane):
    rsv = rsv_gpu
    _say(f"[adjoint] H={H} W={W} D={D} r={r} rho={rho} seed={seed}")
    p = make_pair(RoadScene(H, W, 0.0, plane[0], n_bumps=1, bump_amp=0.5, noise_right=2.0,
                            dtype="f32"), seed)
    rng = np.random.default_rng(seed)
    disp = rng.integers(0, D, (H, W)).astype(np.int32)
    mask = (rng.random((H, W)) < 0.6).astype(np.uint8)
    prm = rsv.StereoParams(D=D, block_radius=r, agg_radius=rho, gamma_d=2.5, gamma_r=0.1)
    L, R = _gpu(p.left), _gpu(p.right)
    wp = rsv.warp(R, plane)
    cref, _ = rsv.cost_volume(L, wp, prm, want_tar=False)
    aref = rsv.aggregate(cref, L, prm)
    gl, gr, gp, loss = rsv.cost_adjoint(L, R, plane, prm, cref, _gpu(disp), _gpu(mask))
    lsum = rsv.selected_cost_sum(aref, _gpu(disp), _gpu(mask))
    lagg = rsv.selected_aggregate_sum(cref, L, prm, _gpu(disp), _gpu(mask))
    jref, _ = rsv.joint_views(rsv.cost_volume_joint(L, wp, prm), W)
    gl2, gr2, gp2, loss2 = rsv.cost_adjoint(L, R, plane, prm, jref, _gpu(disp), _gpu(mask))
    torch.cuda.synchronize()
    ref_loss, rgl, rgr, rgp = OA.grad(p.left, p.right, plane, disp, mask.astype(bool), r, rho, 2.5,
                                      0.1)
    nm = mask.sum()
    assert abs(float(loss) - ref_loss) <= 1e-4 * nm
    # the three forms of the loss: aggregated volume, cost volume, in the adjoint
    assert abs(float(lsum) - float(loss)) <= 1e-5 * nm
    assert abs(float(lagg) - float(loss)) <= 1e-5 * nm
    # the joint volume's reference view is the same cost volume
    assert abs(float(loss2) - float(loss)) <= 1e-9 * nm
    torch.testing.assert_close(gl2, gl, rtol=1e-5, atol=1e-6 * float(gl.abs().max()))
    torch.testing.assert_close(gr2, gr, rtol=1e-5, atol=1e-6 * float(gr.abs().max()))
    torch.testing.assert_close(gp2, gp, rtol=1e-6, atol=0.0)
    _compare("grad_left", gl.cpu().numpy(), rgl, border=r + rho)
    _compare("grad_right", gr.cpu().numpy(), rgr, border=r + rho)
    g = gp.cpu().numpy()
    _say(f"  grad_plane gpu {g}  oracle {rgp}")
    assert np.all(np.abs(g - rgp) <= 1e-3 * np.abs(rgp) + 1e-6 * np.abs(rgp).max())


def test_adjoint_out_of_range_disparity_is_ignored(rsv_gpu):
    rsv = rsv_gpu
    p = make_pair(RoadScene(24, 40, 0.0, 4.0, n_bumps=0, noise_right=2.0, dtype="f32"), 3)
    prm = rsv.StereoParams(D=5, block_radius=2, agg_radius=2, gamma_d=2.0)
    L, R = _gpu(p.left), _gpu(p.right)
    wp = rsv.warp(R, (4.0, 0.0, 0.0, 2.0))
    cref, _ = rsv.cost_volume(L, wp, prm, want_tar=False)
    disp = torch.full((24, 40), 2, dtype=torch.int32, device="cuda")
    mask = torch.ones((24, 40), dtype=torch.uint8, device="cuda")
    bad = disp.clone()
    bad[5:9, 10:20] = 77
    bad[12, :] = -3
    keep = mask.clone()
    keep[5:9, 10:20] = 0
    keep[12, :] = 0
    _say("[adjoint] out-of-range disparities leave the loss")
    a = rsv.cost_adjoint(L, R, (4.0, 0.0, 0.0, 2.0), prm, cref, bad, mask)
    b = rsv.cost_adjoint(L, R, (4.0, 0.0, 0.0, 2.0), prm, cref, disp, keep)
    la = rsv.selected_aggregate_sum(cref, L, prm, bad, mask)
    lb = rsv.selected_aggregate_sum(cref, L, prm, disp, keep)
    assert abs(float(la) - float(lb)) < 1e-9
    assert abs(float(a[3]) - float(b[3])) < 1e-9
    assert torch.allclose(a[0], b[0], atol=1e-5) and torch.allclose(a[1], b[1], atol=1e-5)


def test_adjoint_full_size_sampled_omega(rsv_gpu):
    """1280x720, D = 64 float32 pair; Omega = 2000 random pixels so the oracle finishes."""
    rsv = rsv_gpu
    cases, starts = synth.diff8_road1280(n_pairs=1)
    c, plane = cases[0], starts[0].as_tuple()
    H, W = c.pair.left.shape
    prm = c.params
    _say(f"[adjoint full] {W}x{H} D={prm.D}")
    L, R = _gpu(c.pair.left), _gpu(c.pair.right)
    from paper_1807_07433_amd.autograd import select
    d, _ = select(L, R, plane, prm)
    rng = np.random.default_rng(1)
    mask = np.zeros((H, W), np.uint8)
    mask.flat[rng.choice(H * W, 2000, replace=False)] = 1
    wp = rsv.warp(R, plane)
    cref, _ = rsv.joint_views(rsv.cost_volume_joint(L, wp, prm), W)
    gl, gr, gp, loss = rsv.cost_adjoint(L, R, plane, prm, cref, d, _gpu(mask))
    torch.cuda.synchronize()
    dn = d.cpu().numpy()
    ref_loss, rgl, rgr, rgp = OA.grad(c.pair.left, c.pair.right, plane, dn, mask.astype(bool),
                                      prm.block_radius, prm.agg_radius, prm.gamma_d, prm.gamma_r)
    assert abs(float(loss) - ref_loss) <= 1e-4 * mask.sum()
    _compare("grad_left", gl.cpu().numpy(), rgl, border=prm.block_radius + prm.agg_radius)
    _compare("grad_right", gr.cpu().numpy(), rgr, border=prm.block_radius + prm.agg_radius)
    g = gp.cpu().numpy()
    _say(f"  grad_plane gpu {g}  oracle {rgp}")
    assert np.all(np.abs(g - rgp) <= 1e-3 * np.abs(rgp) + 1e-6 * np.abs(rgp).max())


def test_autograd_function_matches_adjoint(rsv_gpu):
    rsv = rsv_gpu
    from paper_1807_07433_amd.autograd import AggregatedZNCC
    p = make_pair(RoadScene(40, 90, 0.05, 6.0, n_bumps=1, noise_right=2.0, dtype="f32"), 21)
    prm = rsv.StereoParams(D=10, block_radius=3, agg_radius=3, gamma_d=2.0)
    L = _gpu(p.left).requires_grad_(True)
    R = _gpu(p.right).requires_grad_(True)
    theta = torch.tensor([6.2, 0.05, 0.001], dtype=torch.float64, requires_grad=True)
    disp = torch.full((40, 90), 4, dtype=torch.int32, device="cuda")
    mask = torch.ones((40, 90), dtype=torch.uint8, device="cuda")
    _say("[autograd] backward through AggregatedZNCC")
    loss = AggregatedZNCC.apply(L, R, theta, 5.0, prm, disp, mask)
    (2.0 * loss).backward()
    plane = (6.2, 0.05, 0.001, 5.0)
    wp = rsv.warp(R.detach(), plane)
    cref, _ = rsv.cost_volume(L.detach(), wp, prm, want_tar=False)
    gl, gr, gp, l2 = rsv.cost_adjoint(L.detach(), R.detach(), plane, prm, cref, disp, mask)
    assert abs(float(loss.detach()) - float(l2)) < 1e-5 * 40 * 90
    assert torch.allclose(L.grad, 2 * gl, rtol=1e-4, atol=1e-6)
    assert torch.allclose(R.grad, 2 * gr, rtol=1e-4, atol=1e-6)
    assert torch.allclose(theta.grad, 2 * gp.cpu(), rtol=1e-6)


def test_plane_refinement_reduces_shift_error(rsv_gpu):
    """8 float32 1280x720 pairs, D = 64, 50 steps from a plane perturbed by <= 0.4 px."""
    from paper_1807_07433_amd.autograd import refine_plane
    cases, starts = synth.diff8_road1280(n_pairs=8)
    H, W = cases[0].pair.left.shape
    v, u = np.mgrid[0:H, 0:W]

    def shift_err(theta, true):
        s = theta[0] + theta[1] * v + theta[2] * u
        t = true.a0 + true.a1 * v + true.a2 * u
        return float(np.sqrt(np.mean((s - t) ** 2)))

    # every pair shares one plane: start from pair 0's perturbed start
    true = cases[0].plane
    start = starts[0]
    lefts = [_gpu(c.pair.left) for c in cases]
    rights = [_gpu(c.pair.right) for c in cases]
    e0 = shift_err((start.a0, start.a1, start.a2), true)
    _say(f"[refine] start shift rms error {e0:.4f} px")
    theta, hist = refine_plane(lefts, rights, (start.a0, start.a1, start.a2), true.delta,
                               cases[0].params, steps=50, lr=0.02)
    e1 = shift_err(theta.numpy(), true)
    _say(f"[refine] after 50 steps {e1:.4f} px; loss {hist[0]:.5f} -> {hist[-1]:.5f}")
    assert hist[-1] > hist[0]
    assert e1 < 0.5 * e0
