"""Differentiable form: the aggregated reference ZNCC cost at the selected
disparities, as a torch.autograd.Function whose backward is the hand-written
adjoint kernel (rsv_cost_adjoint), plus a plane-refinement loop built on it.

    loss = AggregatedZNCC.apply(left, right, theta, delta, params, disp, mask[, joint[, plane]])

theta = (a0, a1, a2) of the warp shift s = a0 + a1 v + a2 u - delta (Sec. II-A).
The forward runs the plain path's kernels (warp, joint ZNCC volume) and sums the
aggregation of Eq. 8 at disp(p) over mask(p) != 0 (rsv_selected_aggregate_sum); no
aggregated volume is formed.  `joint`, if given, is the joint cost volume of this
very (left, right, plane), e.g. the one `select` returns, and is not recomputed;
`plane`, if given, is theta's value as the host tuple (a0, a1, a2, delta), which saves
reading theta back from the device.
disp and mask are held fixed inside one evaluation (WTA stays exact and is re-run
between steps by `select`).  Gradients flow to left, right (float32 images) and
theta.
"""
from __future__ import annotations

import torch

from . import ops


def _plane(theta: torch.Tensor, delta: float):
    t = theta.detach().to("cpu", torch.float64)
    return (float(t[0]), float(t[1]), float(t[2]), float(delta))


class AggregatedZNCC(torch.autograd.Function):
    @staticmethod
    def forward(ctx, left, right, theta, delta, params, disp, mask, joint=None, plane=None):
        if plane is None:
            plane = _plane(theta, delta)
        if joint is None:
            joint = ops.cost_volume_joint(left, ops.warp(right, plane), params)
        cref, _ = ops.joint_views(joint, left.shape[1])
        loss = ops.selected_aggregate_sum(cref, left, params, disp, mask)
        ctx.save_for_backward(left, right, joint, disp, mask)
        ctx.plane = plane
        ctx.params = params
        ctx.theta_meta = (theta.dtype, theta.device)
        return loss

    @staticmethod
    def backward(ctx, gout):
        left, right, joint, disp, mask = ctx.saved_tensors
        cref, _ = ops.joint_views(joint, left.shape[1])
        gl, gr, gp, _ = ops.cost_adjoint(left, right, ctx.plane, ctx.params, cref, disp, mask)
        dtype, device = ctx.theta_meta
        s = gout.to(torch.float64)
        g_theta = (gp * s).to(device=device, dtype=dtype)
        sf = s.to(torch.float32)
        return gl * sf, gr * sf, g_theta, None, None, None, None, None, None


def select(left, right, plane, params, return_joint: bool = False):
    """Plain-path selection for the current plane, in its fastest form (joint cost
    volume, both views aggregated in one launch with the selection folded in, then the
    left-right check): returns (disp_ref int32, mask uint8) with
    mask = left-right valid and 0 < d < D-1 (pixels where Eq. 12 applies); with
    return_joint, also the joint cost volume, which AggregatedZNCC takes for the same
    plane."""
    W = left.shape[1]
    wp = ops.warp(right, plane)
    joint = ops.cost_volume_joint(left, wp, params)
    cref, ctar = ops.joint_views(joint, W)
    sel = ops.aggregate_views(cref, ctar, left, wp, params)
    sel["valid"] = ops.lr_check(sel["disp_ref"], sel["disp_tar"], params.lr_threshold)
    d = sel["disp_ref"]
    mask = (sel["valid"].bool() & (d > 0) & (d < int(params.D) - 1)).to(torch.uint8)
    return (d, mask, joint) if return_joint else (d, mask)


def refine_plane(lefts, rights, theta0, delta, params, steps=50, lr=0.02, reselect_every=1,
                 callback=None):
    """Gradient ascent of the summed aggregated correlation over a batch of pairs.

    theta0: (a0, a1, a2) starting plane.  Parameters are scaled so one unit of each moves
    the shift by about one pixel across the image (a1 by 1/H, a2 by 1/W), then updated
    with Adam on -loss.  d* and Omega are re-selected every `reselect_every` steps.
    The parameters and the optimiser live on the images' device; the plane is read
    back once per step (the kernels take it by value).
    Returns (theta, history of losses)."""
    H, W = lefts[0].shape
    dev = lefts[0].device
    scale = torch.tensor([1.0, 1.0 / H, 1.0 / W], dtype=torch.float64, device=dev)
    z = (torch.as_tensor(theta0, dtype=torch.float64, device=dev) / scale).clone().requires_grad_(True)
    opt = torch.optim.Adam([z], lr=lr)
    sel = None
    hist = []
    for it in range(steps):
        theta = z * scale
        plane = _plane(theta, delta)
        fresh = sel is None or it % reselect_every == 0
        if fresh:
            sel = []
            for l, r in zip(lefts, rights):
                d, m, joint = select(l, r, plane, params, return_joint=True)
                sel.append((d, m, joint, m.sum(dtype=torch.float64).clamp_min(1.0)))
        opt.zero_grad()
        objective = 0.0
        for (l, r), (d, m, joint, cnt) in zip(zip(lefts, rights), sel):
            loss = AggregatedZNCC.apply(l, r, theta, delta, params, d, m, joint if fresh else None, plane)
            objective = objective + loss / cnt
        objective = objective / len(lefts)
        (-objective).backward()
        opt.step()
        hist.append(objective.detach())
        if callback:
            callback(it, (z * scale).detach().cpu(), float(hist[-1]))
    return (z * scale).detach().cpu(), [float(h) for h in hist]
