"""Torch-tensor front end of the C ABI: checks device, dtype and layout, passes
device pointers and the current HIP stream, raises RsvError on a bad status.
Every step of the path runs in librsv's kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import Camera, Image, Params, Plane, RsvError, check, load


@dataclass(frozen=True)
class StereoParams:
    """Method parameters (Sec. II-B); field names match the C struct."""
    D: int
    block_radius: int = 3
    agg_radius: int = 5
    gamma_d: float = 4.0
    gamma_r: float = 0.1
    lr_threshold: int = 1
    sigma_min: float = 1e-2


def _params(p) -> Params:
    return Params(int(p.D), int(p.block_radius), int(p.agg_radius), int(p.lr_threshold),
                  float(p.gamma_d), float(p.gamma_r), float(p.sigma_min))


def _plane(pl) -> Plane:
    t = pl.as_tuple() if hasattr(pl, "as_tuple") else tuple(pl)
    return Plane(*(float(x) for x in t))


def _camera(cam) -> Camera:
    if hasattr(cam, "f"):
        return Camera(float(cam.f), float(cam.baseline), float(cam.u0), float(cam.v0))
    return Camera(*(float(x) for x in cam))


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev(t: torch.Tensor, name: str, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def image(t: torch.Tensor, name: str = "image") -> Image:
    """rsv_image over a 2-D uint8 / float32 GPU tensor (row stride may exceed width)."""
    _dev(t, name, (torch.uint8, torch.float32))
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride")
    dt = _lib.RSV_U8 if t.dtype == torch.uint8 else _lib.RSV_F32
    return Image(t.data_ptr(), dt, t.shape[0], t.shape[1], t.stride(0))


def _contig(t, name, dtype, shape):
    _dev(t, name, dtype, shape)
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else t.data_ptr()


def warp(right: torch.Tensor, plane, out: torch.Tensor | None = None) -> torch.Tensor:
    lib = load()
    H, W = right.shape
    out = out if out is not None else torch.empty((H, W), dtype=torch.float32, device=right.device)
    _contig(out, "warped", torch.float32, (H, W))
    check(lib.rsv_warp(image(right, "right"), _plane(plane), out.data_ptr(), _stream(right.device)),
          "rsv_warp")
    return out


def cost_volume(left: torch.Tensor, warped: torch.Tensor, params, want_tar: bool = True,
                out_ref: torch.Tensor | None = None, out_tar: torch.Tensor | None = None):
    lib = load()
    H, W = left.shape
    D = int(params.D)
    _contig(warped, "warped", torch.float32, (H, W))
    shp = (D, H, W)
    cref = out_ref if out_ref is not None else torch.empty(shp, dtype=torch.float32, device=left.device)
    _contig(cref, "cost_ref", torch.float32, shp)
    ctar = None
    if want_tar:
        ctar = out_tar if out_tar is not None else torch.empty(shp, dtype=torch.float32, device=left.device)
        _contig(ctar, "cost_tar", torch.float32, shp)
    p = _params(params)
    check(lib.rsv_cost_volume(image(left, "left"), warped.data_ptr(), C.byref(p), cref.data_ptr(),
                              _ptr(ctar), _stream(left.device)), "rsv_cost_volume")
    return cref, ctar


def joint_row_stride(W: int, D: int) -> int:
    """Row stride of the joint volume: W + D - 1 rounded up to a multiple of 64."""
    return (W + D - 1 + 63) // 64 * 64


def cost_volume_joint(left: torch.Tensor, warped: torch.Tensor, params,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """Both cost volumes as one [D][H][row_stride] volume (rsv_cost_volume_joint);
    joint_views gives the reference and target volumes as views of it."""
    lib = load()
    H, W = left.shape
    D = int(params.D)
    _contig(warped, "warped", torch.float32, (H, W))
    shp = (D, H, joint_row_stride(W, D))
    out = out if out is not None else torch.empty(shp, dtype=torch.float32, device=left.device)
    _contig(out, "joint", torch.float32, shp)
    p = _params(params)
    check(lib.rsv_cost_volume_joint(image(left, "left"), warped.data_ptr(), C.byref(p), out.data_ptr(),
                                    shp[2], _stream(left.device)), "rsv_cost_volume_joint")
    return out


def joint_views(joint: torch.Tensor, W: int) -> tuple[torch.Tensor, torch.Tensor]:
    """(cost_ref, cost_tar) [D][H][W] as strided views of a joint volume: the target
    volume's plane stride is one element longer (cost_tar[d][v][x] = joint[d][v][x + d])."""
    D, H, rs = joint.shape
    if not joint.is_contiguous() or rs < W + D - 1:
        raise ValueError("joint must be a contiguous [D][H][row_stride >= W + D - 1] volume")
    ref = joint.as_strided((D, H, W), (H * rs, rs, 1))
    tar = joint.as_strided((D, H, W), (H * rs + 1, rs, 1))
    return ref, tar


def aggregate(cost: torch.Tensor, guide: torch.Tensor, params,
              out: torch.Tensor | None = None) -> torch.Tensor:
    """Bilateral aggregation of a [D][H][W] volume: contiguous (rsv_aggregate) or any
    view with unit column stride, e.g. from joint_views (rsv_aggregate_strided)."""
    lib = load()
    D, H, W = cost.shape
    _dev(cost, "cost", torch.float32, (int(params.D), H, W))
    if tuple(guide.shape) != (H, W):
        raise ValueError("guide must match the volume's H, W")
    out = out if out is not None else torch.empty((D, H, W), dtype=torch.float32, device=cost.device)
    _contig(out, "agg", torch.float32, (D, H, W))
    p = _params(params)
    if cost.is_contiguous():
        check(lib.rsv_aggregate(cost.data_ptr(), image(guide, "guide"), C.byref(p), out.data_ptr(),
                                _stream(cost.device)), "rsv_aggregate")
    else:
        if cost.stride(2) != 1:
            raise ValueError("cost views need unit column stride")
        check(lib.rsv_aggregate_strided(cost.data_ptr(), cost.stride(0), cost.stride(1),
                                        image(guide, "guide"), C.byref(p), out.data_ptr(),
                                        _stream(cost.device)), "rsv_aggregate_strided")
    return out


def aggregate_argmax(cost: torch.Tensor, guide: torch.Tensor, params,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """argmax over d of the aggregation of a [D][H][W] volume or view (ties -> lowest
    d), without writing the aggregated volume (rsv_aggregate_argmax): the target
    disparities that select_subpixel takes in place of the target volume."""
    lib = load()
    D, H, W = cost.shape
    _dev(cost, "cost", torch.float32, (int(params.D), H, W))
    if tuple(guide.shape) != (H, W):
        raise ValueError("guide must match the volume's H, W")
    if cost.stride(2) != 1:
        raise ValueError("cost views need unit column stride")
    out = out if out is not None else torch.empty((H, W), dtype=torch.int32, device=cost.device)
    _contig(out, "disp", torch.int32, (H, W))
    p = _params(params)
    check(lib.rsv_aggregate_argmax(cost.data_ptr(), cost.stride(0), cost.stride(1), image(guide, "guide"),
                                   C.byref(p), out.data_ptr(), _stream(cost.device)), "rsv_aggregate_argmax")
    return out


def aggregate_select_supported(W: int, params) -> bool:
    """Whether rsv_aggregate_select runs for this width and radius (agg_radius <= 5, W >= 4)."""
    return int(params.agg_radius) <= 5 and W >= 4


def aggregate_select(cost: torch.Tensor, guide: torch.Tensor, params, disp_tar: torch.Tensor,
                     out: dict | None = None) -> dict:
    """The reference aggregation with WTA, Eq. 12 and Eq. 11 (against disp_tar) folded
    in (rsv_aggregate_select): disp_ref, disp_sub and valid, bit for bit those of
    aggregate + select_subpixel(agg_ref, None), without the aggregated volume."""
    lib = load()
    D, H, W = cost.shape
    _dev(cost, "cost", torch.float32, (int(params.D), H, W))
    if tuple(guide.shape) != (H, W):
        raise ValueError("guide must match the volume's H, W")
    if cost.stride(2) != 1:
        raise ValueError("cost views need unit column stride")
    _contig(disp_tar, "disp_tar", torch.int32, (H, W))
    dev = cost.device
    o = dict(out) if out else {}
    shapes = {"disp_ref": ((H, W), torch.int32), "disp_sub": ((H, W), torch.float32),
              "valid": ((H, W), torch.uint8)}
    for k, (shp, dt) in shapes.items():
        if k not in o:
            o[k] = torch.empty(shp, dtype=dt, device=dev)
        _contig(o[k], k, dt, shp)
    o["disp_tar"] = disp_tar
    p = _params(params)
    check(lib.rsv_aggregate_select(cost.data_ptr(), cost.stride(0), cost.stride(1), image(guide, "guide"),
                                   C.byref(p), disp_tar.data_ptr(), o["disp_ref"].data_ptr(),
                                   o["disp_sub"].data_ptr(), o["valid"].data_ptr(), _stream(dev)),
          "rsv_aggregate_select")
    return o


def aggregate_views(cost_ref: torch.Tensor, cost_tar: torch.Tensor, guide_ref: torch.Tensor,
                    guide_tar: torch.Tensor, params, out: dict | None = None) -> dict:
    """Both views aggregated in one launch (rsv_aggregate_views): disp_tar as
    aggregate_argmax gives it, disp_ref and disp_sub as the selection gives them (the
    winner and Eq. 12), bit for bit; the left-right check is lr_check's.  guide_tar is
    the float32 warped right image.  Any window radius and width."""
    lib = load()
    D, H, W = cost_ref.shape
    for t, n in ((cost_ref, "cost_ref"), (cost_tar, "cost_tar")):
        _dev(t, n, torch.float32, (int(params.D), H, W))
        if t.stride(2) != 1:
            raise ValueError(f"{n}: cost views need unit column stride")
    for g, n in ((guide_ref, "guide_ref"), (guide_tar, "guide_tar")):
        if tuple(g.shape) != (H, W):
            raise ValueError(f"{n} must match the volume's H, W")
    dev = cost_ref.device
    o = dict(out) if out else {}
    shapes = {"disp_tar": ((H, W), torch.int32), "disp_ref": ((H, W), torch.int32),
              "disp_sub": ((H, W), torch.float32)}
    for k, (shp, dt) in shapes.items():
        if k not in o:
            o[k] = torch.empty(shp, dtype=dt, device=dev)
        _contig(o[k], k, dt, shp)
    p = _params(params)
    check(lib.rsv_aggregate_views(cost_ref.data_ptr(), cost_ref.stride(0), cost_ref.stride(1), cost_tar.data_ptr(),
                                  cost_tar.stride(0), cost_tar.stride(1), image(guide_ref, "guide_ref"),
                                  image(guide_tar, "guide_tar"), C.byref(p), o["disp_tar"].data_ptr(),
                                  o["disp_ref"].data_ptr(), o["disp_sub"].data_ptr(), _stream(dev)),
          "rsv_aggregate_views")
    return o


def aggregate_restricted_views(cost_ref: torch.Tensor, cost_tar: torch.Tensor, guide_ref: torch.Tensor,
                               guide_tar: torch.Tensor, params, coarse_ref: torch.Tensor, coarse_tar: torch.Tensor,
                               radius: int, out: dict | None = None) -> dict:
    """Both views' restricted aggregations in one launch (rsv_aggregate_restricted_views):
    disp_tar, disp_ref and disp_sub as aggregate_restricted_argmax and
    aggregate_restricted_select give them, bit for bit; the left-right check is
    lr_check's."""
    lib = load()
    D, H, W = cost_ref.shape
    for t, n in ((cost_ref, "cost_ref"), (cost_tar, "cost_tar")):
        _dev(t, n, torch.float32, (int(params.D), H, W))
        if t.stride(2) != 1:
            raise ValueError(f"{n}: cost views need unit column stride")
    for g, n in ((guide_ref, "guide_ref"), (guide_tar, "guide_tar")):
        if tuple(g.shape) != (H, W):
            raise ValueError(f"{n} must match the volume's H, W")
    _contig(coarse_ref, "coarse_ref", torch.int32, (H, W))
    _contig(coarse_tar, "coarse_tar", torch.int32, (H, W))
    dev = cost_ref.device
    o = dict(out) if out else {}
    shapes = {"disp_tar": ((H, W), torch.int32), "disp_ref": ((H, W), torch.int32),
              "disp_sub": ((H, W), torch.float32)}
    for k, (shp, dt) in shapes.items():
        if k not in o:
            o[k] = torch.empty(shp, dtype=dt, device=dev)
        _contig(o[k], k, dt, shp)
    p = _params(params)
    check(lib.rsv_aggregate_restricted_views(cost_ref.data_ptr(), cost_ref.stride(0), cost_ref.stride(1),
                                             cost_tar.data_ptr(), cost_tar.stride(0), cost_tar.stride(1),
                                             image(guide_ref, "guide_ref"), image(guide_tar, "guide_tar"), C.byref(p),
                                             coarse_ref.data_ptr(), coarse_tar.data_ptr(), int(radius),
                                             o["disp_tar"].data_ptr(), o["disp_ref"].data_ptr(),
                                             o["disp_sub"].data_ptr(), _stream(dev)),
          "rsv_aggregate_restricted_views")
    return o


def lr_check(disp_ref: torch.Tensor, disp_tar: torch.Tensor, tau: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. 11 on two winner-take-all maps (rsv_lr_check): uint8 valid [H][W]."""
    lib = load()
    H, W = disp_ref.shape
    _contig(disp_ref, "disp_ref", torch.int32, (H, W))
    _contig(disp_tar, "disp_tar", torch.int32, (H, W))
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=disp_ref.device)
    _contig(out, "valid", torch.uint8, (H, W))
    check(lib.rsv_lr_check(disp_ref.data_ptr(), disp_tar.data_ptr(), H, W, int(tau), out.data_ptr(),
                           _stream(disp_ref.device)), "rsv_lr_check")
    return out


def cost_argmax(cost: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """First argmax over d of an unaggregated [D][H][W] cost volume or view
    (rsv_cost_argmax): the calculated disparities of the restricted search (Sec. IV)."""
    lib = load()
    D, H, W = cost.shape
    _dev(cost, "cost", torch.float32)
    if cost.stride(2) != 1:
        raise ValueError("cost views need unit column stride")
    out = out if out is not None else torch.empty((H, W), dtype=torch.int32, device=cost.device)
    _contig(out, "disp", torch.int32, (H, W))
    check(lib.rsv_cost_argmax(cost.data_ptr(), cost.stride(0), cost.stride(1), H, W, D, out.data_ptr(),
                              _stream(cost.device)), "rsv_cost_argmax")
    return out


def cost_argmax_views(cost_ref: torch.Tensor, cost_tar: torch.Tensor, out: tuple | None = None) -> tuple:
    """cost_argmax of two views in one pass (rsv_cost_argmax_views): (coarse_ref,
    coarse_tar), each bit for bit cost_argmax's."""
    lib = load()
    D, H, W = cost_ref.shape
    for t, n in ((cost_ref, "cost_ref"), (cost_tar, "cost_tar")):
        _dev(t, n, torch.float32, (D, H, W))
        if t.stride(2) != 1:
            raise ValueError(f"{n}: cost views need unit column stride")
    dev = cost_ref.device
    cr, ct = out if out is not None else (torch.empty((H, W), dtype=torch.int32, device=dev),
                                          torch.empty((H, W), dtype=torch.int32, device=dev))
    _contig(cr, "disp_ref", torch.int32, (H, W))
    _contig(ct, "disp_tar", torch.int32, (H, W))
    check(lib.rsv_cost_argmax_views(cost_ref.data_ptr(), cost_ref.stride(0), cost_ref.stride(1), cost_tar.data_ptr(),
                                    cost_tar.stride(0), cost_tar.stride(1), H, W, D, cr.data_ptr(), ct.data_ptr(),
                                    _stream(dev)), "rsv_cost_argmax_views")
    return cr, ct


def aggregate_restricted_argmax(cost: torch.Tensor, guide: torch.Tensor, params, coarse: torch.Tensor,
                                radius: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """rsv_aggregate_argmax inside each pixel's window of min(2 radius + 1, D) disparities
    around coarse (rsv_aggregate_restricted_argmax, Sec. IV)."""
    lib = load()
    D, H, W = cost.shape
    _dev(cost, "cost", torch.float32, (int(params.D), H, W))
    if tuple(guide.shape) != (H, W) or cost.stride(2) != 1:
        raise ValueError("guide must match the volume's H, W; cost views need unit column stride")
    _contig(coarse, "coarse", torch.int32, (H, W))
    out = out if out is not None else torch.empty((H, W), dtype=torch.int32, device=cost.device)
    _contig(out, "disp", torch.int32, (H, W))
    p = _params(params)
    check(lib.rsv_aggregate_restricted_argmax(cost.data_ptr(), cost.stride(0), cost.stride(1), image(guide, "guide"),
                                              C.byref(p), coarse.data_ptr(), int(radius), out.data_ptr(),
                                              _stream(cost.device)), "rsv_aggregate_restricted_argmax")
    return out


def aggregate_restricted_select(cost: torch.Tensor, guide: torch.Tensor, params, coarse: torch.Tensor,
                                radius: int, disp_tar: torch.Tensor, out: dict | None = None) -> dict:
    """rsv_aggregate_select inside each pixel's window around coarse
    (rsv_aggregate_restricted_select, Sec. IV): disp_ref, disp_sub, valid."""
    lib = load()
    D, H, W = cost.shape
    _dev(cost, "cost", torch.float32, (int(params.D), H, W))
    if tuple(guide.shape) != (H, W) or cost.stride(2) != 1:
        raise ValueError("guide must match the volume's H, W; cost views need unit column stride")
    _contig(coarse, "coarse", torch.int32, (H, W))
    _contig(disp_tar, "disp_tar", torch.int32, (H, W))
    dev = cost.device
    o = dict(out) if out else {}
    shapes = {"disp_ref": ((H, W), torch.int32), "disp_sub": ((H, W), torch.float32),
              "valid": ((H, W), torch.uint8)}
    for k, (shp, dt) in shapes.items():
        if k not in o:
            o[k] = torch.empty(shp, dtype=dt, device=dev)
        _contig(o[k], k, dt, shp)
    o["disp_tar"] = disp_tar
    p = _params(params)
    check(lib.rsv_aggregate_restricted_select(cost.data_ptr(), cost.stride(0), cost.stride(1),
                                              image(guide, "guide"), C.byref(p), coarse.data_ptr(), int(radius),
                                              disp_tar.data_ptr(), o["disp_ref"].data_ptr(),
                                              o["disp_sub"].data_ptr(), o["valid"].data_ptr(), _stream(dev)),
          "rsv_aggregate_restricted_select")
    return o


def reconstruct_restricted(left: torch.Tensor, right: torch.Tensor, plane, camera, params, radius: int,
                           out: dict | None = None) -> dict:
    """The plain path with the restricted search of Sec. IV: warp -> joint cost volume ->
    calculated disparities of both views in one pass (rsv_cost_argmax_views) -> both views' aggregations
    over the windows of min(2 radius + 1, D) disparities in one launch, with the
    selection folded in (rsv_aggregate_restricted_views) -> left-right check ->
    post-processing + 3-D points."""
    wp = warp(right, plane)
    cref, ctar = joint_views(cost_volume_joint(left, wp, params), left.shape[1])
    cc_ref, cc_tar = cost_argmax_views(cref, ctar)
    sel = aggregate_restricted_views(cref, ctar, left, wp, params, cc_ref, cc_tar, radius, out=out)
    sel["valid"] = lr_check(sel["disp_ref"], sel["disp_tar"], params.lr_threshold,
                            out=(out or {}).get("valid"))
    dfin, xyz = triangulate(sel["disp_sub"], sel["valid"], plane, camera)
    res = dict(warped=wp, cost_ref=cref, cost_tar=ctar, coarse_ref=cc_ref, coarse_tar=cc_tar,
               disp_final=dfin, xyz=xyz)
    res.update(sel)
    return res


def plane_ransac(disp: torch.Tensor, valid: torch.Tensor, samples: torch.Tensor, threshold: float,
                 workspace: torch.Tensor | None = None) -> dict:
    """Road-plane estimation of Sec. II-A (rsv_plane_ransac): RANSAC over the draws
    samples [K][3] (linear pixel indices v*W + u) on the valid pixels of disp, then
    the least-squares plane (a0, a1, a2) of d = a0 + a1 v + a2 u through the best
    hypothesis's inliers.  Returns device tensors: plane float64 [3], counts int32 [K]
    (-1 for degenerate draws), best int32 [2] (hypothesis, inlier count)."""
    lib = load()
    H, W = disp.shape
    _contig(disp, "disp", torch.float32, (H, W))
    _contig(valid, "valid", torch.uint8, (H, W))
    if samples.dim() != 2 or samples.shape[1] != 3:
        raise ValueError("samples must be [K][3]")
    K = int(samples.shape[0])
    _contig(samples, "samples", torch.int32, (K, 3))
    if not 1 <= K <= _lib.RSV_PLANE_MAX_K:
        raise ValueError(f"K = {K} outside 1..{_lib.RSV_PLANE_MAX_K}")
    dev = disp.device
    nbytes = lib.rsv_plane_ransac_workspace_bytes(K)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
    plane = torch.empty(3, dtype=torch.float64, device=dev)
    counts = torch.empty(K, dtype=torch.int32, device=dev)
    best = torch.empty(2, dtype=torch.int32, device=dev)
    check(lib.rsv_plane_ransac(disp.data_ptr(), valid.data_ptr(), H, W, samples.data_ptr(), K,
                               float(threshold), plane.data_ptr(), counts.data_ptr(), best.data_ptr(),
                               workspace.data_ptr(), _stream(dev)), "rsv_plane_ransac")
    return dict(plane=plane, counts=counts, best=best)


def select_subpixel(agg_ref: torch.Tensor, agg_tar: torch.Tensor | None, params, want_top2: bool = False,
                    out: dict | None = None) -> dict:
    """WTA, left-right check and Eq. 12.  With agg_tar None, out["disp_tar"] must hold
    the target disparities (aggregate_argmax) and rsv_select_subpixel_ref runs."""
    lib = load()
    D, H, W = agg_ref.shape
    _contig(agg_ref, "agg_ref", torch.float32, (int(params.D), H, W))
    if agg_tar is not None:
        _contig(agg_tar, "agg_tar", torch.float32, (D, H, W))
    elif not out or "disp_tar" not in out:
        raise ValueError("without agg_tar, out['disp_tar'] must hold the target disparities")
    dev = agg_ref.device
    o = dict(out) if out else {}
    shapes = {"disp_ref": ((H, W), torch.int32), "disp_tar": ((H, W), torch.int32),
              "disp_sub": ((H, W), torch.float32), "valid": ((H, W), torch.uint8)}
    if want_top2:
        shapes["top2"] = ((2, H, W), torch.float32)
    for k, (shp, dt) in shapes.items():
        if k not in o:  # allocate only what the caller did not pass
            o[k] = torch.empty(shp, dtype=dt, device=dev)
    _contig(o["disp_ref"], "disp_ref", torch.int32, (H, W))
    _contig(o["disp_tar"], "disp_tar", torch.int32, (H, W))
    _contig(o["disp_sub"], "disp_sub", torch.float32, (H, W))
    _contig(o["valid"], "valid", torch.uint8, (H, W))
    top2 = o.get("top2")
    if top2 is not None:
        _contig(top2, "top2", torch.float32, (2, H, W))
    p = _params(params)
    if agg_tar is not None:
        check(lib.rsv_select_subpixel(agg_ref.data_ptr(), agg_tar.data_ptr(), H, W, C.byref(p),
                                      o["disp_ref"].data_ptr(), o["disp_tar"].data_ptr(),
                                      o["disp_sub"].data_ptr(), o["valid"].data_ptr(), _ptr(top2),
                                      _stream(dev)), "rsv_select_subpixel")
    else:
        check(lib.rsv_select_subpixel_ref(agg_ref.data_ptr(), o["disp_tar"].data_ptr(), H, W, C.byref(p),
                                          o["disp_ref"].data_ptr(), o["disp_sub"].data_ptr(),
                                          o["valid"].data_ptr(), _ptr(top2), _stream(dev)),
              "rsv_select_subpixel_ref")
    return o


def triangulate(disp_sub: torch.Tensor, valid: torch.Tensor, plane, camera,
                out_disp: torch.Tensor | None = None, out_xyz: torch.Tensor | None = None):
    lib = load()
    H, W = disp_sub.shape
    _contig(disp_sub, "disp_sub", torch.float32, (H, W))
    _contig(valid, "valid", torch.uint8, (H, W))
    dev = disp_sub.device
    dfin = out_disp if out_disp is not None else torch.empty((H, W), dtype=torch.float32, device=dev)
    xyz = out_xyz if out_xyz is not None else torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    _contig(dfin, "disp_final", torch.float32, (H, W))
    _contig(xyz, "xyz", torch.float32, (H, W, 3))
    check(lib.rsv_triangulate(disp_sub.data_ptr(), valid.data_ptr(), H, W, _plane(plane),
                              _camera(camera), dfin.data_ptr(), xyz.data_ptr(), _stream(dev)),
          "rsv_triangulate")
    return dfin, xyz


def selected_cost_sum(agg_ref: torch.Tensor, disp: torch.Tensor, mask: torch.Tensor,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """Loss of the differentiable form: sum of agg_ref[disp(p)][p] over mask(p) != 0."""
    lib = load()
    D, H, W = agg_ref.shape
    _contig(agg_ref, "agg_ref", torch.float32, (D, H, W))
    _contig(disp, "disp", torch.int32, (H, W))
    _contig(mask, "mask", torch.uint8, (H, W))
    out = out if out is not None else torch.empty((), dtype=torch.float64, device=agg_ref.device)
    _contig(out, "out", torch.float64, ())
    check(lib.rsv_selected_cost_sum(agg_ref.data_ptr(), disp.data_ptr(), mask.data_ptr(), H, W, D,
                                    out.data_ptr(), _stream(agg_ref.device)), "rsv_selected_cost_sum")
    return out


def _cost_view(cost: torch.Tensor, D: int, H: int, W: int):
    _dev(cost, "cost", torch.float32, (D, H, W))
    if cost.stride(2) != 1:
        raise ValueError("cost views need unit column stride")
    return cost.stride(0), cost.stride(1)


def selected_aggregate_sum(cost: torch.Tensor, guide: torch.Tensor, params, disp: torch.Tensor,
                           mask: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Loss of the differentiable form from a cost volume or view (rsv_selected_aggregate_sum):
    the aggregation of Eq. 8 at disp(p), summed over mask(p) != 0, with no aggregated volume."""
    lib = load()
    H, W = guide.shape
    D = int(params.D)
    cps, crs = _cost_view(cost, D, H, W)
    _contig(disp, "disp", torch.int32, (H, W))
    _contig(mask, "mask", torch.uint8, (H, W))
    out = out if out is not None else torch.empty((), dtype=torch.float64, device=cost.device)
    _contig(out, "out", torch.float64, ())
    p = _params(params)
    check(lib.rsv_selected_aggregate_sum(cost.data_ptr(), cps, crs, image(guide, "guide"), C.byref(p),
                                         disp.data_ptr(), mask.data_ptr(), out.data_ptr(),
                                         _stream(cost.device)), "rsv_selected_aggregate_sum")
    return out


def cost_adjoint(left: torch.Tensor, right: torch.Tensor, plane, params, cost_ref: torch.Tensor,
                 disp: torch.Tensor, mask: torch.Tensor, workspace: torch.Tensor | None = None):
    """Gradients of the loss sum_{mask} A_ref(p, disp(p)) with respect to the left image,
    the right image and the plane terms (a0, a1, a2); also returns the loss.  left/right
    are float32; cost_ref is the forward's reference cost volume, dense or a view with
    unit column stride (e.g. joint_views(...)[0])."""
    lib = load()
    H, W = left.shape
    D = int(params.D)
    _dev(left, "left", torch.float32)
    _dev(right, "right", torch.float32, (H, W))
    cps, crs = _cost_view(cost_ref, D, H, W)
    _contig(disp, "disp", torch.int32, (H, W))
    _contig(mask, "mask", torch.uint8, (H, W))
    dev = left.device
    nbytes = lib.rsv_cost_adjoint_workspace_bytes(H, W)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty((nbytes + 3) // 4, dtype=torch.float32, device=dev)
    gl = torch.empty((H, W), dtype=torch.float32, device=dev)
    gr = torch.empty((H, W), dtype=torch.float32, device=dev)
    gp = torch.empty(3, dtype=torch.float64, device=dev)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    p = _params(params)
    check(lib.rsv_cost_adjoint(image(left, "left"), image(right, "right"), _plane(plane), C.byref(p),
                               cost_ref.data_ptr(), cps, crs, disp.data_ptr(), mask.data_ptr(),
                               gl.data_ptr(), gr.data_ptr(), gp.data_ptr(), loss.data_ptr(),
                               workspace.data_ptr(), _stream(dev)),
          "rsv_cost_adjoint")
    return gl, gr, gp, loss


def reconstruct(left: torch.Tensor, right: torch.Tensor, plane, camera, params,
                want_top2: bool = False, joint: bool = True, tar_volume: bool = True,
                ref_volume: bool = True) -> dict:
    """The plain path, one C-ABI call per stage on the current stream (Fig. 1):
    warp -> both cost volumes -> aggregation of each -> WTA + L-R + subpixel ->
    post-processing + 3-D points.  With joint=True the two cost volumes are views of
    one joint volume (rsv_cost_volume_joint); otherwise two dense volumes.  With
    tar_volume=False the target volume is reduced to its argmax as it is aggregated
    (rsv_aggregate_argmax) and "agg_tar" is None.  With ref_volume=False as well (and
    without top2) both views are aggregated in one launch with the selection folded in
    (rsv_aggregate_views, then rsv_lr_check) and "agg_ref" is None.  Every other output
    is the same."""
    wp = warp(right, plane)
    if joint:
        cref, ctar = joint_views(cost_volume_joint(left, wp, params), left.shape[1])
    else:
        cref, ctar = cost_volume(left, wp, params)
    if not tar_volume and not ref_volume and not want_top2:
        sel = aggregate_views(cref, ctar, left, wp, params)
        sel["valid"] = lr_check(sel["disp_ref"], sel["disp_tar"], params.lr_threshold)
        dfin, xyz = triangulate(sel["disp_sub"], sel["valid"], plane, camera)
        out = dict(warped=wp, cost_ref=cref, cost_tar=ctar, agg_ref=None, agg_tar=None,
                   disp_final=dfin, xyz=xyz)
        out.update(sel)
        return out
    aref = aggregate(cref, left, params)
    if tar_volume:
        atar = aggregate(ctar, wp, params)
        sel = select_subpixel(aref, atar, params, want_top2=want_top2)
    else:
        atar = None
        sel = select_subpixel(aref, None, params, want_top2=want_top2,
                              out={"disp_tar": aggregate_argmax(ctar, wp, params)})
    dfin, xyz = triangulate(sel["disp_sub"], sel["valid"], plane, camera)
    out = dict(warped=wp, cost_ref=cref, cost_tar=ctar, agg_ref=aref, agg_tar=atar,
               disp_final=dfin, xyz=xyz)
    out.update(sel)
    return out


__all__ = ["StereoParams", "RsvError", "warp", "cost_volume", "cost_volume_joint", "joint_views",
           "joint_row_stride", "aggregate", "aggregate_argmax", "aggregate_select", "aggregate_views", "aggregate_restricted_views", "cost_argmax_views", "lr_check",
           "aggregate_select_supported", "select_subpixel",
           "triangulate", "reconstruct", "selected_cost_sum", "selected_aggregate_sum", "cost_adjoint",
           "cost_argmax", "aggregate_restricted_argmax", "aggregate_restricted_select", "reconstruct_restricted",
           "image", "load"]
