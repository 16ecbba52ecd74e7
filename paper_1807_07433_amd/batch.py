"""Batched form: a plan over many pairs of uneven size and D, run as one graph launch
of persistent work-queue kernels (rsv_batch_plan_create / rsv_batch_run).
Marshalling only."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import Camera, Image, Params, Plane, check, load
from .ops import _camera, _params, _plane, _stream, image


class PairDesc(C.Structure):
    _fields_ = [("left", Image), ("right", Image), ("plane", Plane), ("camera", Camera),
                ("D", C.c_int32), ("reserved", C.c_int32),
                ("disp_ref", C.c_void_p), ("disp_tar", C.c_void_p), ("disp_sub", C.c_void_p),
                ("valid", C.c_void_p), ("disp_final", C.c_void_p), ("xyz", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("largest_first", C.c_int32), ("cost_tiles_per_item", C.c_int32),
                ("cost_blocks_per_cu", C.c_int32), ("agg_blocks_per_cu", C.c_int32),
                ("per_pair_launches", C.c_int32), ("volume_budget_mib", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def default_tuning() -> Tuning:
    t = Tuning()
    load().rsv_tuning_default(C.byref(t))
    return t


class BatchPlan:
    """Owns an rsv_batch_plan and the output tensors of every pair.

    pairs: list of (left_u8, right_u8, plane, camera, D) with GPU uint8 images.
    outputs[i] holds disp_ref, disp_tar, disp_sub, valid, disp_final, xyz of pair i.
    """

    def __init__(self, pairs, params, tuning: Tuning | None = None, want_xyz: bool = True):
        lib = load()
        self._lib = lib
        self.outputs = []
        self._keep = []
        descs = (PairDesc * len(pairs))()
        for i, (left, right, plane, camera, D) in enumerate(pairs):
            if left.dtype != torch.uint8 or right.dtype != torch.uint8:
                raise TypeError("batched pairs must be uint8 images")
            H, W = left.shape
            dev = left.device
            o = {"disp_ref": torch.empty((H, W), dtype=torch.int32, device=dev),
                 "disp_tar": torch.empty((H, W), dtype=torch.int32, device=dev),
                 "disp_sub": torch.empty((H, W), dtype=torch.float32, device=dev),
                 "valid": torch.empty((H, W), dtype=torch.uint8, device=dev),
                 "disp_final": torch.empty((H, W), dtype=torch.float32, device=dev),
                 "xyz": torch.empty((H, W, 3), dtype=torch.float32, device=dev) if want_xyz else None}
            self.outputs.append(o)
            self._keep += [left, right]
            d = descs[i]
            d.left = image(left, "left")
            d.right = image(right, "right")
            d.plane = _plane(plane)
            d.camera = _camera(camera)
            d.D = int(D)
            d.disp_ref = o["disp_ref"].data_ptr()
            d.disp_tar = o["disp_tar"].data_ptr()
            d.disp_sub = o["disp_sub"].data_ptr()
            d.valid = o["valid"].data_ptr()
            d.disp_final = o["disp_final"].data_ptr()
            d.xyz = o["xyz"].data_ptr() if want_xyz else None
        self._descs = descs
        self._params = _params(params)
        self.tuning = tuning if tuning is not None else default_tuning()
        self._plan = C.c_void_p()
        check(lib.rsv_batch_plan_create(descs, len(pairs), C.byref(self._params), C.byref(self.tuning),
                                        C.byref(self._plan)), "rsv_batch_plan_create")

    def run(self, stream=None):
        s = _stream() if stream is None else stream
        check(self._lib.rsv_batch_run(self._plan, s), "rsv_batch_run")

    def info(self):
        n, g, b = (C.c_int32 * 2)(), (C.c_int32 * 2)(), C.c_int64()
        check(self._lib.rsv_batch_plan_info(self._plan, n, g, C.byref(b)), "rsv_batch_plan_info")
        return {"cost_items": n[0], "agg_items": n[1], "cost_blocks": g[0], "agg_blocks": g[1],
                "workspace_bytes": b.value}

    def close(self):
        if self._plan:
            self._lib.rsv_batch_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def autotune(pairs, params):
        """Times candidate launch shapes on this batch; returns (Tuning, ms)."""
        probe = BatchPlan(pairs, params)   # descriptors + output buffers
        lib = probe._lib
        t = Tuning()
        ms = C.c_float()
        check(lib.rsv_autotune(probe._descs, len(pairs), C.byref(probe._params), C.byref(t),
                               C.byref(ms), _stream()), "rsv_autotune")
        probe.close()
        return t, float(ms.value)
