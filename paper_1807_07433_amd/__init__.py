"""Road-surface dense stereo on MI355X (gfx950).

Hand-written HIP kernels behind a C ABI (include/rsv.h, librsv.so) for the path of
Fan et al., arXiv 1807.07433: perspective warp, ZNCC reference/target cost
volumes, bilateral cost aggregation, WTA with left-right check, parabola subpixel
refinement, post-processing and triangulation, and the RANSAC road-plane fit.  This package is the thin Python
binding; PyTorch supplies device memory and streams.
"""
from ._lib import RsvError, load, LIB_PATH  # noqa: F401
from .ops import (StereoParams, aggregate, aggregate_argmax, aggregate_restricted_argmax,  # noqa: F401
                  aggregate_restricted_select, aggregate_restricted_views, aggregate_select,
                  aggregate_select_supported, aggregate_views, cost_adjoint, cost_argmax, cost_argmax_views,
                  cost_volume, cost_volume_joint, image, joint_row_stride, joint_views, lr_check,
                  plane_ransac, reconstruct, reconstruct_restricted, select_subpixel, selected_aggregate_sum,
                  selected_cost_sum, triangulate, warp)

__version__ = "0.1.0"
