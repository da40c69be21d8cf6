"""MI355X-native pose scoring for RenderMap (arXiv 1702.06813).

The package wraps librendermap.so (hand-written HIP for gfx950) through its
C ABI (include/rendermap.h).  PyTorch provides device memory and streams.
"""
from .rendermap import (  # noqa: F401
    ABI_SYMBOLS, FO, FU, NONE, OUT_COUNTS, OUT_E_SOFT, OUT_E_TABLE, OUT_GRAD, OUT_JTJ, OUT_JTR, OUT_N_ACTIVE,
    OUT_N_VISIBLE, OUT_STRIDE, UO, AlignCost, Context, Graph, Mesh, RenderMapError, Scan, align_cost,
    adam_step, align_cost_grad, align_cost_grad_noalloc, context, gn_step, load_library, mesh_from_range, render_depth, scan_image, se3_retract,
    OUT_ICP_COST, OUT_ICP_N_MODEL, OUT_ICP_N_SCAN, OUT_ICP_SSE, depth_downsample, depth_normals, downsample_camera,
    icp_cost_grad, vertex_normals, TABLE_WEIGHTS, N_WEIGHTS, table_cost_weighted, OUT_COLOR_REWARD, OUT_COLOR_PENALTY,
    RM_OK, RM_ERR_INVALID_ARG, RM_ERR_OOM, RM_ERR_DEVICE, RM_ERR_CAPACITY, RM_ERR_UNSUPPORTED,
)
