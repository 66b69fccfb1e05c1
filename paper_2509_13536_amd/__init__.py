"""MemGS hot path on MI355X (gfx950): differentiable tile rasteriser and voxel merge.

The computation lives in libmemgs.so (HIP, C ABI in include/memgs.h); this
package marshals torch device tensors into it.
"""
from ._abi import MemgsError, load as load_library  # noqa: F401
from .api import (  # noqa: F401
    CHI2_3DOF_95,
    AdamState,
    GRAD_TAU,
    LAMBDA_SSIM,
    ForwardState,
    GaussianMap,
    GradStats,
    LossResult,
    PatchGridResult,
    MergeResult,
    View,
    Workspace,
    render_backward,
    adam_step,
    mapping_loss,
    mapping_loss_noalloc,
    merge_mask,
    patch_grid_sample,
    render_forward,
    voxel_merge,
)
