"""MI355X (gfx950) point rasterizer of "A Bag of Tricks for Efficient Implicit
Neural Point Clouds": project, bin, per-tile depth sort, alpha blend (bilinear
2x2 splats, screen-space Gaussians, or world-space Gaussians with the EWA
projection), and the backward pass, as HIP kernels behind a C ABI
(include/inpc_raster.h).
"""
from . import _lib  # noqa: F401
from .batched import BatchedRasterizer, MultiViewRasterizer, ViewInputs, ViewPipeline  # noqa: F401
from .ring import PointRing  # noqa: F401
from .raster import (  # noqa: F401
    Binning,
    BlendGrads,
    RasterSettings,
    Workspace,
    blend_backward,
    blend_forward,
    camera_struct,
    check_capacity,
    envmap_background,
    ewa_max_radius,
    project_backward,
    project_bin_sort,
    rasterize,
    sh_features,
    view_directions,
)

__all__ = [
    "BatchedRasterizer", "MultiViewRasterizer", "ViewInputs", "ViewPipeline", "Binning", "BlendGrads", "RasterSettings", "Workspace", "blend_backward", "blend_forward",
    "camera_struct", "check_capacity", "project_backward", "project_bin_sort", "rasterize", "envmap_background", "view_directions", "sh_features",
    "ewa_max_radius", "PointRing",
]
