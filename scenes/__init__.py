"""Seeded synthetic scenes and cameras for the INPC point rasterizer.

This package only draws inputs (point positions, opacities, features, radii,
upstream gradients, cameras).  It holds none of the rasterizer's arithmetic,
so both the CPU oracle and the GPU path can consume its output without
sharing any computation.
"""
from .generator import (  # noqa: F401
    Camera,
    Scene,
    SceneSpec,
    CONFIGS,
    make_scene,
    make_camera,
    multi_view_scenes,
    multi_view_specs,
    ring_camera,
    tiny_scene,
)
