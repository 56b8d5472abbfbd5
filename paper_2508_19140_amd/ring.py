"""Ring buffer of view-specific point clouds (Sec. 3.1 "Fast and Stable
View-Specific Sampling during Inference"): instead of sampling several
view-specific clouds for every frame, each frame samples one new cloud and
reuses the clouds of the previous frames.

The ring is one device allocation of `slots` slots of `capacity` points
(positions, opacities, features and optionally screen-space radii, laid out
like a single cloud of slots * capacity points).  `push` writes a new cloud
into the oldest slot; `rasterize` renders the union of the live points of
every slot in one pass (inpc_project_ring culls the slot tails), so no cloud
is copied to assemble the frame's point set.
"""
from __future__ import annotations

from typing import List, Optional

import torch

from .raster import RasterSettings, Workspace, rasterize


class PointRing:
    def __init__(self, slots: int, capacity: int, channels: int, device,
                 feat_dtype: torch.dtype = torch.float32, with_radius: bool = False):
        if not 1 <= slots <= 16:
            raise ValueError("a ring holds 1 to 16 slots")
        if capacity < 1 or slots * capacity >= 1 << 31:
            raise ValueError("ring capacity out of range")
        n = slots * capacity
        self.slots, self.capacity, self.channels = slots, capacity, channels
        self.pos = torch.zeros(n, 3, dtype=torch.float32, device=device)
        self.opacity = torch.zeros(n, dtype=torch.float32, device=device)
        self.feat = torch.zeros(n, channels, dtype=feat_dtype, device=device)
        self.radius = (torch.zeros(n, dtype=torch.float32, device=device) if with_radius
                       else None)
        self.counts: List[int] = [0] * slots
        self.next = 0  # the slot the next push overwrites (the oldest)

    def slot_range(self, s: int) -> slice:
        return slice(s * self.capacity, s * self.capacity + self.counts[s])

    def push(self, pos: torch.Tensor, opacity: torch.Tensor, feat: torch.Tensor,
             radius: Optional[torch.Tensor] = None) -> int:
        """Write a new cloud into the oldest slot (stream-ordered device
        copies); returns the slot index."""
        n = int(pos.shape[0])
        if n > self.capacity:
            raise ValueError(f"cloud of {n} points exceeds the slot capacity {self.capacity}")
        if opacity.shape != (n,) or feat.shape != (n, self.channels):
            raise ValueError("opacity must be [n] and feat [n, channels]")
        if (radius is None) != (self.radius is None):
            raise ValueError("radius must be given exactly when the ring holds radii")
        s = self.next
        b = s * self.capacity
        self.pos[b:b + n].copy_(pos)
        self.opacity[b:b + n].copy_(opacity)
        self.feat[b:b + n].copy_(feat)
        if radius is not None:
            self.radius[b:b + n].copy_(radius)
        self.counts[s] = n
        self.next = (s + 1) % self.slots
        return s

    def rasterize(self, camera, bg: Optional[torch.Tensor] = None,
                  settings: RasterSettings = RasterSettings(),
                  workspace: Optional[Workspace] = None):
        """Render the union of the ring's clouds (rasterize's outputs)."""
        return rasterize(self.pos, self.opacity, self.feat, camera, bg=bg, radius=self.radius,
                         settings=settings, workspace=workspace, ring_counts=self.counts)
