"""Preallocated per-view pipelines, and many views in one HIP graph launch.

`ViewPipeline` owns every buffer of one view (the workspace, the tile lists,
the forward state, the gradients) and issues the C-ABI calls of one forward
and one backward pass on a given stream, allocating nothing.

`MultiViewRasterizer` runs a batch of views with uneven point counts and
resolutions as one training step: each view's forward + backward goes on a
stream of its own, the streams fork from and join back to one capture
stream, and the whole batch is captured once into a HIP graph, so a step is
a single graph launch.  Independent views overlap on the device (one view's
single-workgroup scan or longest tile runs beside another view's wide
kernels).  Before capture, an autotuner picks each view's tile size and
points per binning workgroup by timing the candidates on that view.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib as L
from .raster import RasterSettings, camera_struct

_DT = {torch.float32: L.DTYPE_F32, torch.float16: L.DTYPE_F16, torch.bfloat16: L.DTYPE_BF16}


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class ViewInputs:
    """Device tensors of one view: pos [n,3] f32, opacity [n] f32, feat
    [n,C] (f32/f16/bf16), camera (scenes.Camera or L.Camera), grad_out
    [C,H,W] f32 (upstream gradient of the feature image; None: forward only),
    radius [n] f32 for Gaussian splats."""
    pos: torch.Tensor
    opacity: torch.Tensor
    feat: torch.Tensor
    camera: object
    grad_out: Optional[torch.Tensor] = None
    radius: Optional[torch.Tensor] = None


class ViewPipeline:
    """All buffers and ABI calls of one view; nothing is allocated per call."""

    def __init__(self, v: ViewInputs, settings: RasterSettings):
        dev = v.pos.device
        self.v, self.settings = v, settings
        self.gauss = settings.splat == "gaussian"
        self.cam = camera_struct(v.camera)
        self.opts = settings.opts()
        self.cb, self.ob = ctypes.byref(self.cam), ctypes.byref(self.opts)
        lib = L.lib()
        self.lib = lib
        n, C = v.feat.shape
        self.n, self.C = n, C
        self.dtype = _DT[v.feat.dtype]
        nt = int(lib.inpc_num_tiles(self.cb, self.ob))
        cap = int(lib.inpc_copy_capacity(n, self.cb, self.ob))
        self.nt = nt
        wsb = int(lib.inpc_workspace_bytes(n, self.cb, self.ob))
        if wsb == 0:
            raise ValueError("invalid camera or settings")
        H, W = self.cam.height, self.cam.width
        mk = lambda *s, dt=torch.float32: torch.empty(*s, dtype=dt, device=dev)
        i32 = torch.int32
        self.ws = torch.zeros(wsb, dtype=torch.uint8, device=dev)  # overflow flag starts clear
        self.proj, self.key, self.ntiles = mk(n, 4), mk(n, dt=i32), mk(n, dt=i32)
        self.ranges, self.order = mk(nt + 1, dt=i32), mk(max(nt, 1), dt=i32)
        self.list, self.lpos = mk(max(cap, 1), dt=i32), mk(max(cap, 1), dt=torch.int16)
        self.out, self.tf, self.nc = mk(C, H, W), mk(H, W), mk(H, W, dt=i32)
        self.backward_enabled = v.grad_out is not None and not self.gauss
        self.state = None
        if not self.gauss:
            self.state = mk(int(lib.inpc_state_bytes(self.cb, self.ob)), dt=torch.uint8)
        if self.backward_enabled:
            self.gf, self.go, self.guv, self.gpos = mk(n, C), mk(n), mk(n, 2), mk(n, 3)
            self.scratch = mk(int(lib.inpc_backward_scratch_bytes(n, C, self.cb, self.ob)),
                              dt=torch.uint8)

    def _call(self, name, *args):
        st = getattr(self.lib, name)(*args)
        if st != L.INPC_OK:
            L.check(st, name)

    # one method per entry point, each on stream handle s
    def project(self, s):
        v, ws = self.v, self.ws
        self._call("inpc_project", self.cb, self.ob, self.n, _p(v.pos), _p(v.opacity),
                   _p(v.radius), _p(self.proj), _p(self.key), _p(self.ntiles), _p(ws),
                   ws.numel(), s)

    def bin(self, s):
        ws = self.ws
        self._call("inpc_bin", self.cb, self.ob, self.n, _p(self.proj), _p(self.key),
                   _p(self.ntiles), _p(self.ranges), _p(self.order), _p(ws), ws.numel(), s)

    def sort(self, s):
        ws = self.ws
        self._call("inpc_sort", self.cb, self.ob, self.n, _p(self.proj), _p(self.ranges),
                   _p(self.order), _p(self.list), _p(self.lpos), _p(ws), ws.numel(), s)

    def blend_fwd(self, s):
        v, ws = self.v, self.ws
        self._call("inpc_blend_forward", self.cb, self.ob, self.n, _p(self.proj), _p(v.feat),
                   self.C, self.dtype, None, _p(self.ranges), _p(self.order), _p(self.list),
                   None if self.gauss else _p(self.lpos), _p(self.out), _p(self.tf),
                   _p(self.nc), _p(self.state), _p(ws), ws.numel(), s)

    def blend_bwd(self, s):
        v, ws = self.v, self.ws
        self._call("inpc_blend_backward", self.cb, self.ob, self.n, _p(self.proj), _p(v.feat),
                   self.C, self.dtype, None, _p(self.ntiles), _p(self.ranges), _p(self.order),
                   _p(self.list), _p(self.lpos), _p(self.tf), _p(self.state), _p(v.grad_out),
                   None, _p(self.gf), _p(self.go), _p(self.guv), None, _p(self.scratch),
                   self.scratch.numel(), _p(ws), ws.numel(), s)

    def project_bwd(self, s):
        v = self.v
        self._call("inpc_project_backward", self.cb, self.n, _p(v.pos), _p(self.ntiles),
                   _p(self.guv), _p(self.gpos), s)

    def phases(self):
        """(entry point, fn(stream)) of one training pass: forward, then the
        backward with the lists recomputed (unless settings.keep_lists)."""
        ph = [("project", self.project), ("bin", self.bin), ("sort", self.sort),
              ("blend_fwd", self.blend_fwd)]
        if self.backward_enabled:
            if not self.settings.keep_lists:
                ph += [("project", self.project), ("bin", self.bin), ("sort", self.sort)]
            ph += [("blend_bwd", self.blend_bwd), ("project_bwd", self.project_bwd)]
        return ph

    def step(self, s):
        for _, f in self.phases():
            f(s)

    def outputs(self) -> Dict[str, torch.Tensor]:
        r = {"out": self.out, "t_final": self.tf, "n_contrib": self.nc}
        if self.backward_enabled:
            r.update(grad_feat=self.gf, grad_opacity=self.go, grad_uv=self.guv,
                     grad_pos=self.gpos)
        return r


def _handle(stream: torch.cuda.Stream):
    return ctypes.c_void_p(stream.cuda_stream)


def time_pipeline(p: ViewPipeline, reps: int = 3, warmup: int = 1) -> float:
    """Mean milliseconds of one step of p on the current stream."""
    s = torch.cuda.current_stream()
    h = _handle(s)
    for _ in range(warmup):
        p.step(h)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        p.step(h)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


class MultiViewRasterizer:
    """A fixed batch of views, autotuned per view and captured into one graph.

    tiles: candidate tile sizes (8 and 16; 32x32 tiles are not supported by
    the blend kernels).  bin_points: candidate points per binning workgroup
    (0 = the library's default).  cache: optional dict reused across
    instances, keyed by (width, height, n, C, dtype, splat)."""

    def __init__(self, views: Sequence[ViewInputs], settings: RasterSettings = RasterSettings(),
                 tiles: Sequence[int] = (8, 16), bin_points: Sequence[int] = (0, 2048, 4096),
                 autotune: bool = True, cache: Optional[dict] = None, reps: int = 3):
        self.views = list(views)
        self.base = settings
        self.cache = cache if cache is not None else {}
        self.choice: List[Tuple[int, int]] = []
        self.tuning: List[Dict[Tuple[int, int], float]] = []
        for v in self.views:
            cam = camera_struct(v.camera)
            key = (cam.width, cam.height, v.feat.shape[0], v.feat.shape[1], str(v.feat.dtype),
                   settings.splat)
            if key in self.cache:
                self.choice.append(self.cache[key])
                self.tuning.append({})
                continue
            if not autotune:
                self.choice.append((settings.tile, settings.bin_points))
                self.tuning.append({})
                continue
            times = {}
            for t in tiles:
                for bp in bin_points:
                    p = ViewPipeline(v, dataclasses.replace(settings, tile=t, bin_points=bp))
                    times[(t, bp)] = time_pipeline(p, reps=reps)
                    del p
            best = min(times, key=times.get)
            self.cache[key] = best
            self.choice.append(best)
            self.tuning.append(times)
        self.pipes = [ViewPipeline(v, dataclasses.replace(settings, tile=t, bin_points=bp))
                      for v, (t, bp) in zip(self.views, self.choice)]
        self.graph = None
        self.streams = None

    def run_eager(self, stream: Optional[torch.cuda.Stream] = None):
        """Every view in turn on one stream, no graph."""
        h = _handle(stream or torch.cuda.current_stream())
        for p in self.pipes:
            p.step(h)

    def capture(self):
        """Capture the whole batch (a fork per view, then a join) into one graph."""
        self.streams = [torch.cuda.Stream() for _ in self.pipes]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # warm-up outside capture, as torch requires
            self.run_eager(side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            cs = torch.cuda.current_stream()
            for p, st in zip(self.pipes, self.streams):
                st.wait_stream(cs)
                with torch.cuda.stream(st):
                    p.step(_handle(st))
            for st in self.streams:
                cs.wait_stream(st)
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def outputs(self) -> List[Dict[str, torch.Tensor]]:
        return [p.outputs() for p in self.pipes]
