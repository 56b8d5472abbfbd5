"""PyTorch front end of the HIP rasterizer.

PyTorch provides device memory and the current stream; every step of the
rasterizer runs in the HIP library (libinpc_raster.so) through the C ABI.

    out, t_final, n_contrib = rasterize(pos, opacity, feat, camera)

`rasterize` is differentiable with respect to positions, opacities, features
and the background, for every splat kind (bilinear 2x2 splats, screen-space
Gaussians of a given radius, world-space Gaussians projected with the EWA
approximation).  The backward pass re-runs project / bin / sort instead of
keeping the tile lists (set keep_lists=True to keep them), and reads only a
12-byte per-pixel state saved by the forward pass.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Callable, Dict, NamedTuple, Optional, Sequence

import torch

from . import _lib as L

_DTYPES = {torch.float32: L.DTYPE_F32, torch.float16: L.DTYPE_F16, torch.bfloat16: L.DTYPE_BF16}


_SPLATS = {"bilinear": L.SPLAT_BILINEAR, "gaussian": L.SPLAT_GAUSSIAN, "ewa": L.SPLAT_EWA}


@dataclasses.dataclass(frozen=True)
class RasterSettings:
    splat: str = "bilinear"     # "bilinear" (2x2 splats), "gaussian" (screen-space, per-point
                                # radius in pixels) or "ewa" (world-space, one sigma)
    tile: int = 8               # 8, 16 or 32 pixels
    t_min: float = 1e-4         # blend fragment k iff transmittance in front of it >= t_min
    dilation: float = 0.16      # Gaussian dilation variance
    cutoff: float = 3.0         # Gaussian truncation in standard deviations
    max_radius: float = 3.0     # largest screen-space Gaussian radius (px); sizes the workspace
                                # ("ewa" derives its bound from the camera and sigma)
    keep_lists: bool = False    # keep tile lists for the backward instead of recomputing
    bin_points: int = 0         # points per workgroup of the binning passes (0 = automatic)
    ewa_sigma: float = 0.0      # "ewa": world-space standard deviation; 0 = the paper's
                                # default, 5 px at the near plane through the image centre
    ewa_px: float = 5.0         # that default's width in pixels
    ewa_max_radius: float = 0.0  # "ewa": workspace bound on the projected standard deviation
                                 # (px); 0 = derived from the camera and sigma

    def sigma(self, cam: L.Camera) -> float:
        """World-space standard deviation of "ewa" splats for this camera."""
        if self.ewa_sigma > 0.0:
            return float(self.ewa_sigma)
        return self.ewa_px * float(cam.z_near) / max(float(cam.fx), float(cam.fy))

    def opts(self, bg_per_pixel: bool = False, cam: Optional[L.Camera] = None) -> L.Opts:
        splat = _SPLATS[self.splat]
        max_radius, sigma = self.max_radius, 0.0
        if splat == L.SPLAT_EWA:
            if cam is None:
                raise ValueError("world-space Gaussians need the camera for their options")
            sigma = self.sigma(cam)
            max_radius = (self.ewa_max_radius if self.ewa_max_radius > 0.0 else
                          ewa_max_radius(cam, sigma, self.dilation, self.cutoff))
        return L.make_opts(splat, self.tile, self.t_min, self.dilation, self.cutoff,
                           max_radius, self.bin_points, bg_per_pixel, sigma)


def ewa_max_radius(cam: L.Camera, sigma: float, dilation: float, cutoff: float) -> float:
    """Bound on the projected standard deviation (pixels, before dilation) of
    a world-space Gaussian of standard deviation sigma in front of the near
    plane whose footprint meets the image: sqrt(sigma^2 (f/Z)^2 (1 + (x/Z)^2))
    with Z >= z_near and the offset |u - c| at most the image's reach plus the
    footprint's own half-width (a fixed point, reached in a few steps)."""
    zn = max(float(cam.z_near), 1e-12)
    bound = 0.0
    for f, c, size in ((float(cam.fx), float(cam.cx), cam.width),
                       (float(cam.fy), float(cam.cy), cam.height)):
        reach = max(abs(c), abs(size - c)) + 1.0
        r = sigma * f / zn
        for _ in range(32):
            m = (reach + cutoff * math.sqrt(r * r + dilation)) / f
            r_new = sigma * f / zn * math.sqrt(1.0 + m * m)
            if r_new <= r * (1.0 + 1e-9):
                r = r_new
                break
            r = r_new
        bound = max(bound, r)
    return bound * 1.001 + 1e-6


def camera_struct(cam) -> L.Camera:
    """Accepts an object with width, height, fx, fy, cx, cy, R (3x3), t (3),
    z_near attributes (for example scenes.Camera) or an L.Camera."""
    if isinstance(cam, L.Camera):
        return cam
    R = torch.as_tensor(cam.R, dtype=torch.float32).reshape(-1).tolist()
    t = torch.as_tensor(cam.t, dtype=torch.float32).reshape(-1).tolist()
    return L.make_camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, R, t,
                         getattr(cam, "z_near", 0.2))


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Workspace:
    """Device scratch for one rasterizer: grown on demand, reused across calls.

    A workspace holds the tile buckets, counters and the sticky overflow flag
    of the calls made with it, so calls that may run concurrently (on
    different streams) must not share one."""

    def __init__(self):
        self.buf: Optional[torch.Tensor] = None

    def get(self, n: int, cam: L.Camera, opts: L.Opts, device) -> torch.Tensor:
        size = int(L.lib().inpc_workspace_bytes(n, ctypes.byref(cam), ctypes.byref(opts)))
        if size == 0:
            raise ValueError("invalid camera or rasterizer settings")
        if self.buf is None or self.buf.numel() < size or self.buf.device != torch.device(device):
            self.buf = None
            # zeroed: the overflow flag at its start must begin cleared
            self.buf = torch.zeros(size, dtype=torch.uint8, device=device)
        return self.buf


_default_ws = {}


def default_workspace(device) -> Workspace:
    """The workspace of the current stream on `device` (one per stream, so
    that calls issued on different streams never share buckets or flags)."""
    dev = torch.device(device)
    key = (str(dev), torch.cuda.current_stream(dev).cuda_stream)
    if key not in _default_ws:
        _default_ws[key] = Workspace()
    return _default_ws[key]


class Binning(NamedTuple):
    proj: torch.Tensor      # [n, 4] f32 (u, v, opacity, radius)
    key: torch.Tensor       # [n] depth keys (int32 storage of u32)
    ntiles: torch.Tensor    # [n] tiles touched (int32 storage of u32), 0 = culled
    ranges: torch.Tensor    # [num_tiles + 1] (int32 storage of u32)
    list: torch.Tensor      # [copy capacity] point indices (int32 storage of u32)
    order: torch.Tensor     # [num_tiles] blend order, longest tiles first
    lpos: torch.Tensor      # [copy capacity] tile-local splat corner per list entry (int16
                            # storage of u16; bilinear splats)


def project_bin_sort(pos: torch.Tensor, opacity: torch.Tensor, cam: L.Camera, opts: L.Opts,
                     ws: torch.Tensor, radius: Optional[torch.Tensor] = None,
                     ring_counts: Optional[Sequence[int]] = None,
                     before_sort: Optional[Callable[[], None]] = None) -> Binning:
    """Steps 1-3: project, bin into tiles, sort every tile by (depth, index).
    ring_counts: the points are a ring of len(ring_counts) equal slots whose
    first ring_counts[s] points are live (inpc_project_ring).
    before_sort: called after the binning is issued and before the sort."""
    dev = pos.device
    n = pos.shape[0]
    lib = L.lib()
    nt = int(lib.inpc_num_tiles(ctypes.byref(cam), ctypes.byref(opts)))
    cap = int(lib.inpc_copy_capacity(n, ctypes.byref(cam), ctypes.byref(opts)))
    proj = torch.empty(n, 4, dtype=torch.float32, device=dev)
    key = torch.empty(n, dtype=torch.int32, device=dev)
    ntiles = torch.empty(n, dtype=torch.int32, device=dev)
    ranges = torch.empty(nt + 1, dtype=torch.int32, device=dev)
    order = torch.empty(max(nt, 1), dtype=torch.int32, device=dev)
    lst = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    lpos = torch.empty(max(cap, 1), dtype=torch.int16, device=dev)
    s = _stream(dev)
    cb, ob = ctypes.byref(cam), ctypes.byref(opts)
    wsb = ws.numel()
    if ring_counts is None:
        L.call("inpc_project", cb, ob, n, _p(pos), _p(opacity), _p(radius), _p(proj), _p(key),
               _p(ntiles), _p(ws), wsb, s)
    else:
        k = len(ring_counts)
        if k < 1 or n % k:
            raise ValueError("a ring's point count must be slots * slot capacity")
        counts = (ctypes.c_int64 * k)(*[int(c) for c in ring_counts])
        L.call("inpc_project_ring", cb, ob, k, n // k, counts, _p(pos), _p(opacity), _p(radius),
               _p(proj), _p(key), _p(ntiles), _p(ws), wsb, s)
    L.call("inpc_bin", cb, ob, n, _p(proj), _p(key), _p(ntiles), _p(ranges), _p(order), _p(ws),
           wsb, s)
    if before_sort is not None:
        before_sort()
    L.call("inpc_sort", cb, ob, n, _p(proj), _p(ranges), _p(order), _p(lst), _p(lpos), _p(ws),
           wsb, s)
    return Binning(proj, key, ntiles, ranges, lst, order, lpos)


def blend_forward(b: Binning, feat, cam: L.Camera, opts: L.Opts, ws: torch.Tensor, bg=None,
                  with_state=True):
    """Step 4.  Returns out [C,H,W], t_final [H,W], n_contrib [H,W], state."""
    dev = feat.device
    n, C = feat.shape
    H, W = cam.height, cam.width
    out = torch.empty(C, H, W, dtype=torch.float32, device=dev)
    t_final = torch.empty(H, W, dtype=torch.float32, device=dev)
    n_contrib = torch.empty(H, W, dtype=torch.int32, device=dev)
    state = None
    if with_state:
        state = torch.empty(int(L.lib().inpc_state_bytes(ctypes.byref(cam), ctypes.byref(opts))),
                            dtype=torch.uint8, device=dev)
    L.call("inpc_blend_forward", ctypes.byref(cam), ctypes.byref(opts), n, _p(b.proj), _p(feat),
           C, _DTYPES[feat.dtype], _p(bg), _p(b.ranges), _p(b.order), _p(b.list),
           _p(b.lpos if opts.splat == L.SPLAT_BILINEAR else None), _p(out), _p(t_final),
           _p(n_contrib), _p(state), _p(ws), ws.numel(), _stream(dev))
    return out, t_final, n_contrib, state


def backward_scratch_bytes(n: int, C: int, cam: L.Camera, opts: L.Opts) -> int:
    return int(L.lib().inpc_backward_scratch_bytes(n, C, ctypes.byref(cam), ctypes.byref(opts)))


class BlendGrads(NamedTuple):
    feat: torch.Tensor               # [n, C] f32
    opacity: torch.Tensor            # [n]
    uv: torch.Tensor                 # [n, 2]
    z: Optional[torch.Tensor]        # [n] dL/dZ at fixed (u, v) (world-space Gaussians)
    bg: Optional[torch.Tensor]       # like bg


def blend_backward(b: Binning, feat, cam: L.Camera, opts: L.Opts, ws: torch.Tensor, t_final,
                   state, grad_out, grad_t=None, bg=None, scratch=None,
                   outputs=None, prezeroed=False) -> BlendGrads:
    """Step 5.  Returns BlendGrads (grad_z only for world-space Gaussians).
    outputs: optional preallocated (grad_feat, grad_opacity, grad_uv); every element is
    overwritten.  prezeroed: grad_feat and scratch were zeroed by zero_backward_ahead,
    ordered before this call (then both must be given)."""
    if prezeroed and (outputs is None or scratch is None):
        raise ValueError("prezeroed needs the zeroed outputs and scratch")
    dev = feat.device
    n, C = feat.shape
    if outputs is not None:
        grad_feat, grad_opacity, grad_uv = outputs
        if (grad_feat.shape != (n, C) or grad_opacity.shape != (n,) or grad_uv.shape != (n, 2)
                or any(t.dtype != torch.float32 or not t.is_contiguous() for t in outputs)):
            raise ValueError("outputs must be contiguous f32 [n,C], [n], [n,2]")
        if n > 0 and (grad_feat.data_ptr() % 16 or grad_uv.data_ptr() % 8):
            raise ValueError("grad_feat must be 16-byte and grad_uv 8-byte aligned")
    else:
        grad_feat = torch.empty(n, C, dtype=torch.float32, device=dev)
        grad_opacity = torch.empty(n, dtype=torch.float32, device=dev)
        grad_uv = torch.empty(n, 2, dtype=torch.float32, device=dev)
    grad_bg = torch.empty(bg.shape, dtype=torch.float32, device=dev) if bg is not None else None
    grad_z = (torch.empty(n, dtype=torch.float32, device=dev) if opts.splat == L.SPLAT_EWA
              else None)
    if scratch is None:
        scratch = torch.empty(backward_scratch_bytes(n, C, cam, opts), dtype=torch.uint8,
                              device=dev)
    entry = "inpc_blend_backward_prezeroed" if prezeroed else "inpc_blend_backward"
    L.call(entry, ctypes.byref(cam), ctypes.byref(opts), n, _p(b.proj), _p(feat),
           C, _DTYPES[feat.dtype], _p(bg), _p(b.ntiles), _p(b.ranges), _p(b.order), _p(b.list),
           _p(b.lpos), _p(t_final), _p(state), _p(grad_out), _p(grad_t), _p(grad_feat),
           _p(grad_opacity), _p(grad_uv), _p(grad_z), _p(grad_bg), _p(scratch), scratch.numel(),
           _p(ws), ws.numel(), _stream(dev))
    return BlendGrads(grad_feat, grad_opacity, grad_uv, grad_z, grad_bg)


_zero_streams: Dict[str, torch.cuda.Stream] = {}


def zero_backward_ahead(grad_feat: torch.Tensor, scratch: torch.Tensor) -> torch.cuda.Event:
    """The backward blend's zero fill (inpc_backward_zero) on a side stream of
    the device (default priority), forked off the current stream: it runs
    beside whatever the current stream does next.  Returns the event the
    current stream must wait on before blend_backward(..., prezeroed=True)."""
    dev = grad_feat.device
    cur = torch.cuda.current_stream(dev)
    side = _zero_streams.get(str(dev))
    if side is None:
        side = _zero_streams[str(dev)] = torch.cuda.Stream(device=dev)
    fork, join = torch.cuda.Event(), torch.cuda.Event()
    fork.record(cur)
    side.wait_event(fork)
    n, C = grad_feat.shape
    L.call("inpc_backward_zero", n, C, _p(grad_feat), _p(scratch), scratch.numel(),
           ctypes.c_void_p(side.cuda_stream))
    join.record(side)
    return join


def project_backward(pos, b: Binning, cam: L.Camera, grad_uv, grad_z=None):
    """Step 6.  Returns grad_pos [n, 3] (grad_z: the blend's dL/dZ, world-space Gaussians)."""
    grad_pos = torch.empty_like(pos)
    L.call("inpc_project_backward", ctypes.byref(cam), pos.shape[0], _p(pos), _p(b.ntiles),
           _p(grad_uv), _p(grad_z), _p(grad_pos), _stream(pos.device))
    return grad_pos


def check_capacity(ws: torch.Tensor):
    """Synchronises the current stream and raises if a kernel ran out of copy capacity."""
    L.call("inpc_check_sync", _p(ws), ws.numel(), _stream(ws.device))


def _check_inputs(pos, opacity, feat, bg, radius, settings):
    if not pos.is_cuda:
        raise ValueError("rasterize runs on the GPU: inputs must be device tensors")
    if pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be float32 [N, 3]")
    n = pos.shape[0]
    if opacity.dtype != torch.float32 or opacity.shape != (n,):
        raise ValueError("opacity must be float32 [N]")
    if feat.dim() != 2 or feat.shape[0] != n or feat.dtype not in _DTYPES:
        raise ValueError("feat must be [N, C] float32 / float16 / bfloat16")
    C = feat.shape[1]
    if bg is not None and (bg.dtype != torch.float32 or bg.dim() not in (1, 3)
                           or bg.shape[0] != C):
        raise ValueError("bg must be float32 [C] or a per-pixel image [C, H, W]")
    if settings.splat not in _SPLATS:
        raise ValueError(f"unknown splat kind {settings.splat!r}")
    if settings.splat == "gaussian":
        if radius is None or radius.dtype != torch.float32 or radius.shape != (n,):
            raise ValueError("screen-space Gaussian splats need radius float32 [N]")


class _RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, opacity, feat, bg, radius, cam, settings, workspace, ring_counts):
        bg_image = bg is not None and bg.dim() == 3
        if bg_image and tuple(bg.shape[1:]) != (cam.height, cam.width):
            raise ValueError("a background image must be [C, H, W] of the camera's size")
        opts = settings.opts(bg_image, cam)
        ws = workspace.get(pos.shape[0], cam, opts, pos.device)
        if settings.splat != "gaussian":
            radius = None
        b = project_bin_sort(pos, opacity, cam, opts, ws, radius, ring_counts)
        out, t_final, n_contrib, state = blend_forward(b, feat, cam, opts, ws, bg)
        if settings.splat != "bilinear":
            # Gaussians wider than settings.max_radius can make more tile
            # copies than the workspace holds; the kernels then skip their
            # work, so the outputs must not be returned (one sync; bilinear
            # splats make at most four copies per point and cannot overflow)
            check_capacity(ws)
        ctx.cam, ctx.settings, ctx.workspace = cam, settings, workspace
        ctx.ring_counts = ring_counts
        ctx.has_bg, ctx.bg_image = bg is not None, bg_image
        empty = torch.empty(0, device=pos.device)
        saved = [pos, opacity, feat, bg if bg is not None else empty, t_final, state,
                 radius if radius is not None else empty]
        if settings.keep_lists:
            saved += list(b)
        ctx.save_for_backward(*saved)
        ctx.mark_non_differentiable(n_contrib)
        return out, t_final, n_contrib

    @staticmethod
    def backward(ctx, g_out, g_t, _g_n):
        saved = ctx.saved_tensors
        pos, opacity, feat, bg, t_final, state, radius = saved[:7]
        bg = bg if ctx.has_bg else None
        radius = radius if ctx.settings.splat == "gaussian" else None
        cam, opts = ctx.cam, ctx.settings.opts(ctx.bg_image, ctx.cam)
        ws = ctx.workspace.get(pos.shape[0], cam, opts, pos.device)
        n, C = feat.shape
        dev = pos.device
        outs = (torch.empty(n, C, dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.float32, device=dev),
                torch.empty(n, 2, dtype=torch.float32, device=dev))
        scratch = torch.empty(backward_scratch_bytes(n, C, cam, opts), dtype=torch.uint8,
                              device=dev)
        joined = []
        # the zero fill runs beside the tile sort (bound by LDS and latency);
        # under graph capture it stays inside the backward blend
        ahead = not torch.cuda.is_current_stream_capturing()
        fork = (lambda: joined.append(zero_backward_ahead(outs[0], scratch))) if ahead else None
        if ctx.settings.keep_lists:
            b = Binning(*saved[7:])
            if fork is not None:
                fork()
        else:
            b = project_bin_sort(pos, opacity, cam, opts, ws, radius, ctx.ring_counts,
                                 before_sort=fork)
        g_out = g_out.contiguous() if g_out is not None else torch.zeros(
            feat.shape[1], cam.height, cam.width, device=pos.device)
        g_t = g_t.contiguous() if g_t is not None else None
        if joined:
            torch.cuda.current_stream(dev).wait_event(joined[0])
        gr = blend_backward(b, feat, cam, opts, ws, t_final, state, g_out, g_t, bg,
                            scratch=scratch, outputs=outs, prezeroed=bool(joined))
        gpos = project_backward(pos, b, cam, gr.uv, gr.z)
        gf = gr.feat if feat.dtype == torch.float32 else gr.feat.to(feat.dtype)
        # screen-space radii are inputs without a gradient (as in the paper's inference use)
        return gpos, gr.opacity, gf, gr.bg, None, None, None, None, None


def view_directions(camera, device) -> torch.Tensor:
    """[H, W, 3] unit camera-space view directions through the pixel centres
    (they depend only on the intrinsics: compute once and keep)."""
    cam = camera_struct(camera)
    dirs = torch.empty(cam.height, cam.width, 3, dtype=torch.float32, device=device)
    L.call("inpc_view_dirs", ctypes.byref(cam), _p(dirs), _stream(dirs.device))
    return dirs


class _EnvMapFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, env, dirs, cam):
        Hm, Wm, C = env.shape
        bg = torch.empty(C, cam.height, cam.width, dtype=torch.float32, device=env.device)
        L.call("inpc_envmap_forward", ctypes.byref(cam), _p(dirs), _p(env), Hm, Wm, C, _p(bg),
               _stream(env.device))
        ctx.save_for_backward(dirs)
        ctx.cam, ctx.shape = cam, (Hm, Wm, C)
        return bg

    @staticmethod
    def backward(ctx, g):
        (dirs,) = ctx.saved_tensors
        Hm, Wm, C = ctx.shape
        grad_env = torch.empty(Hm, Wm, C, dtype=torch.float32, device=dirs.device)
        L.call("inpc_envmap_backward", ctypes.byref(ctx.cam), _p(dirs), _p(g.contiguous()), Hm,
               Wm, C, _p(grad_env), _stream(dirs.device))
        return grad_env, None, None


def envmap_background(env: torch.Tensor, camera, dirs: Optional[torch.Tensor] = None):
    """Background image [C, H, W] sampled from a spherical environment map
    env [Hm, Wm, C] (equirectangular, bilinear) along every pixel's view
    direction; differentiable with respect to env.  Pass it to rasterize()
    as `bg` to composite it behind the points (F += T_final f_bg)."""
    if env.dtype != torch.float32 or env.dim() != 3 or not env.is_cuda:
        raise ValueError("env must be a float32 [Hm, Wm, C] device tensor")
    cam = camera_struct(camera)
    if dirs is None:
        dirs = view_directions(cam, env.device)
    if dirs.shape != (cam.height, cam.width, 3) or dirs.dtype != torch.float32:
        raise ValueError("dirs must be float32 [H, W, 3]")
    return _EnvMapFn.apply(env.contiguous(), dirs.contiguous(), cam)


class _ShFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, sh, cam):
        n, C, _ = sh.shape
        feat = torch.empty(n, C, dtype=torch.float32, device=pos.device)
        L.call("inpc_sh_features", ctypes.byref(cam), n, _p(pos), _p(sh), C, _p(feat),
               _stream(pos.device))
        ctx.save_for_backward(pos, sh)
        ctx.cam = cam
        return feat

    @staticmethod
    def backward(ctx, g):
        pos, sh = ctx.saved_tensors
        n, C, _ = sh.shape
        grad_sh = torch.empty_like(sh)
        grad_pos = torch.empty_like(pos) if ctx.needs_input_grad[0] else None
        L.call("inpc_sh_features_backward", ctypes.byref(ctx.cam), n, _p(pos), _p(sh), C,
               _p(g.contiguous()), _p(grad_sh), _p(grad_pos), _stream(pos.device))
        return grad_pos, grad_sh, None


def sh_features(pos: torch.Tensor, sh: torch.Tensor, camera) -> torch.Tensor:
    """View-dependent features [N, C] from degree-2 spherical-harmonics
    coefficients sh [N, C, 9] at every point's view direction (from the
    camera centre to the point); differentiable in sh and pos.  Its output
    is the `feat` of rasterize()."""
    if (not pos.is_cuda or pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3
            or sh.dtype != torch.float32 or sh.dim() != 3 or sh.shape[0] != pos.shape[0]
            or sh.shape[2] != 9):
        raise ValueError("pos must be float32 [N, 3] and sh float32 [N, C, 9] device tensors")
    return _ShFn.apply(pos.contiguous(), sh.contiguous(), camera_struct(camera))


def rasterize(pos: torch.Tensor, opacity: torch.Tensor, feat: torch.Tensor, camera,
              bg: Optional[torch.Tensor] = None, radius: Optional[torch.Tensor] = None,
              settings: RasterSettings = RasterSettings(),
              workspace: Optional[Workspace] = None,
              ring_counts: Optional[Sequence[int]] = None):
    """Render a feature image.

    pos [N,3] f32, opacity [N] f32 in [0,1], feat [N,C] f32/f16/bf16,
    bg [C] f32, a per-pixel background [C,H,W] f32 (e.g. envmap_background)
    or None, radius [N] f32 (screen-space Gaussian splats).
    ring_counts: the N points are a ring of len(ring_counts) equal slots of
    which slot s holds ring_counts[s] live points at its start (PointRing);
    the union of the live points is rendered, the rest is ignored.
    Returns out [C,H,W] f32, t_final [H,W] f32, n_contrib [H,W] int32.
    """
    _check_inputs(pos, opacity, feat, bg, radius, settings)
    cam = camera_struct(camera)
    ws = workspace if workspace is not None else default_workspace(pos.device)
    feat = feat.contiguous()
    if feat.data_ptr() % 16:  # feature rows are read as 16-byte vectors
        feat = feat.clone()
    return _RasterizeFn.apply(pos.contiguous(), opacity.contiguous(), feat,
                              None if bg is None else bg.contiguous(),
                              None if radius is None else radius.contiguous(), cam, settings, ws,
                              None if ring_counts is None else tuple(int(c) for c in ring_counts))
