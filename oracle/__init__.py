"""CPU oracle for the INPC point rasterizer -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never does.

Two tiers, sharing nothing with the GPU path:
  * ``inpc_oracle.c`` (built to ``liboracle_inpc.so``): per-pixel fragment
    lists, sort by (depth key, point index), FP64 blending and gradients,
    FP32 decision arithmetic.  Wrapped here with ctypes.
  * ``brute.py``: an O(pixels x points) pure-Python brute force for tiny
    scenes, which pins the C tier.

Pins (tests/test_oracle_pins.py, test_oracle_brute.py, test_oracle_grad.py,
test_golden.py): projection and tile lists by closed-form tile counts per
sub-tile position and their mean (1 + 1/T)^2, by the partition and order of
the ranges, and by the brute force; the forward by closed forms for one,
two and three splats, alpha = 1 occlusion, a single Gaussian's profile,
telescoping, linearity and input-order invariance; the backward by torch
float64 autograd of Eq. (1) and by central finite differences.  Every
function here has a pin.  What the paper leaves open (pixel-centre
convention, near plane, termination threshold, tie-break by index, Gaussian
radius semantics, bounding-box tile membership) is a reading of this
implementation, not a printed value: parity unpinned by the paper for those
readings, which the pins exercise but cannot confirm.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "inpc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_inpc.so")

CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-fopenmp", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no FMA contraction, IEEE FP32)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("z_near", ctypes.c_float)]


class _Opts(ctypes.Structure):
    _fields_ = [("splat", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("t_min", ctypes.c_float), ("dilation", ctypes.c_float),
                ("cutoff", ctypes.c_float), ("ewa_sigma", ctypes.c_float)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_project.argtypes = [P, P, ctypes.c_int64, P, P, P, P, P, P, P, P]
        lib.oracle_project.restype = ctypes.c_int
        lib.oracle_tile_lists.argtypes = [P, P, ctypes.c_int64, P, P, P, P]
        lib.oracle_tile_lists.restype = ctypes.c_int64
        lib.oracle_render.argtypes = [P, P, ctypes.c_int64, P, P, P, P, ctypes.c_int32] + [P] * 18 \
            + [ctypes.c_int32, P, P]
        lib.oracle_render.restype = ctypes.c_int
        lib.oracle_count_fragments.argtypes = [P, P, ctypes.c_int64, P, P]
        lib.oracle_count_fragments.restype = ctypes.c_int64
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _cam(camera) -> _Cam:
    c = _Cam()
    c.width, c.height = int(camera.width), int(camera.height)
    c.fx, c.fy, c.cx, c.cy = float(camera.fx), float(camera.fy), float(camera.cx), float(camera.cy)
    R = np.asarray(camera.R, np.float32).reshape(-1)
    t = np.asarray(camera.t, np.float32).reshape(-1)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.z_near = float(camera.z_near)
    return c


SPLAT_BILINEAR = 0
SPLAT_GAUSSIAN = 1
SPLAT_EWA = 2  # world-space Gaussians of standard deviation ewa_sigma, EWA projection


def _opts(splat=SPLAT_BILINEAR, tile=8, t_min=1e-4, dilation=0.16, cutoff=3.0,
          ewa_sigma=0.0) -> _Opts:
    o = _Opts()
    o.splat, o.tile = int(splat), int(tile)
    o.t_min, o.dilation, o.cutoff = float(t_min), float(dilation), float(cutoff)
    o.ewa_sigma = float(ewa_sigma)
    return o


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    _load().oracle_set_num_threads(int(n))


def project(camera, pos, radius=None, splat=SPLAT_BILINEAR, tile=8, dilation=0.16, cutoff=3.0,
            ewa_sigma=0.0):
    """Decision stage per point: visibility, (u, v), depth key, camera-space
    coordinates, inclusive pixel rect of candidate fragments, tiles touched."""
    lib = _load()
    pos = _f32(pos, (-1, 3))
    n = pos.shape[0]
    rad = None if radius is None else _f32(radius, (n,))
    vis = np.zeros(n, np.uint8)
    uv = np.zeros((n, 2), np.float32)
    key = np.zeros(n, np.uint32)
    xyz = np.zeros((n, 3), np.float32)
    rect = np.zeros((n, 4), np.int32)
    nt = np.zeros(n, np.uint32)
    cam, o = _cam(camera), _opts(splat, tile, 0.0, dilation, cutoff, ewa_sigma)
    lib.oracle_project(ctypes.byref(cam), ctypes.byref(o), n, _ptr(pos), _ptr(rad), _ptr(vis),
                       _ptr(uv), _ptr(key), _ptr(xyz), _ptr(rect), _ptr(nt))
    return dict(visible=vis.astype(bool), uv=uv, key=key, xyz=xyz, rect=rect, ntiles=nt)


def tile_lists(camera, pos, radius=None, splat=SPLAT_BILINEAR, tile=8, dilation=0.16,
               cutoff=3.0, ewa_sigma=0.0):
    """Per-tile counts, ranges [nt+1] and concatenated lists ordered by
    (depth key, point index) inside each tile."""
    lib = _load()
    pos = _f32(pos, (-1, 3))
    n = pos.shape[0]
    rad = None if radius is None else _f32(radius, (n,))
    ntx = (camera.width + tile - 1) // tile
    nty = (camera.height + tile - 1) // tile
    counts = np.zeros(ntx * nty, np.uint32)
    cam, o = _cam(camera), _opts(splat, tile, 0.0, dilation, cutoff, ewa_sigma)
    total = lib.oracle_tile_lists(ctypes.byref(cam), ctypes.byref(o), n, _ptr(pos), _ptr(rad),
                                  _ptr(counts), None)
    lst = np.zeros(max(int(total), 1), np.uint32)
    lib.oracle_tile_lists(ctypes.byref(cam), ctypes.byref(o), n, _ptr(pos), _ptr(rad),
                          _ptr(counts), _ptr(lst))
    ranges = np.zeros(ntx * nty + 1, np.int64)
    ranges[1:] = np.cumsum(counts.astype(np.int64))
    return dict(counts=counts, ranges=ranges, list=lst[:int(total)], ntx=ntx, nty=nty)


def render(camera, pos, opacity, feat, radius=None, bg=None, splat=SPLAT_BILINEAR, tile=8,
           t_min=1e-4, dilation=0.16, cutoff=3.0, grad_out=None, grad_t=None, pixel_mask=None,
           ewa_sigma=0.0):
    """Forward (and, with grad_out, backward) render in FP64.

    feat is upcast exactly to float64 (FP16/BF16 values included).
    bg: [C] constant background features, or a per-pixel background image
    [C,H,W] (grad_bg then per pixel too).
    pixel_mask ([H,W] bool, forward only): compute only these pixels (each
    one exactly; the rest of the outputs stay zero), for scenes whose full
    fragment set would not fit in host memory.
    Returns a dict with out [C,H,W], out_abs, t_final [H,W], n_contrib, flags
    and, for the backward, grad_feat [N,C], grad_opacity [N], grad_uv [N,2],
    grad_pos [N,3], grad_bg [C] and their *_abs magnitude bounds.
    """
    lib = _load()
    pos = _f32(pos, (-1, 3))
    n = pos.shape[0]
    opacity = _f32(opacity, (n,))
    feat = np.ascontiguousarray(np.asarray(feat).astype(np.float64)).reshape(n, -1)
    C = feat.shape[1]
    rad = None if radius is None else _f32(radius, (n,))
    W, H = int(camera.width), int(camera.height)
    P = W * H
    bg_image = bg is not None and np.ndim(bg) == 3
    bgd = None if bg is None else np.ascontiguousarray(
        np.asarray(bg, np.float64).reshape((C, H, W) if bg_image else (C,)))
    r = dict(out=np.zeros((C, H, W)), out_abs=np.zeros((C, H, W)), t_final=np.zeros((H, W)),
             n_contrib=np.zeros((H, W), np.uint32), flags=np.zeros((H, W), np.uint8))
    go = gt = None
    if grad_out is not None:
        go = _f32(grad_out, (C, H, W))
        gt = None if grad_t is None else _f32(grad_t, (H, W))
        for k, shp in (("grad_feat", (n, C)), ("grad_opacity", (n,)), ("grad_uv", (n, 2)),
                       ("grad_pos", (n, 3))):
            r[k] = np.zeros(shp)
            r[k + "_abs"] = np.zeros(shp)
        r["grad_bg"] = (np.zeros((C, H, W) if bg_image else C) if bg is not None else None)
        r["grad_z"] = np.zeros(n)
        r["grad_z_abs"] = np.zeros(n)
    if pixel_mask is not None:
        if grad_out is not None:
            raise ValueError("pixel_mask is for the forward pass only")
        pixel_mask = np.ascontiguousarray(np.asarray(pixel_mask, bool).reshape(H, W), np.uint8)
    cam, o = _cam(camera), _opts(splat, tile, t_min, dilation, cutoff, ewa_sigma)
    g = r.get
    lib.oracle_render(ctypes.byref(cam), ctypes.byref(o), n, _ptr(pos), _ptr(rad), _ptr(opacity),
                      _ptr(feat), C, _ptr(bgd), _ptr(r["out"]), _ptr(r["out_abs"]),
                      _ptr(r["t_final"]), _ptr(r["n_contrib"]), _ptr(r["flags"]), _ptr(go),
                      _ptr(gt), _ptr(g("grad_feat")), _ptr(g("grad_opacity")), _ptr(g("grad_uv")),
                      _ptr(g("grad_pos")), _ptr(g("grad_bg")), _ptr(g("grad_feat_abs")),
                      _ptr(g("grad_opacity_abs")), _ptr(g("grad_uv_abs")),
                      _ptr(g("grad_pos_abs")), _ptr(pixel_mask), int(bg_image),
                      _ptr(g("grad_z")), _ptr(g("grad_z_abs")))
    return r


def count_fragments(camera, pos, radius=None, splat=SPLAT_BILINEAR, tile=8, dilation=0.16,
                    cutoff=3.0, ewa_sigma=0.0) -> int:
    lib = _load()
    pos = _f32(pos, (-1, 3))
    n = pos.shape[0]
    rad = None if radius is None else _f32(radius, (n,))
    cam, o = _cam(camera), _opts(splat, tile, 0.0, dilation, cutoff, ewa_sigma)
    return int(lib.oracle_count_fragments(ctypes.byref(cam), ctypes.byref(o), n, _ptr(pos),
                                          _ptr(rad)))


def within_tolerance(gpu, ref, ref_abs, rel=1e-5, abs_=1e-6):
    """Element-wise check |gpu - ref| <= abs_ + rel * max(|ref|, S_abs), where
    S_abs bounds the magnitudes of the terms the element accumulates (the
    usual floating-point summation error bound).  Returns (ok_mask, stats)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), np.asarray(ref_abs, np.float64))
    err = np.abs(gpu - ref)
    ok = err <= abs_ + rel * scale
    with np.errstate(divide="ignore", invalid="ignore"):
        relerr = np.where(np.abs(ref) > 0, err / np.abs(ref), 0.0)
    # the plain test against the value alone (no summation bound): reported,
    # not gated, because sums with cancellation (position gradients over
    # the four splat corners) can sit far below their terms
    plain_bad = err > abs_ + rel * np.abs(ref)
    stats = dict(max_abs=float(err.max(initial=0.0)),
                 max_rel=float(relerr.max(initial=0.0)),
                 rms=float(np.sqrt(np.mean(err ** 2))) if err.size else 0.0,
                 n_bad=int((~ok).sum()),
                 n_plain_fail=int(plain_bad.sum()),
                 max_plain_excess=float(((err - abs_) / np.maximum(np.abs(ref), 1e-300))[plain_bad]
                                        .max(initial=0.0)))
    return ok, stats
