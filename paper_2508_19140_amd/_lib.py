"""ctypes binding of libinpc_raster.so (argument marshalling only).

The names mirror include/inpc_raster.h.  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libinpc_raster.so")

INPC_OK = 0
INPC_ERR_INVALID = -1
INPC_ERR_CAPACITY = -2
INPC_ERR_HIP = -3
INPC_ERR_UNSUPPORTED = -4

SPLAT_BILINEAR = 0
SPLAT_GAUSSIAN = 1
SPLAT_EWA = 2

DTYPE_F32 = 0
DTYPE_F16 = 1
DTYPE_BF16 = 2

STATIC_SCRATCH_BYTES = 64 << 20  # INPC_STATIC_SCRATCH_BYTES

EXPORTS = (
    "inpc_workspace_bytes", "inpc_state_bytes", "inpc_num_tiles", "inpc_copy_capacity",
    "inpc_project", "inpc_bin", "inpc_sort", "inpc_blend_forward", "inpc_blend_backward",
    "inpc_project_backward", "inpc_check_sync", "inpc_status_string", "inpc_last_error",
    "inpc_backward_scratch_bytes", "inpc_blend_backward_noalloc", "inpc_project_ring",
    "inpc_view_dirs", "inpc_envmap_forward", "inpc_envmap_backward",
    "inpc_batch_workspace_bytes", "inpc_rasterize_batched",
    "inpc_sh_features", "inpc_sh_features_backward",
    "inpc_backward_zero", "inpc_blend_backward_prezeroed",
)

PASS_FORWARD = 0
PASS_BACKWARD = 1


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("z_near", ctypes.c_float)]


class Opts(ctypes.Structure):
    _fields_ = [("splat", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("t_min", ctypes.c_float), ("dilation", ctypes.c_float),
                ("cutoff", ctypes.c_float), ("max_radius", ctypes.c_float),
                ("bin_points", ctypes.c_int32), ("bg_per_pixel", ctypes.c_int32),
                ("ewa_sigma", ctypes.c_float)]


_VP = ctypes.c_void_p


class ViewRecord(ctypes.Structure):
    """inpc_view_t: one view of a batch (camera, points and its buffers)."""
    _fields_ = [("cam", Camera), ("n", ctypes.c_int64),
                ("pos", _VP), ("opacity", _VP), ("radius", _VP), ("feat", _VP), ("bg", _VP),
                ("proj", _VP), ("depth_key", _VP), ("ntiles", _VP), ("tile_ranges", _VP),
                ("tile_order", _VP), ("list", _VP), ("lpos", _VP), ("state", _VP),
                ("ws", _VP), ("ws_bytes", ctypes.c_size_t),
                ("scratch", _VP), ("scratch_bytes", ctypes.c_size_t),
                ("out", _VP), ("t_final", _VP), ("n_contrib", _VP),
                ("grad_out", _VP), ("grad_t", _VP), ("grad_feat", _VP), ("grad_opacity", _VP),
                ("grad_uv", _VP), ("grad_pos", _VP), ("grad_bg", _VP), ("grad_z", _VP),
                ("ring_slots", ctypes.c_int32), ("ring_counts", _VP)]


class InpcError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {msg} (status {status})")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2508_19140_amd.build` "
            "(there is no non-HIP fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    CP, OP = ctypes.POINTER(Camera), ctypes.POINTER(Opts)
    sig = {
        "inpc_workspace_bytes": (SZ, [I64, CP, OP]),
        "inpc_state_bytes": (SZ, [CP, OP]),
        "inpc_num_tiles": (I64, [CP, OP]),
        "inpc_copy_capacity": (I64, [I64, CP, OP]),
        "inpc_project": (I32, [CP, OP, I64, P, P, P, P, P, P, P, SZ, P]),
        "inpc_project_ring": (I32, [CP, OP, I32, I64, P, P, P, P, P, P, P, P, SZ, P]),
        "inpc_bin": (I32, [CP, OP, I64, P, P, P, P, P, P, SZ, P]),
        "inpc_sort": (I32, [CP, OP, I64, P, P, P, P, P, P, SZ, P]),
        "inpc_blend_forward": (I32, [CP, OP, I64, P, P, I32, I32, P, P, P, P, P, P, P, P, P,
                                     P, SZ, P]),
        "inpc_blend_backward": (I32, [CP, OP, I64, P, P, I32, I32, P, P, P, P, P, P, P, P, P,
                                      P, P, P, P, P, P, P, SZ, P, SZ, P]),
        "inpc_blend_backward_prezeroed": (I32, [CP, OP, I64, P, P, I32, I32, P, P, P, P, P, P,
                                                P, P, P, P, P, P, P, P, P, P, SZ, P, SZ, P]),
        "inpc_backward_zero": (I32, [I64, I32, P, P, SZ, P]),
        "inpc_blend_backward_noalloc": (I32, [CP, OP, I64, P, P, I32, I32, P, P, P, P, P, P, P,
                                              P, P, P, P, P, P, P, P, P, SZ, P]),
        "inpc_backward_scratch_bytes": (SZ, [I64, I32, CP, OP]),
        "inpc_view_dirs": (I32, [CP, P, P]),
        "inpc_envmap_forward": (I32, [CP, P, P, I32, I32, I32, P, P]),
        "inpc_envmap_backward": (I32, [CP, P, P, I32, I32, I32, P, P]),
        "inpc_sh_features": (I32, [CP, I64, P, P, I32, P, P]),
        "inpc_sh_features_backward": (I32, [CP, I64, P, P, I32, P, P, P, P]),
        "inpc_batch_workspace_bytes": (SZ, [ctypes.POINTER(ViewRecord), I32, OP]),
        "inpc_rasterize_batched": (I32, [ctypes.POINTER(ViewRecord), P, I32, OP, I32, I32, I32,
                                         P, SZ, P]),
        "inpc_project_backward": (I32, [CP, I64, P, P, P, P, P, P]),
        "inpc_check_sync": (I32, [P, SZ, P]),
        "inpc_status_string": (ctypes.c_char_p, [I32]),
        "inpc_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int, func: str):
    if status != INPC_OK:
        L = lib()
        raise InpcError(status, func, L.inpc_last_error().decode() or
                        L.inpc_status_string(status).decode())


def call(name: str, *args):
    """Call an entry point that returns a status and raise on failure."""
    check(getattr(lib(), name)(*args), name)


def make_camera(width, height, fx, fy, cx, cy, R, t, z_near=0.2) -> Camera:
    c = Camera()
    c.width, c.height = int(width), int(height)
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    R = [float(x) for x in R]
    t = [float(x) for x in t]
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = t[k]
    c.z_near = float(z_near)
    return c


def make_opts(splat=SPLAT_BILINEAR, tile=8, t_min=1e-4, dilation=0.16, cutoff=3.0,
              max_radius=0.0, bin_points=0, bg_per_pixel=False, ewa_sigma=0.0) -> Opts:
    o = Opts()
    o.bin_points = int(bin_points)
    o.bg_per_pixel = int(bool(bg_per_pixel))
    o.ewa_sigma = float(ewa_sigma)
    o.splat, o.tile = int(splat), int(tile)
    o.t_min, o.dilation, o.cutoff, o.max_radius = float(t_min), float(dilation), float(cutoff), \
        float(max_radius)
    return o
