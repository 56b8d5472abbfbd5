"""The C ABI library loads, exports every function include/inpc_raster.h
declares, and rejects bad arguments on the host before any launch (no GPU
needed: every call here returns before touching the device)."""
import ctypes
import os
import re

import pytest

from paper_2508_19140_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "inpc_raster.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(inpc_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def cam(w=64, h=48):
    return L.make_camera(w, h, 32.0, 32.0, w / 2, h / 2, [1, 0, 0, 0, 1, 0, 0, 0, 1], [0, 0, 0])


def test_workspace_and_sizes():
    lib = L.lib()
    c, o = cam(), L.make_opts(tile=8)
    assert lib.inpc_num_tiles(ctypes.byref(c), ctypes.byref(o)) == 8 * 6
    assert lib.inpc_copy_capacity(1000, ctypes.byref(c), ctypes.byref(o)) == 4000
    assert lib.inpc_state_bytes(ctypes.byref(c), ctypes.byref(o)) == 64 * 48 * 12 + 48 * 4
    ws = lib.inpc_workspace_bytes(1000, ctypes.byref(c), ctypes.byref(o))
    assert ws >= 4 * 4000 * 4
    assert lib.inpc_workspace_bytes(2000, ctypes.byref(c), ctypes.byref(o)) > ws
    # Gaussian capacity grows with the largest radius
    g1 = L.make_opts(splat=L.SPLAT_GAUSSIAN, tile=8, max_radius=1.0)
    g3 = L.make_opts(splat=L.SPLAT_GAUSSIAN, tile=8, max_radius=3.0)
    assert lib.inpc_copy_capacity(10, ctypes.byref(c), ctypes.byref(g3)) > \
        lib.inpc_copy_capacity(10, ctypes.byref(c), ctypes.byref(g1))
    # the binning workgroup size is a tuning knob: multiples of 1024 only; fewer
    # points per workgroup means more per-workgroup count rows
    o_small = L.make_opts(tile=8, bin_points=1024)
    big_n = 100_000
    assert lib.inpc_workspace_bytes(big_n, ctypes.byref(c), ctypes.byref(o_small)) > \
        lib.inpc_workspace_bytes(big_n, ctypes.byref(c), ctypes.byref(o))
    assert lib.inpc_workspace_bytes(10, ctypes.byref(c), ctypes.byref(L.make_opts(bin_points=1000))) == 0
    # invalid settings give 0
    assert lib.inpc_workspace_bytes(10, ctypes.byref(c), ctypes.byref(L.make_opts(tile=12))) == 0
    assert lib.inpc_workspace_bytes(-1, ctypes.byref(c), ctypes.byref(o)) == 0
    assert lib.inpc_num_tiles(ctypes.byref(cam(0, 10)), ctypes.byref(o)) == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: the calls fail before any launch


@pytest.mark.parametrize("case", ["null_cam", "bad_tile", "neg_n", "null_ws", "small_ws",
                                  "null_pos", "null_opacity", "gauss_no_radius",
                                  "misaligned_proj"])
def test_project_rejects_bad_arguments(case):
    lib = L.lib()
    c, o = cam(), L.make_opts(tile=8)
    n = 100
    ws_bytes = lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(o))
    args = dict(cam=ctypes.byref(c), opts=ctypes.byref(o), n=n, pos=FAKE, opacity=FAKE,
                radius=None, proj=FAKE, key=FAKE, ntiles=FAKE, ws=FAKE, ws_bytes=ws_bytes)
    if case == "null_cam":
        args["cam"] = None
    elif case == "bad_tile":
        args["opts"] = ctypes.byref(L.make_opts(tile=4))
    elif case == "neg_n":
        args["n"] = -5
    elif case == "null_ws":
        args["ws"] = None
    elif case == "small_ws":
        args["ws_bytes"] = ws_bytes - 1
    elif case == "null_pos":
        args["pos"] = None
    elif case == "null_opacity":
        args["opacity"] = None
    elif case == "misaligned_proj":
        args["proj"] = ctypes.c_void_p(0x1008)
    elif case == "gauss_no_radius":
        g = L.make_opts(splat=L.SPLAT_GAUSSIAN, max_radius=3.0)
        args["opts"] = ctypes.byref(g)
        args["ws_bytes"] = lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(g))
    st = lib.inpc_project(*args.values(), None)
    assert st == L.INPC_ERR_INVALID
    assert lib.inpc_last_error()


def test_blend_rejects_bad_channels_and_dtype():
    lib = L.lib()
    c, o = cam(), L.make_opts(tile=8)
    n = 10
    wsb = lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(o))
    base = [ctypes.byref(c), ctypes.byref(o), n, FAKE, FAKE]
    tail = [None, FAKE, None, FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, wsb, None]
    assert lib.inpc_blend_forward(*base, 0, L.DTYPE_F32, *tail) == L.INPC_ERR_INVALID
    assert lib.inpc_blend_forward(*base, 65, L.DTYPE_F32, *tail) == L.INPC_ERR_INVALID
    assert lib.inpc_blend_forward(*base, 4, 7, *tail) == L.INPC_ERR_INVALID
    assert lib.inpc_blend_forward(*base, 48, L.DTYPE_F32, *tail) == L.INPC_ERR_UNSUPPORTED


def test_world_space_gaussian_options_and_checks():
    """World-space (EWA) splats: sigma must be finite and positive; the
    workspace bound follows max_radius as for a screen-space Gaussian of that
    radius; the backward needs grad_z (and no lpos)."""
    lib = L.lib()
    c = cam()
    n = 10
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        o = L.make_opts(splat=L.SPLAT_EWA, max_radius=2.0, ewa_sigma=bad)
        assert lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(o)) == 0
    e = L.make_opts(splat=L.SPLAT_EWA, max_radius=2.0, ewa_sigma=0.01)
    g = L.make_opts(splat=L.SPLAT_GAUSSIAN, max_radius=2.0)
    wsb = lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(e))
    assert wsb > 0 and wsb == lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(g))
    assert lib.inpc_copy_capacity(n, ctypes.byref(c), ctypes.byref(e)) == \
        lib.inpc_copy_capacity(n, ctypes.byref(c), ctypes.byref(g))
    # backward: feat, ntiles, ranges, list, t_final, state, grad_out, grad_feat,
    # grad_opacity, grad_uv given; grad_z missing
    st = lib.inpc_blend_backward(ctypes.byref(c), ctypes.byref(e), n, FAKE, FAKE, 4,
                                 L.DTYPE_F32, None, FAKE, FAKE, None, FAKE, None, FAKE, FAKE,
                                 FAKE, None, FAKE, FAKE, FAKE, None, None, FAKE, 1 << 20, FAKE,
                                 wsb, None)
    assert st == L.INPC_ERR_INVALID and b"grad_z" in lib.inpc_last_error()
    # project: world-space splats take no radius, but still need the outputs
    st = lib.inpc_project(ctypes.byref(c), ctypes.byref(e), n, FAKE, FAKE, None, None, FAKE,
                          FAKE, FAKE, wsb, None)
    assert st == L.INPC_ERR_INVALID and b"proj" in lib.inpc_last_error()


def test_backward_rejects_small_scratch():
    lib = L.lib()
    c, o = cam(), L.make_opts(tile=8)
    n, C = 10, 4
    wsb = lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(o))
    need = lib.inpc_backward_scratch_bytes(n, C, ctypes.byref(c), ctypes.byref(o))
    nt = lib.inpc_num_tiles(ctypes.byref(c), ctypes.byref(o))
    assert need >= n * 16 + nt * C * 4  # scalar gradient rows, background shares
    args = [ctypes.byref(c), ctypes.byref(o), n, FAKE, FAKE, C, L.DTYPE_F32, None, FAKE,
            FAKE, None, FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, FAKE, None, None]
    assert lib.inpc_blend_backward(*args, FAKE, need - 1, FAKE, wsb, None) == L.INPC_ERR_INVALID
    assert lib.inpc_blend_backward(*args, None, need, FAKE, wsb, None) == L.INPC_ERR_INVALID


def test_sort_and_blend_require_lpos_for_bilinear():
    lib = L.lib()
    c, o = cam(), L.make_opts(tile=8)
    n = 10
    wsb = lib.inpc_workspace_bytes(n, ctypes.byref(c), ctypes.byref(o))
    st = lib.inpc_sort(ctypes.byref(c), ctypes.byref(o), n, FAKE, FAKE, None, FAKE, None, FAKE,
                       wsb, None)
    assert st == L.INPC_ERR_INVALID and b"lpos" in lib.inpc_last_error()
    st = lib.inpc_blend_forward(ctypes.byref(c), ctypes.byref(o), n, FAKE, FAKE, 4,
                                L.DTYPE_F32, None, FAKE, None, FAKE, None, FAKE, FAKE, FAKE,
                                None, FAKE, wsb, None)
    assert st == L.INPC_ERR_INVALID and b"lpos" in lib.inpc_last_error()


def test_status_strings():
    lib = L.lib()
    for s in (L.INPC_OK, L.INPC_ERR_INVALID, L.INPC_ERR_CAPACITY, L.INPC_ERR_HIP,
              L.INPC_ERR_UNSUPPORTED):
        assert lib.inpc_status_string(s)


def test_project_ring_checks():
    """inpc_project_ring: slot count in [1, 16], counts within [0, slot_cap],
    counts given; every check before any launch."""
    lib = L.lib()
    c, o = cam(), L.make_opts(tile=8)
    cap = 100
    wsb = lib.inpc_workspace_bytes(4 * cap, ctypes.byref(c), ctypes.byref(o))
    ok = (ctypes.c_int64 * 4)(100, 0, 37, 100)

    def call(k, slot_cap, counts, ws_bytes=wsb):
        return lib.inpc_project_ring(ctypes.byref(c), ctypes.byref(o), k, slot_cap, counts,
                                     FAKE, FAKE, None, FAKE, FAKE, FAKE, FAKE, ws_bytes, None)
    assert call(0, cap, ok) == L.INPC_ERR_INVALID
    assert call(17, cap, (ctypes.c_int64 * 17)()) == L.INPC_ERR_INVALID
    assert call(4, 0, ok) == L.INPC_ERR_INVALID
    assert call(4, cap, None) == L.INPC_ERR_INVALID
    assert call(4, cap, (ctypes.c_int64 * 4)(100, 101, 0, 0)) == L.INPC_ERR_INVALID
    assert b"slot count" in lib.inpc_last_error()
    assert call(4, cap, (ctypes.c_int64 * 4)(-1, 0, 0, 0)) == L.INPC_ERR_INVALID
    # the workspace is checked for n = slots * slot_cap points
    small = lib.inpc_workspace_bytes(cap, ctypes.byref(c), ctypes.byref(o))
    assert call(4, cap, ok, small) == L.INPC_ERR_INVALID


def test_backward_zero_and_prezeroed_reject_bad_arguments():
    """inpc_backward_zero checks sizes and buffers before any launch;
    inpc_blend_backward_prezeroed takes inpc_blend_backward's checks."""
    lib = L.lib()
    n, C, sb = 100, 4, 1792  # 16 bytes per point, rounded up to 256
    bad = L.INPC_ERR_INVALID
    assert lib.inpc_backward_zero(-1, C, FAKE, FAKE, sb, None) == bad
    assert lib.inpc_backward_zero(n, 0, FAKE, FAKE, sb, None) == bad
    assert lib.inpc_backward_zero(n, 33, FAKE, FAKE, sb, None) == bad
    assert lib.inpc_backward_zero(n, C, None, FAKE, sb, None) == bad
    assert lib.inpc_backward_zero(n, C, FAKE, None, sb, None) == bad
    assert lib.inpc_backward_zero(n, C, ctypes.c_void_p(0x1004), FAKE, sb, None) == bad
    assert lib.inpc_backward_zero(n, C, FAKE, FAKE, sb - 1, None) == bad
    assert lib.inpc_backward_zero(0, C, None, None, 0, None) == L.INPC_OK
    c, o = cam(), L.make_opts(tile=8)
    wsb = lib.inpc_workspace_bytes(10, ctypes.byref(c), ctypes.byref(o))
    need = lib.inpc_backward_scratch_bytes(10, C, ctypes.byref(c), ctypes.byref(o))
    args = [ctypes.byref(c), ctypes.byref(o), 10, FAKE, FAKE, C, L.DTYPE_F32, None, FAKE,
            FAKE, None, FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, FAKE, None, None]
    assert lib.inpc_blend_backward_prezeroed(*args, FAKE, need - 1, FAKE, wsb, None) == bad
    assert lib.inpc_blend_backward_prezeroed(*args, None, need, FAKE, wsb, None) == bad
