"""inpc_blend_backward_noalloc: the backward pass with its scratch in the
library's static device array, for callers that cannot allocate.  Through
the C ABI it must give what inpc_blend_backward gives with a caller-owned
scratch, on consecutive calls (the second smaller, so stale contents of the
shared array from the first would show), and it must refuse sizes beyond
the array."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2508_19140_amd import _lib as L


def test_noalloc_rejects_more_than_the_static_scratch():
    """Host check, no GPU: a request whose scratch exceeds the static array
    returns INPC_ERR_INVALID before touching the device."""
    lib = L.lib()
    c = L.make_camera(1920, 1080, 960.0, 960.0, 960.0, 540.0, [1, 0, 0, 0, 1, 0, 0, 0, 1],
                      [0, 0, 0])
    o = L.make_opts(tile=8)
    n = L.STATIC_SCRATCH_BYTES // 16 + 1
    need = lib.inpc_backward_scratch_bytes(n, 16, ctypes.byref(c), ctypes.byref(o))
    assert need > L.STATIC_SCRATCH_BYTES
    st = lib.inpc_blend_backward_noalloc(ctypes.byref(c), ctypes.byref(o), n, *([None] * 2), 16,
                                         L.DTYPE_F32, *([None] * 16), 0, None)
    assert st == L.INPC_ERR_INVALID
    assert b"static" in lib.inpc_last_error()


def _backward_both(scene, bg):
    import paper_2508_19140_amd as inpc
    from paper_2508_19140_amd import raster
    dev = "cuda:0"
    cam = inpc.camera_struct(scene.camera)
    opts = inpc.RasterSettings().opts()
    pos = torch.from_numpy(scene.pos).to(dev)
    op = torch.from_numpy(scene.opacity).to(dev)
    ft = torch.from_numpy(scene.feat).to(dev)
    g = torch.from_numpy(scene.grad).to(dev)
    bgt = torch.as_tensor(bg, dtype=torch.float32, device=dev)
    ws = inpc.Workspace().get(pos.shape[0], cam, opts, dev)
    b = inpc.project_bin_sort(pos, op, cam, opts, ws)
    out, tf, nc, state = inpc.blend_forward(b, ft, cam, opts, ws, bgt)
    ref = inpc.blend_backward(b, ft, cam, opts, ws, tf, state, g, None, bgt)
    n, C = ft.shape
    nan = lambda *s: torch.full(s, float("nan"), dtype=torch.float32, device=dev)
    gf, go, guv, gbg = nan(n, C), nan(n), nan(n, 2), nan(C)
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    L.call("inpc_blend_backward_noalloc", ctypes.byref(cam), ctypes.byref(opts), n, p(b.proj),
           p(ft), C, L.DTYPE_F32, p(bgt), p(b.ntiles), p(b.ranges), p(b.order), p(b.list),
           p(b.lpos), p(tf), p(state), p(g), None, p(gf), p(go), p(guv), None, p(gbg), p(ws),
           ws.numel(), ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    torch.cuda.synchronize()
    assert raster.backward_scratch_bytes(n, C, cam, opts) <= L.STATIC_SCRATCH_BYTES
    ref = [ref.feat, ref.opacity, ref.uv, ref.bg]
    return [t.cpu().numpy() for t in ref], [gf.cpu().numpy(), go.cpu().numpy(),
                                            guv.cpu().numpy(), gbg.cpu().numpy()], b


@pytest.mark.gpu
@pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")
def test_noalloc_matches_the_scratch_entry_point_on_two_calls():
    import oracle
    from scenes import SceneSpec, make_scene
    for n, W, H, seed in ((300_000, 480, 270, 1), (40_000, 200, 120, 2)):
        print(f"case n={n} {W}x{H} seed={seed}", flush=True)
        sc = make_scene(SceneSpec(n=n, s=4.0, z_lo=2.0, z_hi=20.0, width=W, height=H,
                                  channels=16, feat_dist="normal", opacity_range=(0.05, 0.95),
                                  with_grad=True, seed=seed))
        bg = np.linspace(-1.0, 1.0, 16)
        ref, got, b = _backward_both(sc, bg)
        rr = oracle.render(sc.camera, sc.pos, sc.opacity, sc.feat, bg=bg, grad_out=sc.grad)
        single = b.ntiles.cpu().numpy() <= 1
        names = ("grad_feat", "grad_opacity", "grad_uv")
        for k, name in enumerate(names):
            assert not np.isnan(got[k]).any(), name
            # points in one tile: stored, not added, so bit for bit
            np.testing.assert_array_equal(got[k][single], ref[k][single])
            # points split over tiles: float atomics in the order tiles finish
            ok, st = oracle.within_tolerance(got[k], rr[name], rr[name + "_abs"])
            assert st["n_bad"] == 0, (name, st)
            ok, st = oracle.within_tolerance(ref[k], rr[name], rr[name + "_abs"])
            assert st["n_bad"] == 0, (name, st)
        mag = np.abs(rr["t_final"][None] * sc.grad.astype(np.float64)).sum(axis=(1, 2))
        np.testing.assert_array_equal(got[3], ref[3])
        ok, st = oracle.within_tolerance(got[3], rr["grad_bg"], mag)
        assert st["n_bad"] == 0, st
