"""The preallocated single-view pipeline in the form the benchmark times:
the backward's zero fill (inpc_backward_zero) on a stream of its own, forked
before the forward's tile sort, and the backward blend without its own fill
(inpc_blend_backward_prezeroed), against the oracle and against the
pipeline with the fill inside the backward."""
import ctypes

import numpy as np
import pytest
import torch

from scenes import SceneSpec, make_scene

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2508_19140_amd as inpc  # noqa: E402
from gpu_helpers import assert_backward, assert_forward, run_oracle, settings_opts  # noqa: E402

DEV = "cuda:0"

# 8x8 tiles over a 40x25-tile image, many points split over tiles, a ragged
# last tile row (200 = 25 x 8, 324 = 40 x 8 + 4)
SPEC = SceneSpec(n=200_000, s=4.0, z_lo=2.0, z_hi=20.0, width=324, height=200, focal=300.0,
                 channels=16, feat_dist="normal", opacity_range=(0.05, 0.95), with_grad=True,
                 seed=11)


def _outputs(p):
    g = {k: t.cpu().numpy() for k, t in p.outputs().items()}
    g["n_contrib"] = g["n_contrib"].view(np.uint32)
    return g


def _pipeline(sc, zero_ahead, keep_lists=False):
    t = lambda a: torch.from_numpy(a).to(DEV)
    v = inpc.ViewInputs(pos=t(sc.pos), opacity=t(sc.opacity), feat=t(sc.feat),
                        camera=sc.camera, grad_out=t(sc.grad))
    return inpc.ViewPipeline(v, inpc.RasterSettings(tile=8, keep_lists=keep_lists),
                             zero_ahead=zero_ahead)


@pytest.mark.parametrize("keep_lists", [False, True])
def test_zero_ahead_passes_match_oracle(keep_lists):
    """Three passes in a row with the gradient rows and the scratch poisoned
    (NaN) before each; every pass against the oracle, on the current stream
    given as an int and as a ctypes handle.  Lists recomputed: the fill in
    two halves, beside the forward's and the backward's sorts; lists kept:
    all of it beside the forward's sort."""
    sc = make_scene(SPEC)
    _, _, rr = run_oracle(sc, settings_opts(tile=8))
    p = _pipeline(sc, zero_ahead=True, keep_lists=keep_lists)
    names = [nm for nm, _ in p.phases()]
    assert names[:4] == ["project", "bin", "backward_zero", "sort"]
    assert names.count("backward_zero") == (1 if keep_lists else 2)
    assert p.zero_split == (SPEC.n if keep_lists else SPEC.n // 2)
    h = torch.cuda.current_stream().cuda_stream
    for rep, s in enumerate((h, ctypes.c_void_p(h), h)):
        print(f"  pass {rep}", flush=True)
        for t in (p.gf, p.go, p.guv, p.gpos):
            t.fill_(float("nan"))
        p.scratch.fill_(0xff)
        p.step(s)
        torch.cuda.synchronize()
        g = _outputs(p)
        assert_forward(g, rr)
        assert_backward(g, rr, sc.grad)


def test_zero_ahead_on_a_side_stream_matches_the_inline_fill():
    """Pipeline passes issued on a non-default stream: the forked fill form
    against the form that zeroes inside the backward (forward outputs bit
    for bit, gradients of single-tile points bit for bit, the rest within
    float-atomic reordering)."""
    sc = make_scene(SPEC)
    a, b = _pipeline(sc, zero_ahead=True), _pipeline(sc, zero_ahead=False)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(2):
            a.step(st.cuda_stream)
            b.step(st.cuda_stream)
    torch.cuda.synchronize()
    ga, gb = _outputs(a), _outputs(b)
    for k in ("out", "t_final", "n_contrib"):
        np.testing.assert_array_equal(ga[k], gb[k])
    single = b.ntiles.cpu().numpy() == 1
    np.testing.assert_array_equal(ga["grad_feat"][single], gb["grad_feat"][single])
    for k in ("grad_feat", "grad_opacity", "grad_uv", "grad_pos"):
        np.testing.assert_allclose(ga[k], gb[k], rtol=1e-4, atol=1e-5)


def test_zero_ahead_refuses_graph_capture(monkeypatch):
    """The forked fill is for eager use: under stream capture it raises before
    it records or launches anything (capture status forced from the host)."""
    sc = make_scene(SceneSpec(n=4096, s=4.0, z_lo=2.0, z_hi=20.0, width=64, height=48,
                              focal=64.0, channels=4, feat_dist="normal",
                              opacity_range=(0.05, 0.95), with_grad=True, seed=2))
    p = _pipeline(sc, zero_ahead=True)
    monkeypatch.setattr(torch.cuda, "is_current_stream_capturing", lambda: True)
    with pytest.raises(RuntimeError, match="cannot be captured"):
        p.zero(torch.cuda.current_stream().cuda_stream)
    monkeypatch.undo()
    p.step(torch.cuda.current_stream().cuda_stream)  # eager use still works
    torch.cuda.synchronize()
