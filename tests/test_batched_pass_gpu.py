"""Many views in one pass: the batched entry point (inpc_rasterize_batched,
one persistent blend launch over every (view, tile) item of the batch) and
its graph capture, against the views run one by one and against the
oracle; the autotuned setting persisted in the JSON cache."""
import json

import numpy as np
import pytest
import torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2508_19140_amd as inpc  # noqa: E402
from gpu_helpers import assert_backward, assert_forward, run_oracle, settings_opts  # noqa: E402
from scenes import multi_view_scenes  # noqa: E402

DEV = "cuda:0"


def _views(scenes):
    t = lambda a: torch.from_numpy(a).to(DEV)
    return [inpc.ViewInputs(pos=t(s.pos), opacity=t(s.opacity), feat=t(s.feat),
                            camera=s.camera, grad_out=t(s.grad)) for s in scenes]


def _check_views(br, scenes, single=None):
    for k, (sc, o) in enumerate(zip(scenes, br.outputs())):
        print(f"  view {k}: n={sc.pos.shape[0]} {sc.camera.width}x{sc.camera.height}",
              flush=True)
        g = {key: v.cpu().numpy() for key, v in o.items()}
        g["n_contrib"] = g["n_contrib"].view(np.uint32)
        st = settings_opts(tile=br.choice[0])
        _, _, rr = run_oracle(sc, st)
        assert_forward(g, rr)
        assert_backward(g, rr, sc.grad)
        if single is not None:  # forward bit for bit against the view run alone
            for key in ("out", "t_final", "n_contrib"):
                np.testing.assert_array_equal(g[key], single[k][key])


def test_batched_small_views_graph_and_cache(tmp_path):
    """Six small views of uneven size: the batched pass, its graph replays
    (with other GPU work between them) and the JSON autotune cache."""
    scenes = multi_view_scenes(6, seed=3, n_lo=20_000, n_hi=90_000, channels=4,
                               resolutions=((160, 90), (200, 112), (96, 64)))
    views = _views(scenes)
    cache = str(tmp_path / "autotune.json")
    br = inpc.BatchedRasterizer(views, cache_path=cache, reps=1)
    assert br.choice in br.tuning
    d = json.load(open(cache))
    assert d[br.key] == list(br.choice)
    # the views run alone through the single-view pipeline
    single = []
    for v in views:
        p = inpc.ViewPipeline(v, inpc.RasterSettings(tile=br.choice[0],
                                                     bin_points=br.choice[1]))
        p.step(torch.cuda.current_stream().cuda_stream)
        single.append({k: t.cpu().numpy().view(np.uint32) if k == "n_contrib" else
                       t.cpu().numpy() for k, t in p.outputs().items()})
    br.step()
    torch.cuda.synchronize()
    _check_views(br, scenes, single)
    br.capture()
    for rep in range(3):
        for o in br.outputs():
            for t in o.values():
                t.fill_(float("nan")) if t.is_floating_point() else t.fill_(-1)
        br.replay()
        torch.cuda.synchronize()
        x = torch.randn(1 << 20, device=DEV).sum().item()  # other work between replays
        assert np.isfinite(x)
        for k, o in enumerate(br.outputs()):
            for key in ("out", "t_final"):
                np.testing.assert_array_equal(o[key].cpu().numpy(), single[k][key])
    # a second instance reads the cached choice without tuning
    br2 = inpc.BatchedRasterizer(views, cache_path=cache)
    assert br2.choice == br.choice and br2.tuning == {}


@pytest.mark.timeout(900)
def test_batched_c4_full_size():
    """The C4 batch at its real size (8 views, 0.5M-6M points each, 960x540
    to 1920x1080, ring cameras with near-plane culling): every view against
    the oracle."""
    scenes = multi_view_scenes(8, seed=0)
    views = _views(scenes)
    br = inpc.BatchedRasterizer(views, autotune=False, settings=inpc.RasterSettings(tile=8))
    br.capture()
    br.replay()
    torch.cuda.synchronize()
    _check_views(br, scenes)
