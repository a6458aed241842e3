"""Batched persistent rendering (one hipGraph launch) against per-scene renders."""
import os

import numpy as np
import pytest

from gpss_inputs import scenes as sc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_00280_amd import gpss
    return gpss


def _small_batch():
    """Uneven sizes and sample counts from the batch generator, shrunk for a test."""
    out = sc.batch_scenes(n=7, seed=4, resolutions=(16, 24, 40), spps=(1, 3, 8), max_depth=12)
    out.append(sc.plane_scene(width=20, height=12, spp=5).replace(scene_id=99))
    out.append(sc.mixed_scene(width=16, height=16, spp=2, var_res=32).replace(scene_id=100))
    return out


def test_batch_equals_individual_renders(G):
    scenes = _small_batch()
    print("[batch]", [(s.width, s.height, s.spp) for s in scenes], flush=True)
    gs = [G.GpssScene(s) for s in scenes]
    ref = [g.render().cpu().numpy() for g in gs]
    imgs = G.render_batch(gs)
    torch.cuda.synchronize()
    for a, b in zip(imgs, ref):
        assert np.array_equal(a.cpu().numpy(), b)
    # graph replay into fresh image buffers
    imgs2 = G.render_batch(gs)
    for a, b in zip(imgs2, ref):
        assert np.array_equal(a.cpu().numpy(), b)


def test_batch_sees_parameter_updates(G):
    scenes = _small_batch()[:3]
    gs = [G.GpssScene(s) for s in scenes]
    G.render_batch(gs)
    gs[1].set_params(variance=0.004, lengthscale=0.07, albedo=0.6)
    fresh = G.GpssScene(scenes[1].replace(variance=0.004, lengthscale=0.07, albedo=0.6))
    imgs = G.render_batch(gs)
    assert np.array_equal(imgs[1].cpu().numpy(), fresh.render().cpu().numpy())


def test_batch_calls_are_stream_ordered(G):
    """Calls return without waiting: several replays into different image buffers and a
    parameter update between them, queued on one side stream with no host synchronization,
    each give the image of its own parameters."""
    scenes = _small_batch()[:4]
    gs = [G.GpssScene(s) for s in scenes]
    G.render_batch(gs)                      # plan and graph
    torch.cuda.synchronize()
    ref0 = [g.render().cpu().numpy() for g in gs]
    upd = dict(variance=0.004, lengthscale=0.07, albedo=0.6)
    ref1 = G.GpssScene(scenes[2].replace(**upd)).render().cpu().numpy()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = [[torch.empty(g.shape, device="cuda") for g in gs] for _ in range(6)]
        for k in range(6):
            if k == 3:   # the record changes between queued replays
                gs[2].set_params(stream=stream, **upd)
            G.render_batch(gs, outs[k], stream=stream)
    stream.synchronize()
    for k in range(6):
        for i, (o, r) in enumerate(zip(outs[k], ref0)):
            want = ref1 if (k >= 3 and i == 2) else r
            assert np.array_equal(o.cpu().numpy(), want), (k, i)


def test_batch_autotune_and_cache(G, tmp_path):
    os.environ["GPSS_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        scenes = _small_batch()[:4]
        gs = [G.GpssScene(s) for s in scenes]
        ref = [g.render().cpu().numpy() for g in gs]
        outs = [torch.empty(g.shape, device="cuda") for g in gs]
        best = G.gpss_batch_autotune([g.handle for g in gs], [o.data_ptr() for o in outs])
        print("   tuned", best, flush=True)
        assert best["tile"] in (1024, 4096, 16384) and best["waves_per_cu"] in (8, 12)
        assert (tmp_path / "tune.txt").exists()
        imgs = G.render_batch(gs)
        for a, b in zip(imgs, ref):
            assert np.array_equal(a.cpu().numpy(), b)
        # a new scene list with the same signature picks the cached configuration
        gs2 = [G.GpssScene(s) for s in scenes]
        imgs = G.render_batch(gs2)
        for a, b in zip(imgs, ref):
            assert np.array_equal(a.cpu().numpy(), b)
    finally:
        os.environ.pop("GPSS_TUNE_CACHE", None)


def test_batch_rejects_bad_arguments(G):
    g = G.GpssScene(sc.plane_scene(width=8, height=8, spp=1))
    with pytest.raises(G.GpssError):
        G.gpss_render_batch([], [])
    with pytest.raises(G.GpssError):
        G.gpss_render_batch([g.handle], [0])
