"""Parity at the workloads' full sizes, in the launch configuration bench.py times, on
pixels sampled at random (the oracle computes only those pixels).  Each sample holds 20 000
pixels (the batch: 300 per scene), so that the raw fraction of pixels off by more than the
relative tolerance resolves the 0.1 % bar: at most 20 of them."""
import numpy as np
import pytest

from gpss_inputs import scenes as sc
from oracle import oracle as orc
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_00280_amd import gpss
    return gpss


def _sample(s, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(s.n_pixels, size=min(n, s.n_pixels), replace=False))


def _check(img, s, px, label):
    ref = orc.OracleScene(s).render_pixels(px)
    st = gh.compare_sampled(np.asarray(img).ravel()[px], ref, s.spp, label)
    print("   ", gh.fmt(st), flush=True)
    gh.assert_sampled_parity(st)


@pytest.mark.parametrize("l", sc.SPHERE_LENGTHSCALES)
def test_sphere_full_size(G, l):
    s = sc.sphere_scene(l)
    print(f"[fullsize] sphere l={l} {s.width}x{s.height} spp {s.spp} depth {s.max_depth}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy()
    _check(img, s, _sample(s, gh.NPIX_SAMPLED, 7), f"sphere l={l}")


def test_mixed_full_size(G):
    s = sc.mixed_scene()
    print(f"[fullsize] mixed {s.width}x{s.height} spp {s.spp} depth {s.max_depth}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy()
    _check(img, s, _sample(s, gh.NPIX_SAMPLED, 8), "mixed16")


def test_offset_sphere_full_size(G):
    for target in (True, False):
        s = sc.offset_sphere_scene(target)
        print(f"[fullsize] offset sphere target={target}", flush=True)
        img = G.GpssScene(s).render().cpu().numpy()
        _check(img, s, _sample(s, gh.NPIX_SAMPLED, 9), f"offset target={target}")


def test_batch_full_size(G):
    scenes = sc.batch_scenes()
    print(f"[fullsize] batch of {len(scenes)} scenes", flush=True)
    gs = [G.GpssScene(s) for s in scenes]
    imgs = G.render_batch(gs)
    torch.cuda.synchronize()
    vals, means, vars_, spps = [], [], [], []
    for i, (s, im) in enumerate(zip(scenes, imgs)):
        px = _sample(s, 300, 100 + i)
        ref = orc.OracleScene(s).render_pixels(px)
        vals.append(im.cpu().numpy().ravel()[px])
        # fold the per-scene spp into the variance so that one comparison covers the batch
        means.append(ref["mean"])
        vars_.append(ref["var"] / s.spp)
    st = gh.compare_sampled(np.concatenate(vals), {"mean": np.concatenate(means),
                                                   "var": np.concatenate(vars_)}, 1, "batch64")
    print("   ", gh.fmt(st), flush=True)
    gh.assert_sampled_parity(st)
