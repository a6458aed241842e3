"""GPU parity of the conductor Fresnel term (F of Eq. phase with a complex index of
refraction, F = albedo x Fresnel reflectance at the half vector) with the FP64 oracle, and
RGB rendering as three channel scenes in one batched launch."""
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


CASES = {
    "plane_gold_r": lambda: sc.fresnel_rgb_scenes(sc.plane_scene(), "gold")[0],
    "plane_gold_b": lambda: sc.fresnel_rgb_scenes(sc.plane_scene(), "gold")[2],
    "sphere_copper_g": lambda: sc.fresnel_rgb_scenes(sc.sphere_scene(0.05, width=64, height=64, spp=8), "copper")[1],
    "ggx_sphere_gold_r": lambda: sc.fresnel_rgb_scenes(sc.ggx_sphere_scene(0.3, width=64, height=64, spp=8),
                                                       "gold")[0],
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fresnel_parity(G, name):
    s = CASES[name]()
    print(f"[fresnel] parity {name} eta {s.fresnel_eta} k {s.fresnel_k}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy()
    ref = orc.OracleScene(s).render()
    st = gh.compare_images(img, ref, s.spp, name)
    print("   ", gh.fmt(st), flush=True)
    assert ref["counters"]["violations"] == 0
    gh.assert_parity(st)


def test_fresnel_kernels_bitwise(G):
    s = CASES["sphere_copper_g"]().replace(width=40, height=40, spp=4)
    g = G.GpssScene(s, kernel="mega")
    a = g.render_paths().cpu().numpy()
    for k in ("wavefront", "persistent"):
        g.set_kernel(k)
        b = g.render_paths().cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), k


def test_rgb_channels_in_one_batch(G):
    """Three channel scenes rendered by one batched launch equal their single renders, and
    the channels differ (gold reflects red more than blue)."""
    scenes = sc.fresnel_rgb_scenes(sc.sphere_scene(0.05, width=96, height=96, spp=8), "gold")
    gs = [G.GpssScene(s) for s in scenes]
    outs = G.render_batch(gs)
    torch.cuda.synchronize()
    for g, o in zip(gs, outs):
        assert torch.equal(o, g.render())
    r, gch, b = [o.cpu().numpy() for o in outs]
    assert r.mean() > gch.mean() > b.mean()


def test_fresnel_adjoint_matches_oracle(G):
    """The adjoint with the Fresnel term (a constant factor of the phase weights)."""
    s0 = sc.offset_sphere_scene(False, width=32, height=32, spp=4, max_depth=8, grid_res=16,
                                majorant_res=(16, 16, 16)).replace(fresnel_eta=0.27, fresnel_k=3.61)
    tgt = sc.offset_sphere_scene(True, width=32, height=32, spp=4, max_depth=8, grid_res=16,
                                 majorant_res=(16, 16, 16)).replace(fresnel_eta=0.27, fresnel_k=3.61)
    I = orc.OracleScene(s0).render()["mean"]
    T = orc.OracleScene(tgt).render()["mean"]
    dl = 2.0 * (I - T) / I.size
    ids = [-1, -2, -3] + [int(i) for i in sc.grad_param_indices(s0, n_nodes=12)]
    g_orc, _ = orc.OracleScene(s0).render_grad(dl, ids)
    g_off, g_sc = G.GpssScene(s0).render_adjoint(torch.as_tensor(dl, dtype=torch.float32))
    torch.cuda.synchronize()
    g_off = g_off.cpu().numpy().ravel()
    g_sc = g_sc.cpu().numpy()
    g_gpu = np.array([g_sc[0], g_sc[1], g_sc[2]] + [g_off[i] for i in ids[3:]], np.float64)
    print("[fresnel] adjoint", np.c_[g_gpu, g_orc][:6], flush=True)
    from tests.test_gpu_adjoint import _check_groups
    _check_groups(g_gpu, g_orc)


@pytest.mark.parametrize("channel", [0, 2])
def test_fresnel_full_size_sampled(G, channel):
    """The measured Fresnel workload (sphere l = 0.1 at 512^2, 64 spp, depth 32, gold, one
    channel scene): the GPU image at 20 000 oracle-traced pixels."""
    s = sc.fresnel_rgb_scenes(sc.sphere_scene(0.1), "gold")[channel]
    rng = np.random.default_rng(20 + channel)
    px = np.sort(rng.choice(s.n_pixels, gh.NPIX_SAMPLED, replace=False)).astype(np.int64)
    print(f"[fresnel] full size {s.name} {s.width}x{s.height} spp {s.spp}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy().ravel()
    ref = orc.OracleScene(s).render_pixels(px)
    st = gh.compare_sampled(img[px], ref, s.spp, s.name)
    print("   ", st, flush=True)
    gh.assert_sampled_parity(st)
