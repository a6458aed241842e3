"""GPU parity of the GP conditioned on point observations (Sec. 3.1, Eq. condition_gp) with
the FP64 oracle, through the C-ABI: majorants, the medium at points, images at small size
and sampled pixels at the full 512^2, 64 spp launch."""
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


def _small(which, **kw):
    kw = {**dict(width=64, height=64, spp=8), **kw}
    return sc.cond_sphere_scene(**kw) if which == "sphere" else sc.cond_blob_scene(**kw)


@pytest.mark.parametrize("which", ["sphere", "blob"])
def test_cond_majorants_match_oracle_bitwise(G, which):
    s = _small(which)
    print(f"[cond] majorants {s.name}", flush=True)
    a = G.GpssScene(s).majorants()
    b = orc.OracleScene(s).majorants()
    assert np.array_equal(a.view(np.uint32), b.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("which", ["sphere", "blob", "sphere-1", "sphere-6", "sphere-13", "sphere-31"])
def test_cond_medium_matches_oracle(G, which):
    """Medium evaluation against the oracle; sphere-N conditions on N observations, so that
    the observation blocks of four end part-filled (N not a multiple of 4)."""
    if "-" in which:
        s = sc.cond_sphere_scene(n_obs=int(which.split("-")[1]), width=64, height=64, spp=8)
    else:
        s = _small(which)
    rng = np.random.default_rng(11)
    n = 3000 if "-" not in which else 600
    lo, hi = s.bounds[:3].astype(np.float64), s.bounds[3:].astype(np.float64)
    obs = s.observations[:, :3].astype(np.float64)
    pts = np.concatenate([lo + rng.random((n // 2, 3)) * (hi - lo),
                          obs[rng.integers(len(obs), size=n - n // 2)] + rng.normal(scale=0.06, size=(n - n // 2, 3))])
    pts = np.clip(pts, lo, hi).astype(np.float32)
    dirs = rng.normal(size=(n, 3))
    dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
    print(f"[cond] medium {s.name} n={n}", flush=True)
    out = G.GpssScene(s).eval_medium(pts, dirs).cpu().numpy().astype(np.float64)
    o = orc.OracleScene(s)
    worst = {}
    for i in range(n):
        x, d = pts[i].astype(np.float64), dirs[i].astype(np.float64)
        e = o.eval_point(x)
        post = o.posterior(x)
        st = o.sigma_t(x, d)
        sp = orc.sigma_proj_cov(post["mg"], post["Sg"], d)
        D = orc.ndf_cov(post["mg"], post["Sg"], d)
        peak = orc.ndf_cov(post["mg"], post["Sg"], post["mg"] / np.linalg.norm(post["mg"]))
        # mu enters the medium only through mu / sigma: its error is measured in units of sigma
        worst["mu/sigma"] = max(worst.get("mu/sigma", 0.0), abs(out[i, 0] - e["mu"]) / e["sigma"])
        for name, gv, ov, floor in (("sigma", out[i, 1], e["sigma"], 0.0),
                                    ("proj", out[i, 4], sp, 1e-6), ("sigma_t", out[i, 5], st, 1e-6),
                                    ("ndf", out[i, 6], D, 1e-6 * peak)):
            err = abs(gv - ov) / max(abs(ov), floor, 1e-30)
            worst[name] = max(worst.get(name, 0.0), err)
    print("   ", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for k in ("mu/sigma", "sigma", "proj", "sigma_t", "ndf"):
        assert worst[k] < 1e-4, (k, worst)


@pytest.mark.parametrize("which", ["sphere", "blob"])
def test_cond_image_parity(G, which):
    s = _small(which)
    print(f"[cond] parity {s.name} {s.width}x{s.height} spp {s.spp}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy()
    ref = orc.OracleScene(s).render()
    st = gh.compare_images(img, ref, s.spp, s.name)
    print("   ", gh.fmt(st), flush=True)
    assert ref["counters"]["violations"] == 0
    gh.assert_parity(st)


def test_cond_image_parity_ragged(G):
    """Odd image size and few observations: ragged chunks and a partly filled observation set."""
    s = sc.cond_sphere_scene(n_obs=5, width=37, height=29, spp=3)
    print(f"[cond] parity {s.name} {s.width}x{s.height} spp {s.spp}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy()
    ref = orc.OracleScene(s).render()
    st = gh.compare_images(img, ref, s.spp, s.name)
    print("   ", gh.fmt(st), flush=True)
    gh.assert_parity(st)


def test_cond_full_size_sampled(G):
    """512^2, 64 spp, depth 32 (the sphere workload's launch) with 32 observations: the GPU
    image at 20 000 oracle-traced pixels."""
    s = sc.cond_sphere_scene()
    rng = np.random.default_rng(12)
    px = np.sort(rng.choice(s.n_pixels, gh.NPIX_SAMPLED, replace=False)).astype(np.int64)
    print(f"[cond] full size {s.name} {s.width}x{s.height} spp {s.spp}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy().ravel()
    ref = orc.OracleScene(s).render_pixels(px)
    st = gh.compare_sampled(img[px], ref, s.spp, s.name)
    print("   ", st, flush=True)
    gh.assert_sampled_parity(st)


def test_conditioning_changes_the_image(G):
    a = G.GpssScene(_small("sphere")).render().cpu().numpy()
    b = G.GpssScene(_small("sphere").replace(observations=None, obs_noise=0.0)).render().cpu().numpy()
    assert np.abs(a - b).mean() > 0.02 * np.abs(b).mean()


def test_cond_unsupported_paths_raise(G):
    s = _small("sphere", width=16, height=16, spp=2)
    g = G.GpssScene(s)
    for k in ("mega", "wavefront"):
        g.set_kernel(k)
        with pytest.raises(G.GpssError):
            g.render()
    g.set_kernel("auto")
    with pytest.raises(G.GpssError):
        g.render_adjoint(torch.zeros(s.height, s.width, dtype=torch.float32))
    with pytest.raises(G.GpssError):
        g.set_params(variance=0.003)
    with pytest.raises(G.GpssError):
        G.render_batch([g])
    with pytest.raises(G.GpssError):
        g.debug_trace([(0, 0)])
