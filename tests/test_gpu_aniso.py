"""GPU parity of the anisotropic kernel (lengthscale l across and l_n along the local
mean-gradient direction; Fig. cmp_aniso: alpha_z = 0.01 against the isotropic 0.8) with
the FP64 oracle, through the C-ABI."""
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


def _small(alpha_z, **kw):
    return sc.aniso_sphere_scene(alpha_z, **{**dict(width=64, height=64, spp=8), **kw})


def _plane(ln):
    return sc.plane_scene().replace(lengthscale_n=ln, name=f"plane_ln{ln:g}")


def test_aniso_majorants_match_oracle_bitwise(G):
    for s in (_small(0.01), _small(0.2), _plane(0.2), _plane(0.01)):
        print(f"[aniso] majorants {s.name}", flush=True)
        a = G.GpssScene(s).majorants()
        b = orc.OracleScene(s).majorants()
        assert np.array_equal(a.view(np.uint32), b.astype(np.float32).view(np.uint32))


def test_aniso_medium_matches_oracle(G):
    rng = np.random.default_rng(3)
    for s in (_small(0.01), _small(0.2), _plane(0.2), _plane(0.01)):
        n = 3000
        lo, hi = s.bounds[:3], s.bounds[3:]
        pts = (lo + rng.random((n, 3)) * (hi - lo)).astype(np.float32)
        dirs = rng.normal(size=(n, 3))
        dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
        print(f"[aniso] medium {s.name} n={n}", flush=True)
        out = G.GpssScene(s).eval_medium(pts, dirs).cpu().numpy().astype(np.float64)
        o = orc.OracleScene(s)
        worst = {}
        for i in range(n):
            x, d = pts[i].astype(np.float64), dirs[i].astype(np.float64)
            e = o.eval_point(x)
            assert e["sn"] != e["s"]
            sp = orc.sigma_proj_n(e["G"], e["s"], e["sn"], d)
            D = orc.ndf_n(e["G"], e["s"], e["sn"], d)
            st = o.sigma_t(x, d)
            for name, gv, ov in (("proj", out[i, 4], sp), ("sigma_t", out[i, 5], st), ("ndf", out[i, 6], D)):
                err = abs(gv - ov) / max(abs(ov), 1e-6)
                worst[name] = max(worst.get(name, 0.0), err)
        print("   ", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
        assert worst["proj"] < 1e-4 and worst["sigma_t"] < 1e-4 and worst["ndf"] < 1e-4


@pytest.mark.parametrize("alpha_z", [0.01, 0.2, 0.8])
def test_aniso_sphere_parity(G, alpha_z):
    s = _small(alpha_z)
    print(f"[aniso] parity {s.name} {s.width}x{s.height} spp {s.spp}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy()
    ref = orc.OracleScene(s).render()
    st = gh.compare_images(img, ref, s.spp, s.name)
    print("   ", gh.fmt(st), flush=True)
    assert ref["counters"]["violations"] == 0
    gh.assert_parity(st)


def test_aniso_plane_parity(G):
    s = _plane(0.2)
    print(f"[aniso] parity {s.name}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy()
    ref = orc.OracleScene(s).render()
    st = gh.compare_images(img, ref, s.spp, s.name)
    print("   ", gh.fmt(st), flush=True)
    gh.assert_parity(st)


def test_aniso_full_size_sampled(G):
    """512^2, 64 spp, depth 32 (the sphere workload's launch) at alpha_z = 0.01: the GPU
    image at 20 000 oracle-traced pixels."""
    s = sc.aniso_sphere_scene(0.01)
    rng = np.random.default_rng(7)
    px = np.sort(rng.choice(s.n_pixels, gh.NPIX_SAMPLED, replace=False)).astype(np.int64)
    print(f"[aniso] full size {s.name} {s.width}x{s.height} spp {s.spp}", flush=True)
    img = G.GpssScene(s).render().cpu().numpy().ravel()
    ref = orc.OracleScene(s).render_pixels(px)
    st = gh.compare_sampled(img[px], ref, s.spp, s.name)
    print("   ", st, flush=True)
    gh.assert_sampled_parity(st)


def test_aniso_alpha_z_changes_the_image(G):
    """The anisotropic and isotropic kernels (Fig. cmp_aniso) give different images."""
    a = G.GpssScene(_small(0.01)).render().cpu().numpy()
    b = G.GpssScene(_small(0.8)).render().cpu().numpy()
    assert np.abs(a - b).mean() > 0.05 * np.abs(b).mean()


def test_adjoint_rejects_anisotropic_kernel(G):
    s = _small(0.01)
    g = G.GpssScene(s)
    with pytest.raises(G.GpssError):
        g.render_adjoint(torch.zeros(s.height, s.width, dtype=torch.float32))
