"""GPU parity of the forward renderer against the FP64 oracle (through the C-ABI).

Both sides draw the same Philox numbers, so images agree path by path up to float
rounding, except for the rare branch flips that rounding causes (bounded below)."""
import math

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


def _render(G, s, s0=0, s1=None):
    g = G.GpssScene(s)
    img = g.render(s0, s1).cpu().numpy()
    torch.cuda.synchronize()
    return g, img


def _parity(G, s, label, s0=0, s1=None):
    s1 = s.spp if s1 is None else s1
    print(f"[parity] {label} {s.width}x{s.height} spp[{s0},{s1}) depth {s.max_depth}", flush=True)
    g, img = _render(G, s, s0, s1)
    ref = orc.OracleScene(s).render(s0, s1)
    st = gh.compare_images(img, ref, s1 - s0, label)
    print("   ", gh.fmt(st), flush=True)
    assert ref["counters"]["violations"] == 0
    gh.assert_parity(st)
    return g, img, ref


def _small_mixed(**kw):
    return sc.mixed_scene(**{**dict(width=48, height=48, spp=2, max_depth=64), **kw})


def test_majorants_match_oracle_bitwise(G):
    cases = [sc.plane_scene(), sc.sphere_scene(0.005, width=8, height=8),
             sc.sphere_scene(0.5, width=8, height=8), sc.mixed_scene(width=8, height=8),
             sc.offset_sphere_scene(True, width=8, height=8),
             sc.plane_scene(majorant_res=(3, 5, 7)).replace(mean_kind=sc.MEAN_CONST, mean_const=0.1)]
    for s in cases:
        gm = G.GpssScene(s).majorants()
        om = orc.OracleScene(s).majorants()
        assert gm.shape == om.shape
        diff = np.flatnonzero(gm.view(np.uint32) != om.view(np.uint32))
        assert diff.size == 0, (s.name, diff[:5], gm[diff[:5]], om[diff[:5]])
        # five significant bits (or 0, or infinity): the walk's copy of the grid, the top 16
        # bits of each float, holds every majorant exactly
        assert not np.any(gm.view(np.uint32) & np.uint32(0xFFFF)), s.name


def test_medium_evaluation_matches_oracle(G):
    rng = np.random.default_rng(0)
    for s in (sc.plane_scene(), sc.sphere_scene(0.02, width=8, height=8),
              sc.sphere_scene(0.5, width=8, height=8), sc.mixed_scene(width=8, height=8),
              sc.offset_sphere_scene(True, width=8, height=8)):
        n = 4000
        lo, hi = s.bounds[:3], s.bounds[3:]
        pts = (lo + rng.random((n, 3)) * (hi - lo)).astype(np.float32)
        dirs = rng.normal(size=(n, 3))
        dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
        out = G.GpssScene(s).eval_medium(pts, dirs).cpu().numpy().astype(np.float64)
        o = orc.OracleScene(s)
        worst = {}
        for i in range(n):
            e = o.eval_point(pts[i].astype(np.float64))
            st = o.sigma_t(pts[i].astype(np.float64), dirs[i].astype(np.float64))
            D = orc.ndf(e["G"], e["s"], dirs[i].astype(np.float64))
            sp = orc.sigma_proj(e["G"], e["s"], dirs[i].astype(np.float64))
            rho = orc.rho(e["mu"], e["sigma"])
            for name, gv, ov, scale in (("mu", out[i, 0], e["mu"], 1.0), ("sigma", out[i, 1], e["sigma"], 0),
                                        ("rho", out[i, 3], rho, 1e-3),
                                        ("proj", out[i, 4], sp, 1e-3), ("sigma_t", out[i, 5], st, 1e-3),
                                        ("ndf", out[i, 6], D, 1e-3)):
                err = abs(gv - ov) / max(abs(ov), scale * 1e-3 if scale else 1e-30)
                worst[name] = max(worst.get(name, 0.0), err)
            worst["mu_abs"] = max(worst.get("mu_abs", 0.0), abs(out[i, 0] - e["mu"]))
            assert out[i, 7] == pytest.approx(e["albedo"], rel=1e-6)
        print(s.name, {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
        # mu: single-precision evaluation of distances of order 1, so an absolute error of a few
        # units in the last place of 1 (2^-23 = 1.2e-7)
        assert worst["mu_abs"] < 5e-7
        assert worst["sigma"] < 5e-6
        assert worst["rho"] < 1e-4
        assert worst["proj"] < 1e-4 and worst["sigma_t"] < 1e-4 and worst["ndf"] < 1e-4


def _union_points(s, rng, n=6000):
    """Random points, points on majorant-cell faces and corners, and points near the
    primitives' surfaces, each also one float step either side; all inside the box."""
    lo, hi = s.bounds[:3].astype(np.float64), s.bounds[3:].astype(np.float64)
    M = np.array(s.majorant_res)
    cw = (hi - lo) / M
    pts = [lo + rng.random((n, 3)) * (hi - lo)]
    b = lo + rng.random((n, 3)) * (hi - lo)
    ax = rng.integers(0, 3, n)
    b[np.arange(n), ax] = lo[ax] + rng.integers(1, M[ax]) * cw[ax]     # on a cell face
    pts.append(b)
    pts.append(lo + (rng.integers(1, M, (n, 3))) * cw)                  # on cell corners
    prim = s.prims[rng.integers(0, len(s.prims), n)].astype(np.float64)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts.append(prim[:, 1:4] + d * (prim[:, 4:5] + rng.normal(0.0, 0.02, (n, 1))))
    p32 = np.concatenate(pts).astype(np.float32)
    p32 = np.concatenate([p32, np.nextafter(p32, np.float32(np.inf)), np.nextafter(p32, np.float32(-np.inf))])
    return p32[np.all((p32 >= lo) & (p32 <= hi), axis=1)]


def _tie_scene():
    """Seven primitives with exact ties (a duplicated sphere, a duplicated box) and a cluster
    of small spheres closer together than a majorant cell (cells with more than three
    candidates take every primitive)."""
    P = sc.PRIM_SPHERE, sc.PRIM_BOX
    prims = np.array([[P[0], 0.2, 0.1, 0.0, 0.3, 0, 0, 0.9],
                      [P[1], -0.4, 0.3, 0.2, 0.2, 0.25, 0.15, 0.7],
                      [P[0], 0.2, 0.1, 0.0, 0.3, 0, 0, 0.6],          # same sphere as 0
                      [P[1], -0.4, 0.3, 0.2, 0.2, 0.25, 0.15, 0.5],   # same box as 1
                      [P[0], 0.70, -0.6, 0.5, 0.02, 0, 0, 0.8],
                      [P[0], 0.71, -0.6, 0.5, 0.02, 0, 0, 0.65],
                      [P[0], 0.70, -0.59, 0.51, 0.02, 0, 0, 0.55]], np.float32)
    return sc.mixed_scene(width=8, height=8, n_prims=7).replace(prims=prims)


@pytest.mark.parametrize("name", ["mixed", "ties"])
def test_union_candidate_table_equals_full_union(G, name):
    """The per-cell candidate primitives of a union mean give the full union's result bit for
    bit: the scene with its majorant grid (the mixed scene: 80^3, about 1.3 candidates per
    cell) against the same scene with one majorant cell (more than three candidates: every
    primitive), at random points, points on cell boundaries and one float step either side
    of them, and points near the primitives' surfaces (the union's argmin changes there).
    The tie scene has exact ties, where the lower index must win in both loops."""
    rng = np.random.default_rng(21)
    s = sc.mixed_scene(width=8, height=8) if name == "mixed" else _tie_scene()
    p32 = _union_points(s, rng)
    dirs = rng.normal(size=p32.shape)
    dirs = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
    a = G.GpssScene(s).eval_medium(p32, dirs).cpu().numpy()
    full = G.GpssScene(s.replace(majorant_res=(1, 1, 1))).eval_medium(p32, dirs).cpu().numpy()
    print(f"[union table] {name}: {p32.shape[0]} points", flush=True)
    assert a.shape == full.shape
    bad = np.nonzero(np.any(a.view(np.uint32) != full.view(np.uint32), axis=1))[0]
    assert bad.size == 0, (bad[:5], p32[bad[:5]], a[bad[:5]], full[bad[:5]])
    if name == "ties":
        # on the duplicated sphere's surface region the lower index (albedo 0.9) wins
        x = np.array([[0.2, 0.1, 0.31]], np.float32)
        out = G.GpssScene(s).eval_medium(x, np.array([[0, 0, 1]], np.float32)).cpu().numpy()
        assert out[0, 7] == np.float32(0.9)


def test_parity_plane_full_size(G):
    """The tiny planar workload at its full size: 64x64, 16 spp, depth 8."""
    _parity(G, sc.plane_scene(), "plane")


def test_parity_plane_paths_and_counters(G):
    s = sc.plane_scene()
    g = G.GpssScene(s)
    paths, cnt = g.render_paths(counters=True)
    ref = orc.OracleScene(s).render(want_paths=True)
    st = gh.compare_paths(paths.cpu().numpy(), ref["paths"])
    c = G.counters_dict(cnt)
    print("   paths", gh.fmt(st), flush=True)
    print("   gpu counters", c, "\n   oracle counters", ref["counters"], flush=True)
    assert c["violations"] == 0 and c["capped"] == 0
    assert st["path_flip_fraction"] < 1e-3
    for k in ("track_steps", "real", "nee_steps", "escaped", "phase", "nee"):
        assert c[k] == pytest.approx(ref["counters"][k], rel=2e-3)


@pytest.mark.parametrize("l", sc.SPHERE_LENGTHSCALES)
def test_parity_sphere_reduced(G, l):
    """Single-object sphere across the surface-to-volume lengthscale sweep, reduced size."""
    _parity(G, sc.sphere_scene(l, width=64, height=64, spp=4), f"sphere l={l}")


def test_parity_mixed_reduced(G):
    """Union of 16 primitives with the full 128^3 variance grid, reduced image size."""
    _parity(G, _small_mixed(), "mixed16")


@pytest.mark.parametrize("target", [True, False])
def test_parity_offset_sphere(G, target):
    s = sc.offset_sphere_scene(target, width=64, height=64, spp=4)
    _parity(G, s, "offset_sphere target" if target else "offset_sphere theta0")


def test_chunked_equals_monolithic_and_deterministic(G):
    s = sc.sphere_scene(0.1, width=40, height=24, spp=12, max_depth=8)
    g = G.GpssScene(s)
    full = g.render_paths(0, 12).cpu().numpy()
    a = g.render_paths(0, 5).cpu().numpy()
    b = g.render_paths(5, 12).cpu().numpy()
    assert np.array_equal(np.concatenate([a, b], axis=2), full)
    img1 = g.render().cpu().numpy()
    img2 = g.render().cpu().numpy()
    assert np.array_equal(img1, img2)
    # the image is the per-pixel mean of the path radiances, in sample order
    assert np.allclose(img1, full.mean(axis=2), rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("w,h,spp,s0", [(1, 1, 1, 0), (37, 23, 3, 2), (5, 7, 1, 9)])
def test_ragged_and_tiny_sizes(G, w, h, spp, s0):
    s = sc.sphere_scene(0.02, width=w, height=h, spp=spp + s0, max_depth=8)
    _parity(G, s, f"ragged {w}x{h}", s0, s0 + spp)


def test_white_furnace_gpu(G):
    s = sc.plane_scene(width=32, height=32, spp=32, max_depth=64, albedo=1.0, env=1.0, light_E=0.0)
    _, img = _render(G, s)
    ref = orc.OracleScene(s).render()
    tot = img.mean() + ref["trunc"].mean()
    assert abs(tot - 1.0) < 5 * math.sqrt(ref["var"].mean() / (s.spp * s.n_pixels)) + 1e-3


def _sphere_small(**kw):
    return sc.sphere_scene(0.1, width=40, height=40, spp=4, max_depth=8).replace(**kw)


def _box_union():
    s = sc.mixed_scene(width=40, height=40, spp=2, max_depth=16, n_prims=6, var_res=16)
    p = s.prims.copy()
    sph = p[:, 0] == sc.PRIM_SPHERE
    p[sph, 0] = sc.PRIM_BOX
    p[sph, 5] = p[sph, 4]
    p[sph, 6] = p[sph, 4]
    return s.replace(prims=p, name="box_union")


DEGENERATE = {
    # no real scattering allowed: paths end at their first real collision (only escapes count)
    "depth0": lambda: _sphere_small(max_depth=0),
    # black medium: light arrives only along paths that escape without a real collision
    "albedo0": lambda: _sphere_small(albedo=0.0),
    # camera inside the medium's box and inside the surface (dense interior)
    "camera_inside": lambda: _sphere_small(cam_eye=(0.0, 0.1, 0.3), cam_target=(0.0, 0.0, -1.0)),
    # boxes only, per-primitive albedo, variance grid
    "box_union": _box_union,
}


@pytest.mark.parametrize("name", sorted(DEGENERATE))
def test_degenerate_scenes_parity(G, name):
    s = DEGENERATE[name]()
    _parity(G, s, name)


def test_no_light_gives_exact_zero(G):
    s = _sphere_small(point_light=np.zeros(4, np.float32), env_radiance=0.0)
    _, img = _render(G, s)
    assert np.count_nonzero(img) == 0


def test_empty_medium_gives_exact_environment(G):
    """A constant mean far above the shell: every majorant cell rounds to 0 (skipped), so every
    path escapes at once and sees the environment exactly."""
    s = _sphere_small().replace(mean_kind=sc.MEAN_CONST, mean_const=50.0, prims=np.zeros((0, 8), np.float32))
    g, img = _render(G, s)
    assert np.count_nonzero(g.majorants()) == 0
    assert np.all(img == np.float32(s.env_radiance))
    ref = orc.OracleScene(s).render()
    assert np.all(ref["mean"] == np.float32(s.env_radiance))


def test_depth0_equals_albedo0_bitwise(G):
    """Depth 0 ends each path at its first real collision; albedo 0 zeroes the throughput and
    every light term there: the same path radiances."""
    a = G.GpssScene(DEGENERATE["depth0"]()).render().cpu().numpy()
    b = G.GpssScene(DEGENERATE["albedo0"]()).render().cpu().numpy()
    assert np.array_equal(a, b)


def test_oversized_sample_range_is_rejected_before_allocation(G):
    """16384^2 pixels x 8 samples = 2^31 paths: one more than a call may render."""
    s = sc.sphere_scene(0.1, width=16384, height=16384, spp=8, max_depth=1)
    g = G.GpssScene(s)
    img = torch.empty(s.height, s.width, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    with pytest.raises(G.GpssError, match="at most 2"):
        g.render(0, 8, out=img)
    # no 8 GiB per-path buffer was allocated for the rejected call
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)
    del img
