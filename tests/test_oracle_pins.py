"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks an oracle function against an independent computation: published
known answers, definitions evaluated by quadrature or Monte Carlo, textbook special
cases, exact identities or closed forms derived from the paper's equations.
"""
import math
import os

import numpy as np
import pytest
from scipy import special, stats

from gpss_inputs import scenes as sc
from oracle import oracle as orc
from tests import refmath as ref

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Random numbers
# ---------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert list(out) == v[6:10]


def test_uniform_addressing():
    """Uniform k of stream (pixel, sample, bounce, stream) is word k%4 of the Philox block
    k//4 at counter (pixel, sample, bounce | stream<<16, block), top 24 bits."""
    seed, sid = 0x0123456789ABCDEF, 7
    key = [seed & 0xFFFFFFFF, (seed >> 32) ^ sid]
    u = orc.uniforms(seed, sid, 11, 3, 5, 2, 9)
    for k in range(9):
        blk = orc.philox([11, 3, 5 | (2 << 16), k // 4], key)
        assert u[k] == (int(blk[k % 4]) >> 8) / 2.0 ** 24


# ---------------------------------------------------------------------------
# Special functions
# ---------------------------------------------------------------------------
def test_erfcx_and_erfinv_against_scipy():
    xs = np.concatenate([np.linspace(-20, 5, 301), np.geomspace(5, 1e4, 200)])
    for x in xs:
        assert orc.erfcx(x) == pytest.approx(special.erfcx(x), rel=2e-13)
    ys = np.concatenate([np.linspace(-0.999999, 0.999999, 401), [1 - 2 ** -24, -1 + 2 ** -24]])
    for y in ys:
        assert orc.erfinv(y) == pytest.approx(special.erfinv(y), rel=1e-12, abs=1e-15)


# ---------------------------------------------------------------------------
# Density (Eq. h_density mapped to the SDF, Sec. 4)
# ---------------------------------------------------------------------------
def test_rho_matches_gaussian_ratio_and_is_monotone():
    for sigma in (0.01, 0.05, 0.1, 1.0):
        mus = np.linspace(-60 * sigma, 20 * sigma, 400)
        vals = [orc.rho(m, sigma) for m in mus]
        for m, v in zip(mus, vals):
            assert v == pytest.approx(ref.rho_reference(m, sigma), rel=1e-11)
        assert np.all(np.diff(vals) < 0)          # Fig. monotonic_density


# ---------------------------------------------------------------------------
# Projected area (Eqs. generalized_sigma_t, generalized_lambda, complex_sigma_t)
# ---------------------------------------------------------------------------
def _rand_dir(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_projected_area_is_negative_part_mean():
    """sigma(w) = E[max(0, -w.g)] with g ~ N(grad mu, s^2 I) (the numerator of
    Eq. complex_sigma_t), for unit and non-unit mean gradients and both travel senses."""
    rng = np.random.default_rng(1)
    for _ in range(40):
        G = _rand_dir(rng) * rng.choice([1.0, 0.6, 1.4])
        s = rng.choice([0.02, 0.1, 0.5, 2.0])
        d = _rand_dir(rng)
        want = ref.projected_area_by_expectation(d, G, np.full(3, s * s))
        got = orc.sigma_proj(G, s, d)
        assert got == pytest.approx(want, rel=1e-8, abs=1e-300)
    # |G| = 0: E[max(0, X)], X ~ N(0, s^2)
    assert orc.sigma_proj([0, 0, 0], 0.3, [0, 0, 1]) == pytest.approx(0.3 / math.sqrt(2 * math.pi))


def test_generalized_lambda_anisotropic_definition():
    """Eq. generalized_lambda with three roughnesses equals E[max(0, -w.g)] for
    g ~ N((0,0,1), diag(alpha^2 / 2)) divided by cos(theta)."""
    rng = np.random.default_rng(2)
    for _ in range(30):
        ax, ay, az = rng.uniform(0.1, 2.0, 3)
        w = _rand_dir(rng)
        if abs(w[2]) < 0.05:
            continue
        want = ref.projected_area_by_expectation(w, np.array([0, 0, 1.0]),
                                                 np.array([ax, ay, az]) ** 2 / 2) / w[2]
        assert orc.lambda_aniso(ax, ay, az, w) == pytest.approx(want, rel=1e-8)


# ---------------------------------------------------------------------------
# NDF (Eq. macro_ndf, Appendix A) and the identities it satisfies
# ---------------------------------------------------------------------------
def test_ndf_equals_gdf_integral():
    """Eq. macro_ndf equals its defining integral int_0^inf P(t wm) t^3 dt (Eq. gdf_to_ndf)
    with g' ~ N((0,0,1), diag(alpha^2/2)) (Eq. gdf)."""
    rng = np.random.default_rng(3)
    for _ in range(40):
        ax, ay, az = rng.uniform(0.15, 3.0, 3)
        wm = _rand_dir(rng)
        want = ref.ndf_by_gdf(wm, np.array([0, 0, 1.0]), np.array([ax, ay, az]) ** 2 / 2)
        assert orc.ndf_aniso(ax, ay, az, wm) == pytest.approx(want, rel=1e-8, abs=1e-250)
    # isotropic form for an arbitrary mean gradient G (reading: g ~ N(G, s^2 I))
    for _ in range(30):
        G = _rand_dir(rng) * rng.uniform(0.3, 1.5)
        s = rng.uniform(0.05, 1.5)
        wm = _rand_dir(rng)
        want = ref.ndf_by_gdf(wm, G, np.full(3, s * s))
        assert orc.ndf(G, s, wm) == pytest.approx(want, rel=1e-8, abs=1e-250)


def test_height_field_limit_is_beckmann():
    """alpha_z -> 0 (l_z -> inf): Eq. macro_ndf -> Beckmann NDF and Eq. generalized_lambda
    -> the Beckmann Smith Lambda (Sec. 4.1 / 4.2); the error shrinks like alpha_z^2."""
    for alpha in (0.1, 0.3, 0.7, 1.0):
        for th in (0.05, 0.3, 0.7, 1.1):
            wm = np.array([math.sin(th) * 0.6, math.sin(th) * 0.8, math.cos(th)])
            want = ref.beckmann_D(alpha, math.cos(th))
            got1 = orc.ndf_aniso(alpha, alpha, 1e-3, wm)
            got2 = orc.ndf_aniso(alpha, alpha, 1e-4, wm)
            e1 = abs(got1 / want - 1)
            e2 = abs(got2 / want - 1)
            assert e2 < 2e-3 and e2 < 0.02 * e1 + 1e-6   # O(alpha_z^2) convergence
            a = math.cos(th) / (alpha * math.sin(th))
            assert orc.lambda_aniso(alpha, alpha, 1e-5, wm) == pytest.approx(
                ref.beckmann_lambda(a), rel=1e-6, abs=1e-14)
            assert orc.beckmann_ndf(alpha, math.cos(th)) == pytest.approx(want, rel=1e-12)
            assert orc.beckmann_lambda(a) == pytest.approx(ref.beckmann_lambda(a), rel=1e-12,
                                                           abs=1e-300)


def test_vndf_normalizer_equals_projected_area():
    """int <-w, wm> D(wm) dwm = sigma(w) exactly (Sec. 4.2.2, Fig. generalized_projected_area)."""
    rng = np.random.default_rng(4)
    for _ in range(6):
        G = _rand_dir(rng) * rng.uniform(0.7, 1.3)
        s = rng.choice([0.25, 0.7, 2.0])
        w = _rand_dir(rng)
        dirs, W = ref.sphere_grid(-w, 160, 200, hemisphere=True)
        vals = np.array([orc.ndf(G, s, m) for m in dirs]) * (dirs @ (-w))
        assert float(np.sum(vals * W)) == pytest.approx(orc.sigma_proj(G, s, w), rel=1e-6)


def test_signed_projected_area():
    """int (w.wm) D(wm) dwm = w.grad mu (Eq. spa, read with w_g on the right)."""
    rng = np.random.default_rng(5)
    for _ in range(6):
        G = _rand_dir(rng) * rng.uniform(0.7, 1.3)
        s = rng.choice([0.25, 0.7, 2.0])
        w = _rand_dir(rng)
        dirs, W = ref.sphere_grid(G, 200, 160)
        vals = np.array([orc.ndf(G, s, m) for m in dirs]) * (dirs @ w)
        assert float(np.sum(vals * W)) == pytest.approx(float(np.dot(w, G)), rel=1e-6, abs=1e-7)


# ---------------------------------------------------------------------------
# Phase function (Eqs. phase, microfacet_vndf) and its sampling
# ---------------------------------------------------------------------------
def test_phase_normalization_and_reciprocity():
    rng = np.random.default_rng(6)
    for _ in range(5):
        G = _rand_dir(rng)
        s = rng.choice([0.3, 0.8, 2.0])
        d = _rand_dir(rng)
        alb = 0.7
        dirs, W = ref.sphere_grid(-d, 200, 200)
        p = np.array([orc.phase_eval(G, s, alb, d, wi) for wi in dirs])
        assert float(np.sum(p * W)) == pytest.approx(alb, rel=2e-4)
        # reciprocity: sigma(d) p(d -> wi) = sigma(-wi) p(-wi -> -d)
        for _ in range(10):
            wi = _rand_dir(rng)
            lhs = orc.sigma_proj(G, s, d) * orc.phase_eval(G, s, alb, d, wi)
            rhs = orc.sigma_proj(G, s, -wi) * orc.phase_eval(G, s, alb, -wi, -d)
            assert lhs == pytest.approx(rhs, rel=1e-10)


def test_homogeneous_phase_is_isotropic():
    """Constant mean (grad mu = 0): the phase function is albedo / (4 pi) (Sec. 3.1)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        d, wi = _rand_dir(rng), _rand_dir(rng)
        assert orc.phase_eval([0, 0, 0], 0.37, 0.8, d, wi) == pytest.approx(0.8 / (4 * math.pi),
                                                                            rel=1e-12)


def test_mixture_pdf_normalized():
    rng = np.random.default_rng(8)
    for _ in range(5):
        G = _rand_dir(rng)
        s = rng.choice([0.3, 0.8, 2.0])
        d = _rand_dir(rng)
        dirs, W = ref.sphere_grid(G, 240, 240)
        p = np.array([orc.mixture_pdf(G, s, 0.5, d, m) for m in dirs])
        assert float(np.sum(p * W)) == pytest.approx(1.0, rel=2e-4)


def _u24(rng, n):
    return rng.integers(0, 2 ** 24, size=(n, 3)) / 2.0 ** 24


def test_phase_sampler_weight_is_unbiased():
    """E[weight] = albedo and E[weight * f(wi)] = int p f dwi for the mixture sampler
    (R = 0.5, and uniform-only R = 0), weight = albedo D_wo(wm) / pdf_mix(wm).  (R = 1 is
    not unbiased: the Beckmann proposal never reaches normals facing away from grad mu.)"""
    rng = np.random.default_rng(9)
    for R in (0.5, 0.0):
        for G, s, d in (([0, 0, 1.0], 0.4, [0.6, 0, -0.8]), ([0.3, -0.2, 0.9], 1.2, [0, 0.6, -0.8]),
                        ([0, 0, 1.0], 0.15, [0.9, 0, -0.43589])):
            d = np.asarray(d) / np.linalg.norm(d)
            n = 20000
            U = _u24(rng, n)
            ws, fz = np.zeros(n), np.zeros(n)
            for k in range(n):
                wi, wm, w, p = orc.phase_sample(G, s, 0.8, R, d, U[k])
                ws[k], fz[k] = w, w * wi[2]
            dirs, W = ref.sphere_grid(-d, 160, 200)
            p = np.array([orc.phase_eval(G, s, 0.8, d, wi) for wi in dirs])
            want_fz = float(np.sum(p * dirs[:, 2] * W))
            assert abs(ws.mean() - 0.8) < 5 * ws.std() / math.sqrt(n) + 1e-12
            assert abs(fz.mean() - want_fz) < 5 * fz.std() / math.sqrt(n) + 1e-12


def test_beckmann_vndf_sampler_histogram():
    """Half vectors drawn with R = 1 follow the Beckmann visible-normal density: chi^2 of a
    cos(theta_m) histogram against the quadrature of the same pdf over each bin."""
    rng = np.random.default_rng(10)
    G, s = np.array([0, 0, 1.0]), 0.3
    d = np.array([0.5, 0.0, -math.sqrt(0.75)])
    n = 40000
    U = _u24(rng, n)
    U[:, 0] = 0.0   # always the Beckmann component
    cos_m = np.array([orc.phase_sample(G, s, 1.0, 1.0, d, U[k])[1][2] for k in range(n)])
    edges = np.linspace(0.55, 1.0, 16)
    obs, _ = np.histogram(cos_m, bins=edges)
    dirs, W = ref.sphere_grid(G, 400, 256, hemisphere=True)
    pdf = np.array([orc.mixture_pdf(G, s, 1.0, d, m) for m in dirs])
    exp = np.array([np.sum((pdf * W)[(dirs[:, 2] >= a) & (dirs[:, 2] < b)])
                    for a, b in zip(edges[:-1], edges[1:])]) * n
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-3
    assert np.sum(cos_m < edges[0]) < 0.002 * n


# ---------------------------------------------------------------------------
# Tracking and transmittance (Eqs. sm2tr and generalized_sigma_t, Sec. 5)
# ---------------------------------------------------------------------------
def test_planar_transmittance_closed_form():
    """Ratio tracking through the planar GPSS reproduces the closed form
    Tr = (Phi(z0/s)/Phi(z1/s))^(sigma(d)/d_z) (integral of Eq. generalized_sigma_t, Fig. tr)."""
    scene = sc.plane_scene(majorant_res=(2, 2, 16))
    o_s = orc.OracleScene(scene)
    sigma = math.sqrt(orc.f32(0.01))
    s0 = sigma / orc.f32(0.05)
    for d, z0, t in (([0.6, 0.0, 0.8], -0.1, 0.3), ([0.0, 0.6, -0.8], 0.35, 0.5),
                     ([0.8, 0.0, 0.6], -0.05, 0.4)):
        d = np.asarray(d)
        o = np.array([0.2, 0.2, z0])
        proj = ref.projected_area_by_expectation(d, np.array([0, 0, 1.0]), np.full(3, s0 * s0))
        want = ref.planar_transmittance(z0, z0 + t * d[2], d[2], sigma, proj)
        T = o_s.ratio_tracking(o, d, t, 40000)
        assert abs(T.mean() - want) < 5 * T.std() / math.sqrt(T.size) + 1e-9
        # free flights: P(t_hit > tau) = Tr(tau) (Kolmogorov-Smirnov on the hit distances)
        th = o_s.free_flight(o, d, t, 20000)
        frac_esc = np.mean(np.isinf(th))
        assert abs(frac_esc - want) < 5 * math.sqrt(want * (1 - want) / th.size) + 1e-9
        hits = th[np.isfinite(th)]

        def cdf(tau):
            tau = np.atleast_1d(tau)
            return np.array([(1 - ref.planar_transmittance(z0, z0 + x * d[2], d[2], sigma, proj))
                             / (1 - want) for x in tau])
        assert stats.kstest(hits, cdf).pvalue > 1e-3


def test_homogeneous_medium_transmittance():
    """Constant mean c: sigma_t = rho(c) s / sqrt(2 pi) and Tr = exp(-sigma_t t) (Sec. 3.1)."""
    scene = sc.plane_scene(majorant_res=(4, 4, 4)).replace(mean_kind=sc.MEAN_CONST,
                                                            mean_const=0.05)
    o_s = orc.OracleScene(scene)
    sigma = math.sqrt(orc.f32(0.01))
    s0 = sigma / orc.f32(0.05)
    st = ref.rho_reference(orc.f32(0.05), sigma) * s0 / math.sqrt(2 * math.pi)
    for t in (0.02, 0.05, 0.1):
        T = o_s.ratio_tracking([0.1, 0.1, -0.3], [0.6, 0.0, 0.8], t, 40000)
        want = math.exp(-st * t)
        assert abs(T.mean() - want) < 5 * T.std() / math.sqrt(T.size) + 1e-12


def test_majorants_bound_extinction():
    """Every majorant bounds sigma_t at random points of its cell for random directions."""
    rng = np.random.default_rng(11)
    scs = [sc.plane_scene(), sc.sphere_scene(0.02, majorant_res=(16, 16, 16)),
           sc.mixed_scene(var_res=32, majorant_res=(12, 12, 12)),
           sc.offset_sphere_scene(True, grid_res=16, offset_std=0.05, majorant_res=(16, 16, 16))]
    for s in scs:
        o_s = orc.OracleScene(s)
        maj = o_s.majorants()
        M = np.array(s.majorant_res)
        lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
        cells = rng.integers(0, maj.size, 300)
        for c in cells:
            k = np.array([c % M[0], (c // M[0]) % M[1], c // (M[0] * M[1])])
            for _ in range(6):
                x = lo + (k + rng.random(3)) * (hi - lo) / M
                d = _rand_dir(rng)
                st = o_s.sigma_t(x, d)
                # cells whose bound is below 2^-40 are given majorant 0 (negligible density)
                assert st <= maj[c] or (maj[c] == 0.0 and st < 2.0 ** -40)


# ---------------------------------------------------------------------------
# Whole-estimator pins
# ---------------------------------------------------------------------------
def test_white_furnace():
    """Albedo 1, unit environment, no delta lights: every path either escapes with weight
    beta or is cut at the depth limit, so E[L] + E[cut beta] = 1 (phase normalization)."""
    cases = [sc.plane_scene(width=16, height=16, spp=64, max_depth=256, albedo=1.0, env=1.0,
                            light_E=0.0),
             sc.sphere_scene(0.1, width=16, height=16, spp=64, max_depth=256,
                             albedo=1.0, majorant_res=(16, 16, 16))]
    cases[1].env_radiance = 1.0
    cases[1].point_light = np.zeros(4, np.float32)
    for s in cases:
        r = orc.OracleScene(s).render()
        tot = r["mean"] + r["trunc"]
        se = math.sqrt(r["var"].mean() / (s.spp * s.n_pixels))
        assert abs(tot.mean() - 1.0) < 5 * se + 1e-3 * r["trunc"].mean() + 1e-12
        assert r["counters"]["violations"] == 0


def test_planar_single_scattering_closed_form():
    """Depth 1 on the planar GPSS: I = albedo E D(w_h) / (4 cos_v (1 + L(v) + L(l))), with
    1 + L(v) = sigma(-v)/cos_v and L(l) = sigma(l)/cos_l, up to the (Phi_b/Phi_t)^n leak of the
    bounded shell; independent of sigma."""
    s = sc.plane_scene(width=32, height=32, spp=256, max_depth=1)
    r = orc.OracleScene(s).render()
    sigma = math.sqrt(orc.f32(0.01))
    s0 = sigma / orc.f32(0.05)
    cov = np.full(3, s0 * s0)
    G = np.array([0, 0, 1.0])
    v = np.array([math.sin(math.pi / 4), 0, math.cos(math.pi / 4)])
    ld = np.asarray(s.dir_light[:3], float)
    n = (ref.projected_area_by_expectation(-v, G, cov) / v[2]
         + ref.projected_area_by_expectation(ld, G, cov) / ld[2])
    h = (v + ld) / np.linalg.norm(v + ld)
    D = ref.ndf_by_gdf(h, G, cov)
    leak = (special.ndtr(-0.4 / sigma) / special.ndtr(0.4 / sigma)) ** n
    want = 0.9 * 1.0 * D / (4 * v[2] * n) * (1 - leak)
    inner = r["mean"][10:22, 10:22]
    se = math.sqrt(r["var"][10:22, 10:22].mean() / (s.spp * inner.size))
    assert abs(inner.mean() - want) < 5 * se
    assert want == pytest.approx(0.087221, abs=2e-6)


def test_frozen_sampling_reduces_to_forward():
    s = sc.offset_sphere_scene(False, width=24, height=24, spp=4, max_depth=6, grid_res=16,
                               majorant_res=(16, 16, 16))
    a = orc.OracleScene(s)
    r = a.render()
    f = a.render_frozen(a)
    assert np.array_equal(r["mean"], f)


def test_chunked_render_equals_monolithic():
    s = sc.plane_scene(width=16, height=16, spp=8)
    o_s = orc.OracleScene(s)
    full = o_s.render(0, 8, want_paths=True)
    a = o_s.render(0, 3, want_paths=True)
    b = o_s.render(3, 8, want_paths=True)
    assert np.array_equal(np.concatenate([a["paths"], b["paths"]], axis=2), full["paths"])


def test_dual_gradient_matches_central_differences():
    """Gradient of the frozen-sampling estimator (decisions at theta0, weights at theta) by
    dual numbers equals central differences of the same estimator (h = 1e-4)."""
    s0 = sc.offset_sphere_scene(False, width=20, height=20, spp=4, max_depth=8, grid_res=16,
                                majorant_res=(16, 16, 16))
    s0.offset_grid = (np.random.default_rng(5).normal(0, 0.01, s0.offset_grid.shape)
                      .astype(np.float32))
    base = orc.OracleScene(s0)
    img0 = base.render()["mean"]
    rng = np.random.default_rng(12)
    dloss = rng.normal(size=img0.shape)
    nodes = sc.grad_param_indices(s0, n_nodes=6, seed=3)
    ids = [-1, -2, -3] + [int(i) for i in nodes]
    g, img = base.render_grad(dloss, ids)
    assert np.allclose(img, img0, rtol=0, atol=1e-12)
    h = 1e-4
    for j, pid in enumerate(ids):
        imgs = []
        for sgn in (+1, -1):
            if pid == -1:
                pert = s0.replace(variance=float(orc.f32(s0.variance)) * (1 + sgn * h))
                scale = float(orc.f32(s0.variance)) * h
            elif pid == -2:
                pert = s0.replace(lengthscale=float(orc.f32(s0.lengthscale)) * (1 + sgn * h))
                scale = float(orc.f32(s0.lengthscale)) * h
            elif pid == -3:
                pert = s0.replace(albedo=float(orc.f32(s0.albedo)) * (1 + sgn * h))
                scale = float(orc.f32(s0.albedo)) * h
            else:
                off = s0.offset_grid.astype(np.float64).copy()
                off.ravel()[pid] += sgn * 1e-5
                pert = s0.replace(offset_grid=off.astype(np.float32))
                scale = float(np.float32(off.ravel()[pid])) - float(s0.offset_grid.ravel()[pid])
                scale = abs(scale)
            imgs.append(base.render_frozen(_unrounded(pert)))
        fd = float(np.sum(dloss * (imgs[0] - imgs[1]))) / (2 * scale)
        assert g[j] == pytest.approx(fd, rel=2e-4, abs=1e-9 * max(1.0, abs(fd)))


def _unrounded(scene):
    """Oracle scene whose scalar parameters keep their double values (finite differences
    need perturbations smaller than float32 resolution)."""
    o = orc.OracleScene(scene)
    d = o._desc
    d.variance = float(scene.variance)
    d.lengthscale = float(scene.lengthscale)
    d.albedo = float(scene.albedo)
    import ctypes
    h = ctypes.c_void_p()
    assert orc.lib().oracle_scene_create(ctypes.byref(d), ctypes.byref(h)) == 0
    orc.lib().oracle_scene_destroy(o.handle)
    o.handle = h
    return o


def test_pixel_list_render_equals_full_render():
    s = sc.sphere_scene(0.1, width=24, height=20, spp=3, max_depth=6)
    o = orc.OracleScene(s)
    full = o.render()
    px = np.array([0, 7, 133, 479, 250])
    r = o.render_pixels(px)
    assert np.array_equal(r["mean"], full["mean"].ravel()[px])
    assert np.allclose(r["var"], full["var"].ravel()[px], rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------
# Anisotropic kernel: lengthscale l across and l_n along the local mean-gradient direction
# (Eq. se_kernel in the frame of the geometric normal; Eqs. generalized_lambda and
# macro_ndf with alpha_x = alpha_y != alpha_z)
# ---------------------------------------------------------------------------
def _aniso_cases(rng, n):
    for k in range(n):
        G = np.zeros(3) if k % 5 == 0 else _rand_dir(rng) * rng.choice([1.0, 0.5, 1.6])
        s = float(rng.choice([0.05, 0.3, 1.0]))
        sn = float(rng.choice([0.01, 0.2, 0.7, 2.5]))
        yield G, s, sn, _rand_dir(rng)


def test_anisotropic_projected_area_is_negative_part_mean():
    rng = np.random.default_rng(31)
    for G, s, sn, d in _aniso_cases(rng, 40):
        want = ref.projected_area_full(d, G, ref.aniso_cov(G, s, sn))
        assert orc.sigma_proj_n(G, s, sn, d) == pytest.approx(want, rel=1e-8, abs=1e-300)


def test_anisotropic_ndf_equals_gdf_integral():
    rng = np.random.default_rng(32)
    for G, s, sn, wm in _aniso_cases(rng, 40):
        want = ref.ndf_by_gdf_full(wm, G, ref.aniso_cov(G, s, sn))
        assert orc.ndf_n(G, s, sn, wm) == pytest.approx(want, rel=1e-7, abs=1e-300)


def test_anisotropic_identities_on_the_sphere():
    """Signed projected area (Eq. spa) and vNDF normalizer = projected area
    (Fig. generalized_projected_area) for alpha_z != alpha_x = alpha_y."""
    rng = np.random.default_rng(33)
    for G, s, sn in [(np.array([0.0, 0.0, 1.0]), 0.4, 0.05), (np.array([0.3, -0.5, 0.8]), 0.2, 0.9),
                     (np.zeros(3), 0.5, 0.2)]:
        dirs, W = ref.sphere_grid(G if np.linalg.norm(G) > 0 else [0, 0, 1.0], 400, 256)
        D = np.array([orc.ndf_n(G, s, sn, w) for w in dirs])
        for _ in range(3):
            w = _rand_dir(rng)
            signed = float(np.sum(W * (dirs @ w) * D))
            assert signed == pytest.approx(float(np.dot(w, G)), abs=2e-6 * max(1.0, np.linalg.norm(G)))
            # visible part: a hemisphere grid about -w, aligned with the kink of max(0, .)
            hd, hw = ref.sphere_grid(-w, 600, 400, hemisphere=True)
            vis = float(np.sum(hw * (hd @ (-w)) * np.array([orc.ndf_n(G, s, sn, m) for m in hd])))
            assert vis == pytest.approx(orc.sigma_proj_n(G, s, sn, w), rel=2e-5)


def test_anisotropic_reduces_to_isotropic_and_height_field():
    rng = np.random.default_rng(34)
    for _ in range(10):
        G = _rand_dir(rng) * 0.8
        s = 0.3
        w = _rand_dir(rng)
        assert orc.sigma_proj_n(G, s, s, w) == pytest.approx(orc.sigma_proj(G, s, w), rel=1e-13)
        assert orc.ndf_n(G, s, s, w) == pytest.approx(orc.ndf(G, s, w), rel=1e-13)
    # s_n -> 0 about n = z with |G| = 1: the Beckmann NDF of roughness sqrt(2) s (height field)
    s = 0.25
    for c in (0.95, 0.8, 0.5):
        wm = np.array([math.sqrt(1 - c * c), 0.0, c])
        e1 = abs(orc.ndf_n([0, 0, 1.0], s, 1e-3, wm) / ref.beckmann_D(math.sqrt(2) * s, c) - 1)
        e2 = abs(orc.ndf_n([0, 0, 1.0], s, 5e-4, wm) / ref.beckmann_D(math.sqrt(2) * s, c) - 1)
        assert e1 < 2e-3 and e2 < 0.3 * e1 + 1e-9


def test_planar_single_scattering_anisotropic():
    """The depth-1 planar closed form with an anisotropic kernel (l_n along the plane normal):
    the same formula with the full-covariance projected areas and NDF (Eqs.
    generalized_lambda, macro_ndf with alpha_z != alpha_x = alpha_y)."""
    ln = 0.2
    s = sc.plane_scene(width=32, height=32, spp=256, max_depth=1).replace(lengthscale_n=ln)
    r = orc.OracleScene(s).render()
    assert r["counters"]["violations"] == 0
    sigma = math.sqrt(orc.f32(0.01))
    s0, sn = sigma / orc.f32(0.05), sigma / orc.f32(ln)
    G = np.array([0, 0, 1.0])
    cov = ref.aniso_cov(G, s0, sn)
    v = np.array([math.sin(math.pi / 4), 0, math.cos(math.pi / 4)])
    ld = np.asarray(s.dir_light[:3], float)
    n = ref.projected_area_full(-v, G, cov) / v[2] + ref.projected_area_full(ld, G, cov) / ld[2]
    h = (v + ld) / np.linalg.norm(v + ld)
    D = ref.ndf_by_gdf_full(h, G, cov)
    leak = (special.ndtr(-0.4 / sigma) / special.ndtr(0.4 / sigma)) ** n
    want = 0.9 * 1.0 * D / (4 * v[2] * n) * (1 - leak)
    inner = r["mean"][10:22, 10:22]
    se = math.sqrt(r["var"][10:22, 10:22].mean() / (s.spp * inner.size))
    assert abs(inner.mean() - want) < 5 * se
    # and it differs from the isotropic value by far more than the noise
    assert abs(want - 0.087221) > 20 * se


# ---------------------------------------------------------------------------
# GGX height-field macrofacet (end of Sec. 4.1: the NDF may be chosen freely under the
# Smith assumption; Fig. cmp_ggx): D and Lambda of GGX about n = G/|G|, roughness
# sqrt(2) s / |G|, scaled by |G|
# ---------------------------------------------------------------------------
def test_ggx_ndf_identities_by_quadrature():
    rng = np.random.default_rng(41)
    for G, s in ((np.array([0, 0, 1.0]), 0.3), (np.array([0.4, -0.3, 0.7]), 0.6), (np.array([0.0, 1.3, 0.0]), 0.1)):
        dirs, W = ref.sphere_grid(G, 1200, 96, hemisphere=True)
        D = np.array([orc.ndf_ggx(G, s, m) for m in dirs])
        gn = np.linalg.norm(G)
        n = G / gn
        assert float(np.sum(W * (dirs @ n) * D)) == pytest.approx(gn, rel=2e-5)   # projected area of the micro-surface
        for _ in range(3):
            w = _rand_dir(rng)
            assert float(np.sum(W * (dirs @ w) * D)) == pytest.approx(float(w @ G), abs=5e-5 * gn)
            vis = float(np.sum(W * np.maximum(0.0, dirs @ (-w)) * D))
            assert vis == pytest.approx(orc.sigma_proj_ggx(G, s, w), rel=1e-3, abs=1e-6)
        # textbook values about the normal
        alpha = math.sqrt(2) * s / gn
        for c in (1.0, 0.9, 0.5):
            m = c * n + math.sqrt(1 - c * c) * ref.frame(n)[0]
            assert orc.ndf_ggx(G, s, m) == pytest.approx(gn * ref.ggx_D(alpha, c), rel=1e-12)


def test_ggx_projected_area_is_cos_one_plus_lambda():
    rng = np.random.default_rng(42)
    for _ in range(30):
        G = _rand_dir(rng) * rng.choice([1.0, 0.6, 1.4])
        s = float(rng.choice([0.05, 0.3, 1.0]))
        w = _rand_dir(rng)
        gn = np.linalg.norm(G)
        alpha = math.sqrt(2) * s / gn
        c = -float(w @ G) / gn   # cosine of the back-travel direction with n
        want = gn * (c * (1 + ref.ggx_lambda(alpha, c)) if c > 0 else -c * ref.ggx_lambda(alpha, -c))
        assert orc.sigma_proj_ggx(G, s, w) == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_ggx_phase_normalization_and_sampler():
    rng = np.random.default_rng(43)
    G, s, alb = np.array([0.2, 0.1, 0.9]), 0.25, 0.7
    for d in (np.array([0.5, 0.0, -math.sqrt(0.75)]), np.array([0.0, 0.6, 0.8])):
        dirs, W = ref.sphere_grid(-d, 600, 400)
        p = np.array([orc.phase_eval(G, s, alb, d, wi, ggx=True) for wi in dirs])
        assert float(np.sum(p * W)) == pytest.approx(alb, rel=2e-3)
        n = 20000
        U = _u24(rng, n)
        ws = np.array([orc.phase_sample(G, s, alb, 0.5, d, U[k], ggx=True)[2] for k in range(n)])
        assert abs(ws.mean() - alb) < 5 * ws.std() / math.sqrt(n) + 1e-12


def test_ggx_vndf_sampler_histogram():
    """R = 1: half vectors follow the textbook GGX visible-normal density
    <v, m> D(m) / (cos_v (1 + Lambda(v)))."""
    rng = np.random.default_rng(44)
    G, s = np.array([0, 0, 1.0]), 0.35
    alpha = math.sqrt(2) * s
    d = np.array([0.6, 0.0, -0.8])
    v = -d
    n = 40000
    U = _u24(rng, n)
    U[:, 0] = 0.0
    ms = np.array([orc.phase_sample(G, s, 1.0, 1.0, d, U[k], ggx=True)[1] for k in range(n)])
    edges = np.linspace(0.3, 1.0, 15)
    obs, _ = np.histogram(ms[:, 2], bins=edges)
    dirs, W = ref.sphere_grid(G, 600, 256, hemisphere=True)
    pdf = np.array([max(0.0, float(m @ v)) * ref.ggx_D(alpha, m[2]) for m in dirs])
    pdf /= v[2] * (1 + ref.ggx_lambda(alpha, v[2]))
    exp = np.array([np.sum((pdf * W)[(dirs[:, 2] >= a) & (dirs[:, 2] < b)])
                    for a, b in zip(edges[:-1], edges[1:])]) * n
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-3
    assert np.all(ms[:, 2] > 0)


def test_planar_single_scattering_ggx_surface_limit():
    """Depth 1 on a GGX planar macrofacet: the GGX microfacet BRDF with the Smith
    height-correlated masking-shadowing, I = albedo E D(h) / (4 cos_v (1 + L(v) + L(l)))
    (surface limit, Fig. cmp_ggx), up to the bounded shell's leak."""
    s = sc.plane_scene(width=32, height=32, spp=256, max_depth=1).replace(ndf_kind=sc.NDF_GGX)
    r = orc.OracleScene(s).render()
    assert r["counters"]["violations"] == 0
    sigma = math.sqrt(orc.f32(0.01))
    alpha = math.sqrt(2) * sigma / orc.f32(0.05)
    v = np.array([math.sin(math.pi / 4), 0, math.cos(math.pi / 4)])
    ld = np.asarray(s.dir_light[:3], float)
    h = (v + ld) / np.linalg.norm(v + ld)
    lv, ll = ref.ggx_lambda(alpha, v[2]), ref.ggx_lambda(alpha, ld[2])
    n = (1 + lv) + ll
    leak = (special.ndtr(-0.4 / sigma) / special.ndtr(0.4 / sigma)) ** n
    want = 0.9 * 1.0 * ref.ggx_D(alpha, h[2]) / (4 * v[2] * n) * (1 - leak)
    inner = r["mean"][10:22, 10:22]
    se = math.sqrt(r["var"][10:22, 10:22].mean() / (s.spp * inner.size))
    assert abs(inner.mean() - want) < 5 * se


# ---------------------------------------------------------------------------
# Conductor Fresnel term (the F of Eq. phase with a complex index of refraction)
# ---------------------------------------------------------------------------
def test_fresnel_conductor_against_snell_form():
    for eta, k in ((0.2, 3.0), (1.5, 0.0), (0.05, 4.2), (2.5, 1.1), (1.0, 0.5)):
        for c in np.linspace(0.0, 1.0, 41):
            want = ref.fresnel_conductor_snell(c, eta, k)
            assert orc.fresnel_conductor(c, eta, k) == pytest.approx(want, rel=1e-12, abs=1e-15)
        # normal incidence and grazing limits
        assert orc.fresnel_conductor(1.0, eta, k) == pytest.approx(((eta - 1) ** 2 + k * k) / ((eta + 1) ** 2 + k * k),
                                                                   rel=1e-12)
        assert orc.fresnel_conductor(0.0, eta, k) == pytest.approx(1.0, rel=1e-12)


def test_planar_single_scattering_with_fresnel():
    """The planar depth-1 closed form with F = albedo x conductor Fresnel at the half vector
    (gold, approximately eta = 0.2, k = 3.0 at 600 nm)."""
    eta, k = 0.2, 3.0
    s = sc.plane_scene(width=32, height=32, spp=256, max_depth=1).replace(fresnel_eta=eta, fresnel_k=k)
    r = orc.OracleScene(s).render()
    assert r["counters"]["violations"] == 0
    sigma = math.sqrt(orc.f32(0.01))
    s0 = sigma / orc.f32(0.05)
    cov = np.full(3, s0 * s0)
    G = np.array([0, 0, 1.0])
    v = np.array([math.sin(math.pi / 4), 0, math.cos(math.pi / 4)])
    ld = np.asarray(s.dir_light[:3], float)
    n = (ref.projected_area_by_expectation(-v, G, cov) / v[2]
         + ref.projected_area_by_expectation(ld, G, cov) / ld[2])
    h = (v + ld) / np.linalg.norm(v + ld)
    D = ref.ndf_by_gdf(h, G, cov)
    F = 0.9 * ref.fresnel_conductor_snell(float(v @ h), orc.f32(eta), orc.f32(k))
    leak = (special.ndtr(-0.4 / sigma) / special.ndtr(0.4 / sigma)) ** n
    want = F * D / (4 * v[2] * n) * (1 - leak)
    inner = r["mean"][10:22, 10:22]
    se = math.sqrt(r["var"][10:22, 10:22].mean() / (s.spp * inner.size))
    assert abs(inner.mean() - want) < 5 * se


def test_fresnel_phase_normalization_and_sampler():
    """int p dwi = int F(<v, m>) D_v(m) dm (< albedo) and E[weight] equals it."""
    rng = np.random.default_rng(45)
    # the phase entry points take the scene-less form; a scene point carries the Fresnel term
    s = sc.plane_scene(width=4, height=4, spp=1).replace(fresnel_eta=0.2, fresnel_k=3.0)
    o = orc.OracleScene(s)
    x = np.array([0.5, 0.5, 0.02])
    d = np.array([0.5, 0.0, -math.sqrt(0.75)])
    e = o.eval_point(x)
    assert e["G"][2] == pytest.approx(1.0)
    dirs, W = ref.sphere_grid(-d, 300, 300)
    vis_d, vis_w = ref.sphere_grid(e["G"], 600, 256, hemisphere=False)
    D = np.array([orc.ndf(e["G"], e["s"], m) for m in vis_d])
    vm = np.maximum(0.0, vis_d @ (-d))
    Fm = np.array([orc.f32(e["albedo"]) * ref.fresnel_conductor_snell(c, orc.f32(0.2), orc.f32(3.0)) for c in vm])
    want = float(np.sum(vis_w * Fm * vm * D)) / orc.sigma_proj(e["G"], e["s"], d)
    got = float(np.sum(W * np.array([o.phase_eval_at(x, d, wi) for wi in dirs])))
    assert got == pytest.approx(want, rel=2e-3)
    assert want < e["albedo"]
