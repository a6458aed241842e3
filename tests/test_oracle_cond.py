"""Pins of the oracle's GP conditioning on point observations (Sec. 3.1, Eq. condition_gp)
and of the full-covariance medium it needs (projected area and generalized NDF for a
gradient g ~ N(m, Sigma) with an arbitrary covariance, Sec. 4.2).

Independent checks only: quadrature of the defining integrals, exact identities on the
sphere, reductions to the already pinned isotropic and anisotropic forms, the textbook
closed form of conditioning on one noisy observation, Bayes' rule by importance sampling on
a tiny problem, and derivative identities of the posterior mean and variance.
"""
import math

import numpy as np
import pytest

from gpss_inputs import scenes as sc
from oracle import oracle as orc
from tests import refmath as ref


def _rand_dir(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _rand_spd(rng, scale):
    A = rng.normal(size=(3, 3))
    return scale * scale * (A @ A.T / 3.0 + 0.2 * np.eye(3))


# ---------------------------------------------------------------------------
# Full-covariance projected area and NDF
# ---------------------------------------------------------------------------
def _peak(G, S):
    """NDF at the mean-gradient direction: the scale for absolute tolerances in the far tail
    (b << 0), where the closed form cancels and the NDF is < 1e-20 of this."""
    g = np.linalg.norm(G)
    return orc.ndf_cov(G, S, np.asarray(G) / g if g > 0 else [0, 0, 1.0])


def _cov_cases(rng, n):
    for k in range(n):
        G = _rand_dir(rng) * rng.choice([0.0, 0.3, 1.0, 1.7])
        S = _rand_spd(rng, float(rng.choice([0.05, 0.3, 1.0])))
        yield G, S, _rand_dir(rng)


def test_full_cov_projected_area_is_negative_part_mean():
    rng = np.random.default_rng(61)
    for G, S, d in _cov_cases(rng, 40):
        want = ref.projected_area_full(d, G, S)
        assert orc.sigma_proj_cov(G, S, d) == pytest.approx(want, rel=1e-8, abs=1e-300)


def test_full_cov_ndf_equals_gdf_integral():
    rng = np.random.default_rng(62)
    for G, S, wm in _cov_cases(rng, 40):
        want = ref.ndf_by_gdf_full(wm, G, S)
        assert orc.ndf_cov(G, S, wm) == pytest.approx(want, rel=1e-7, abs=1e-20 * _peak(G, S))


def test_full_cov_identities_on_the_sphere():
    """Signed projected area int D(m) (m.w) dm = w.G and the visible-normal normalizer
    int_{m.v > 0} D(m) (m.v) dm = sigma(-v) for a full covariance."""
    rng = np.random.default_rng(63)
    for G, S in [(np.array([0.2, -0.4, 0.9]), _rand_spd(rng, 0.3)),
                 (np.array([0.0, 0.6, 0.3]), _rand_spd(rng, 0.15)),
                 (np.zeros(3), _rand_spd(rng, 0.5))]:
        ax = G if np.linalg.norm(G) > 0 else np.array([0, 0, 1.0])
        dirs, W = ref.sphere_grid(ax, 500, 320)
        D = np.array([orc.ndf_cov(G, S, w) for w in dirs])
        for _ in range(3):
            w = _rand_dir(rng)
            signed = float(np.sum(W * (dirs @ w) * D))
            assert signed == pytest.approx(float(np.dot(w, G)), abs=3e-6 * max(1.0, np.linalg.norm(G)))
            hd, hw = ref.sphere_grid(-w, 600, 400, hemisphere=True)
            vis = float(np.sum(hw * (hd @ (-w)) * np.array([orc.ndf_cov(G, S, m) for m in hd])))
            assert vis == pytest.approx(orc.sigma_proj_cov(G, S, w), rel=3e-5)


def test_full_cov_reduces_to_isotropic_and_anisotropic_forms():
    rng = np.random.default_rng(64)
    for _ in range(20):
        G = _rand_dir(rng) * float(rng.choice([0.4, 1.0, 1.5]))
        s, sn = float(rng.choice([0.1, 0.3, 0.8])), float(rng.choice([0.05, 0.3, 1.2]))
        w = _rand_dir(rng)
        iso = (s * s) * np.eye(3)
        assert orc.sigma_proj_cov(G, iso, w) == pytest.approx(orc.sigma_proj(G, s, w), rel=1e-11, abs=1e-300)
        assert orc.ndf_cov(G, iso, w) == pytest.approx(orc.ndf(G, s, w), rel=1e-10, abs=1e-20 * _peak(G, iso))
        an = ref.aniso_cov(G, s, sn)
        assert orc.sigma_proj_cov(G, an, w) == pytest.approx(orc.sigma_proj_n(G, s, sn, w), rel=1e-11, abs=1e-300)
        assert orc.ndf_cov(G, an, w) == pytest.approx(orc.ndf_n(G, s, sn, w), rel=1e-9, abs=1e-20 * _peak(G, an))


def test_full_cov_projected_area_monte_carlo():
    """E[max(0, -d.g)] by sampling g directly."""
    rng = np.random.default_rng(65)
    G = np.array([0.3, -0.2, 0.5])
    S = _rand_spd(rng, 0.4)
    g = rng.multivariate_normal(G, S, size=2_000_000)
    for _ in range(4):
        d = _rand_dir(rng)
        x = np.maximum(0.0, -(g @ d))
        assert orc.sigma_proj_cov(G, S, d) == pytest.approx(x.mean(), abs=4 * x.std() / math.sqrt(x.size))


# ---------------------------------------------------------------------------
# Posterior (Eq. condition_gp)
# ---------------------------------------------------------------------------
def _sphere_with(obs, noise_frac=0.05, variance=0.0025, lengthscale=0.25):
    return sc.sphere_scene(lengthscale=lengthscale, variance=variance, width=16, height=16, spp=1,
                           majorant_res=(16, 16, 16)).replace(
        observations=np.asarray(obs, np.float32), obs_noise=float(noise_frac * variance))


def _sphere_prior(x):
    x = np.asarray(x, float)
    r = np.linalg.norm(x)
    return r - 1.0, x / r


def test_posterior_single_observation_closed_form():
    """One noisy observation y = f(x0) + e, e ~ N(0, s_n^2): the textbook scalar conditioning
    for f(x) and, through the kernel derivatives, for grad f(x); then g given f(x) = 0."""
    x0 = np.array([0.1, 0.2, 1.05], np.float32).astype(float)
    m0 = orc.f32(0.02)
    S = _sphere_with([[*x0, m0]])
    o = orc.OracleScene(S)
    s2 = orc.f32(S.variance)
    sn2 = orc.f32(S.obs_noise)
    l = orc.f32(S.lengthscale)
    A = s2 + sn2
    mu_x0, _ = _sphere_prior(x0)
    rng = np.random.default_rng(66)
    for _ in range(12):
        x = x0 + rng.normal(scale=0.2, size=3)
        mu, gmu = _sphere_prior(x)
        d = x - x0
        k = s2 * math.exp(-float(d @ d) / (2 * l * l))
        p = o.posterior(x)
        mu_c = mu + k * (m0 - mu_x0) / A
        g_c = gmu - k * d / (l * l) * (m0 - mu_x0) / A
        var_c = s2 - k * k / A
        c = k * k * d / (l * l * A)
        Sgg = s2 / (l * l) * np.eye(3) - k * k * np.outer(d, d) / (l ** 4 * A)
        assert p["mu"] == pytest.approx(mu_c, rel=1e-12, abs=1e-15)
        np.testing.assert_allclose(p["grad"], g_c, rtol=1e-12, atol=1e-14)
        assert p["var"] == pytest.approx(var_c, rel=1e-12)
        np.testing.assert_allclose(p["c"], c, rtol=1e-10, atol=1e-17)
        np.testing.assert_allclose(p["Sgg"], Sgg, rtol=1e-12, atol=1e-16)
        np.testing.assert_allclose(p["mg"], g_c - c * mu_c / var_c, rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(p["Sg"], Sgg - np.outer(c, c) / var_c, rtol=1e-10, atol=1e-15)


def _se_joint_cov(points, x, s2, l):
    """Prior covariance of (f(points), f(x), grad f(x)) under the squared-exponential kernel:
    kappa, its first derivative in the second argument and the mixed second derivative."""
    P = np.asarray(points, float)
    n = P.shape[0]
    C = np.zeros((n + 4, n + 4))
    k = lambda a, b: s2 * math.exp(-float((a - b) @ (a - b)) / (2 * l * l))
    for i in range(n):
        for j in range(n):
            C[i, j] = k(P[i], P[j])
        C[i, n] = C[n, i] = k(P[i], x)
        # cov(f(p_i), d f(x)/dx_a) = d/dx_a kappa(p_i, x) = kappa (p_i - x)_a / l^2
        for a in range(3):
            C[i, n + 1 + a] = C[n + 1 + a, i] = k(P[i], x) * (P[i, a] - x[a]) / (l * l)
    C[n, n] = s2
    for a in range(3):
        C[n + 1 + a, n + 1 + a] = s2 / (l * l)
    return C


def test_posterior_importance_sampling_brute_force():
    """Bayes' rule by brute force: sample (f(C), f(x), grad f(x)) from the prior, weight by
    the likelihood of the noisy observations, and compare the weighted moments."""
    obs = np.array([[0.0, 0.0, 1.02, 0.01], [0.2, 0.1, 0.97, -0.02], [-0.15, 0.2, 1.0, 0.0]], np.float32)
    S = _sphere_with(obs, noise_frac=0.4)
    o = orc.OracleScene(S)
    s2, sn2, l = orc.f32(S.variance), orc.f32(S.obs_noise), orc.f32(S.lengthscale)
    P = obs[:, :3].astype(float)
    m = obs[:, 3].astype(float)
    muC = np.array([_sphere_prior(p)[0] for p in P])
    x = np.array([0.05, 0.1, 1.0])
    mu_x, g_x = _sphere_prior(x)
    C = _se_joint_cov(P, x, s2, l)
    rng = np.random.default_rng(67)
    N = 2_000_000
    z = rng.multivariate_normal(np.zeros(7), C, size=N, method="eigh")
    fC = z[:, :3] + muC
    fx = z[:, 3] + mu_x
    gx = z[:, 4:] + g_x
    lw = -0.5 * np.sum((fC - m) ** 2, axis=1) / sn2
    w = np.exp(lw - lw.max())
    w /= w.sum()
    ess = 1.0 / np.sum(w * w)
    assert ess > 1e5
    p = o.posterior(x)
    mean_f = float(w @ fx)
    mean_g = w @ gx
    var_f = float(w @ (fx - mean_f) ** 2)
    cov_gf = (w[:, None] * (gx - mean_g)).T @ (fx - mean_f)
    cov_gg = (w[:, None] * (gx - mean_g)).T @ (gx - mean_g)
    se = 5.0 / math.sqrt(ess)
    assert abs(mean_f - p["mu"]) < se * math.sqrt(s2)
    assert np.all(np.abs(mean_g - p["grad"]) < se * math.sqrt(s2) / l)
    assert abs(var_f - p["var"]) < se * s2 * math.sqrt(2)
    assert np.all(np.abs(cov_gf - p["c"]) < se * s2 / l * math.sqrt(2))
    assert np.all(np.abs(cov_gg - p["Sgg"]) < se * s2 / (l * l) * math.sqrt(2))


@pytest.mark.parametrize("which", ["sphere", "blob"])
def test_posterior_derivative_identities(which):
    """grad mu_C is the derivative of the posterior mean, and c = cov(grad f, f) is half the
    derivative of the posterior variance kappa_C(x, x)."""
    s = sc.cond_sphere_scene(width=16, height=16, spp=1, majorant_res=(16, 16, 16)) if which == "sphere" else \
        sc.cond_blob_scene(width=16, height=16, spp=1, majorant_res=(16, 16, 16))
    o = orc.OracleScene(s)
    rng = np.random.default_rng(68)
    obs = s.observations[:, :3].astype(float)
    h = 1e-5
    for i in range(12):
        x = obs[i % len(obs)] + rng.normal(scale=0.15, size=3)
        p = o.posterior(x)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            pp, pm = o.posterior(x + e), o.posterior(x - e)
            assert (pp["mu"] - pm["mu"]) / (2 * h) == pytest.approx(p["grad"][a], rel=1e-6, abs=1e-8)
            assert (pp["var"] - pm["var"]) / (4 * h) == pytest.approx(p["c"][a], rel=1e-5, abs=1e-11)


def test_posterior_covariance_is_psd_and_below_prior():
    s = sc.cond_sphere_scene(width=16, height=16, spp=1, majorant_res=(16, 16, 16))
    o = orc.OracleScene(s)
    s2, l = orc.f32(s.variance), orc.f32(s.lengthscale)
    prior = np.diag([s2, s2 / l ** 2, s2 / l ** 2, s2 / l ** 2])
    rng = np.random.default_rng(69)
    obs = s.observations[:, :3].astype(float)
    for i in range(30):
        x = obs[i % len(obs)] + rng.normal(scale=0.1, size=3)
        p = o.posterior(x)
        P = np.zeros((4, 4))
        P[0, 0] = p["var"]
        P[0, 1:] = P[1:, 0] = p["c"]
        P[1:, 1:] = p["Sgg"]
        scale = np.sqrt(np.diag(prior))
        ev = np.linalg.eigvalsh(P / np.outer(scale, scale))
        assert ev.min() > 0.0
        assert np.linalg.eigvalsh((prior - P) / np.outer(scale, scale)).min() > -1e-12
        # the gradient given f(x) = 0 is a Schur complement: still positive definite
        assert np.linalg.eigvalsh(p["Sg"]).min() > 0.0


def test_far_observations_leave_the_prior():
    """Observations 40 lengthscales away change nothing: same medium as the unconditioned GP."""
    far = [[12.0, 0.0, 0.0, 0.3], [0.0, -11.0, 0.0, -0.2]]
    S = _sphere_with(far)
    o, u = orc.OracleScene(S), orc.OracleScene(S.replace(observations=None, obs_noise=0.0))
    rng = np.random.default_rng(70)
    for _ in range(20):
        x = rng.uniform(-1.2, 1.2, 3)
        d, wi = _rand_dir(rng), _rand_dir(rng)
        assert o.sigma_t(x, d) == pytest.approx(u.sigma_t(x, d), rel=1e-12, abs=1e-300)
        assert o.phase_eval_at(x, d, wi) == pytest.approx(u.phase_eval_at(x, d, wi), rel=1e-10, abs=1e-300)


def test_posterior_mean_is_linear_in_the_observed_values():
    base = sc.cond_sphere_scene(n_obs=8, width=16, height=16, spp=1, majorant_res=(16, 16, 16))
    rng = np.random.default_rng(71)
    m1, m2 = rng.normal(scale=0.03, size=8), rng.normal(scale=0.03, size=8)

    def with_values(m):
        obs = base.observations.copy()
        obs[:, 3] = m
        return orc.OracleScene(base.replace(observations=obs))
    o0, o1, o2, o12 = (with_values(v) for v in (np.zeros(8), m1, m2, m1 + m2))
    for _ in range(10):
        x = base.observations[rng.integers(8), :3] + rng.normal(scale=0.2, size=3)
        a, b, c, d = (o.posterior(x)["mu"] for o in (o0, o1, o2, o12))
        assert d - a == pytest.approx((b - a) + (c - a), rel=1e-5, abs=1e-9)
        assert o12.posterior(x)["var"] == o0.posterior(x)["var"]


# ---------------------------------------------------------------------------
# Majorant and scene rules
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["sphere", "blob"])
def test_conditioned_majorant_bounds_sigma_t(which):
    s = sc.cond_sphere_scene(width=16, height=16, spp=1, majorant_res=(24, 24, 24)) if which == "sphere" else \
        sc.cond_blob_scene(width=16, height=16, spp=1, majorant_res=(24, 24, 24))
    o = orc.OracleScene(s)
    maj = o.majorants().reshape(24, 24, 24)
    lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
    rng = np.random.default_rng(72)
    obs = s.observations[:, :3].astype(float)
    pts = np.concatenate([lo + rng.random((3000, 3)) * (hi - lo),
                          obs[rng.integers(len(obs), size=3000)] + rng.normal(scale=0.05, size=(3000, 3))])
    pts = np.clip(pts, lo + 1e-9, hi - 1e-9)
    worst = 0.0
    for x in pts:
        cell = np.minimum(((x - lo) / (hi - lo) * 24).astype(int), 23)
        m = maj[cell[2], cell[1], cell[0]]
        st = o.sigma_t(x, _rand_dir(rng))
        if m == 0.0:   # bounds below 2^-40 skip the cell
            assert st < 2.0 ** -40
        else:
            worst = max(worst, st / m)
    assert worst <= 1.0
    # and the majorant is not vacuous near the observed surface
    assert worst > 0.02


def _cell_points(lo, cw, k, n=4):
    t = np.linspace(0.0, 1.0, n)
    return [lo + (k + np.array([u, v, w])) * cw for u in t for v in t for w in t]


@pytest.mark.parametrize("which", ["sphere", "blob"])
def test_conditioned_majorant_dense_cells(which):
    """Every sampled point of a cell (a 4^3 lattice with the corners) and every direction
    (64 spread directions and the steepest one, minus the mean gradient given f = 0) stays
    under the cell's majorant: near the surface, near observations and outside."""
    s = sc.cond_sphere_scene(width=16, height=16, spp=1, majorant_res=(32, 32, 32)) if which == "sphere" else \
        sc.cond_blob_scene(width=16, height=16, spp=1, majorant_res=(32, 32, 32))
    o = orc.OracleScene(s)
    M = 32
    maj = o.majorants().reshape(M, M, M)
    lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
    cw = (hi - lo) / M
    rng = np.random.default_rng(73)
    obs = s.observations[:, :3].astype(float)
    near_obs = np.minimum(((obs - lo) / cw).astype(int), M - 1)[:, ::-1]
    nz = np.argwhere(maj > 0)
    cells = np.concatenate([nz[rng.choice(len(nz), 40, replace=False)], near_obs[:10],
                            np.argwhere(maj >= 0)[rng.choice(M ** 3, 10, replace=False)]])
    dirs = sc.fibonacci_directions(64)
    for kz, ky, kx in cells:
        k = np.array([kx, ky, kz])
        m = maj[kz, ky, kx]
        for x in _cell_points(lo, cw, k):
            x = np.clip(x, lo, hi)
            mg = o.posterior(x)["mg"]
            cand = list(dirs) + ([-mg / np.linalg.norm(mg)] if np.linalg.norm(mg) > 0 else [])
            st = max(o.sigma_t(x, d) for d in cand)
            if m == 0.0:
                assert st < 2.0 ** -40
            else:
                assert st <= m, (which, (kx, ky, kz), x, st, m)


def test_conditioned_majorant_is_tight():
    """The conditioned majorant stays within a small factor of the largest extinction
    sampled in its cell: median below 1.8 over cells around the observed sphere at the
    128^3 grid the conditioned scenes use (the triangle-inequality slope bound with
    sigma_proj <= |m| + sd / sqrt(2 pi) gave 2.25)."""
    s = sc.cond_sphere_scene(width=16, height=16, spp=1)
    o = orc.OracleScene(s)
    M = s.majorant_res[0]
    maj = o.majorants().reshape(M, M, M)
    lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
    cw = (hi - lo) / M
    idx = np.argwhere(maj > 0)
    cen = lo + (idx[:, ::-1] + 0.5) * cw
    shell = idx[np.abs(np.linalg.norm(cen, axis=1) - 1.0) < 0.06]
    rng = np.random.default_rng(74)
    dirs = sc.fibonacci_directions(32)
    ratios = []
    for kz, ky, kx in shell[rng.choice(len(shell), 30, replace=False)]:
        pts = _cell_points(lo, cw, np.array([kx, ky, kz]))
        best = 0.0
        for x in pts:
            mg = o.posterior(x)["mg"]
            cand = list(dirs) + ([-mg / np.linalg.norm(mg)] if np.linalg.norm(mg) > 0 else [])
            best = max(best, max(o.sigma_t(x, d) for d in cand))
        ratios.append(maj[kz, ky, kx] / best)
    assert min(ratios) >= 1.0
    assert np.median(ratios) < 1.8


def test_majorant_constants_z_times_mills_ratio():
    """z r(z), r = phi / Phi, over z >= 0: its maximum is below 0.2946 (near z = 0.84) and it
    decreases from z = 0.9 on (brute force on the oracle's erfcx)."""
    z = np.linspace(0.0, 12.0, 24001)
    v = np.array([zz * math.sqrt(2.0 / math.pi) / orc.erfcx(-zz / math.sqrt(2.0)) for zz in z])
    assert v.max() < 0.2946
    assert 0.80 < z[v.argmax()] < 0.88
    tail = v[z >= 0.9]
    assert np.all(np.diff(tail) <= 0.0)


def test_se_kernel_hessian_bound():
    """Spectral norm of the Hessian of kappa(x - x_j) = s^2 e^{-|x - x_j|^2 / (2 l^2)} over a box
    is at most (s^2/l^2) e^{-dmin^2/(2l^2)} max(1, dmax^2/l^2 - 1) (dmin, dmax: nearest and
    farthest distances from x_j to the box), checked on central-difference Hessians."""
    rng = np.random.default_rng(75)
    s2, l = 0.0025, 0.25
    kap = lambda x, xj: s2 * math.exp(-np.sum((x - xj) ** 2) / (2 * l * l))
    h = 1e-4
    for _ in range(200):
        lo = rng.uniform(-1, 1, 3)
        w = rng.uniform(0.01, 0.3, 3)
        hi = lo + w
        xj = rng.uniform(-1.2, 1.2, 3)
        dn = np.where(xj < lo, lo - xj, np.where(xj > hi, xj - hi, 0.0))
        df = np.maximum(np.abs(xj - lo), np.abs(xj - hi))
        bound = (s2 / l / l) * math.exp(-np.sum(dn ** 2) / (2 * l * l)) * max(1.0, np.sum(df ** 2) / (l * l) - 1.0)
        for _ in range(5):
            x = lo + rng.random(3) * w
            H = np.zeros((3, 3))
            for a in range(3):
                for b in range(3):
                    ea, eb = np.eye(3)[a] * h, np.eye(3)[b] * h
                    H[a, b] = (kap(x + ea + eb, xj) - kap(x + ea - eb, xj) - kap(x - ea + eb, xj)
                               + kap(x - ea - eb, xj)) / (4 * h * h)
            assert np.linalg.norm(H, 2) <= bound * (1 + 1e-4) + 1e-12


def test_conditioned_scene_rules():
    s = sc.cond_sphere_scene(n_obs=4, width=16, height=16, spp=1, majorant_res=(16, 16, 16))
    orc.OracleScene(s)
    for bad in (dict(obs_noise=0.0), dict(lengthscale_n=0.05), dict(ndf_kind=sc.NDF_GGX),
                dict(variance_grid=np.full((2, 2, 2), 0.0025, np.float32))):
        with pytest.raises(ValueError):
            orc.OracleScene(s.replace(**bad))
