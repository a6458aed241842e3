"""A 16x16 single-scatter image of the planar GPSS from explicit realizations of the Gaussian
process, against the oracle's depth-1 image of the same scene (the GPIS that the macrofacet
medium stands for without realizations: Sec. 3.1, Sec. 4.1, Sec. 4.2.1 and Fig. tr).

Scene: mean m(x) = z, so f = z + xi with xi a zero-mean GP of variance sigma^2 and a
squared-exponential kernel of lengthscale l (roughness alpha = sqrt(2) sigma / l, Eq. roughness),
seen from a pinhole camera at 60 deg from the normal (pixels span about 45..75 deg), lit by a
constant environment of radiance 1; albedo 1 (mirror microflakes without Fresnel), one
scattering event.  Two kernels: the isotropic one, and the fully anisotropic one with infinite
correlation along z (a height field, the Beckmann limit of Sec. 4.1), which the oracle takes as
lengthscale_n = 1e4 l.

Realizations: random Fourier features (Rahimi and Recht), xi(x) = sigma sqrt(2/M) sum_i
cos(w_i . x + b_i) with w_i ~ N(0, I / l^2) (w_z = 0 for the height field) and b_i uniform,
drawn afresh for every camera sample.  A sample marches its camera ray from z = 4 sigma to the
first point with f <= 0 (bisection inside the step), reflects the ray about the realization's
normal grad f / |grad f| there, and marches the reflected ray: it scores 1 if the ray reaches
z = 4 sigma without meeting f <= 0 again, else 0 (a second scattering event).  The oracle's
depth-1 image has the same expectation where the medium's independence assumption holds.

Where the paper says the model agrees with realizations (the height field, Sec. 4.1; short
optical depth, Fig. tr), at roughness 0.3 both images agree within Monte Carlo confidence
intervals.  At roughness 1 the realizations escape more often than the medium predicts: the
medium draws the reflected ray's next crossing as if the surface near the scattering point were
unknown (the decorrelation of Sec. 4.2.1; the paper's Fig. impact_independent), while a real
surface lies below a ray that leaves it.  That gap is the model's, and is only bounded here.
"""
import math

import numpy as np
import pytest

from gpss_inputs import scenes as sc
from oracle import oracle as orc

from tests import refmath

SIGMA = 1.0
W = H = 16
CAM_ZENITH = 60.0
EYE = 20.0 * np.array([math.sin(math.radians(CAM_ZENITH)), 0.0, math.cos(math.radians(CAM_ZENITH))])
FOV = 30.0
Z_TOP = 4.0 * SIGMA         # start of the camera march, end of the reflected one (P(f < 0) ~ 3e-5)
ORACLE_SPP = 4096
REAL_SPP = 160              # realization samples per pixel
N_FEATURES = 96
STEPS_PER_L = 10            # march steps per lengthscale (converged: 20 and 40 agree)


def _lengthscale(alpha):
    return math.sqrt(2.0) * SIGMA / alpha


def _scene(alpha, height_field):
    ell = _lengthscale(alpha)
    s = sc.plane_scene(width=W, height=H, spp=ORACLE_SPP, max_depth=1, variance=SIGMA ** 2, lengthscale=ell,
                       albedo=1.0, env=1.0, light_E=0.0, half_thickness=7.0 * SIGMA, majorant_res=(1, 1, 256))
    s = s.replace(bounds=np.array([-1e3, -1e3, -7.0 * SIGMA, 1e3, 1e3, 7.0 * SIGMA], np.float32),
                  cam_kind=sc.CAM_PINHOLE, cam_eye=tuple(EYE), cam_target=(0.0, 0.0, 0.0),
                  cam_up=(0.0, 0.0, 1.0), cam_fov_deg=FOV)
    return s.replace(lengthscale_n=1e4 * ell) if height_field else s


def _march(o, d, t, xi_phase0, xi_phase1, amp, h, stop_up):
    """March rays o + t d (t advanced in steps h) until f = z + xi <= 0 (returns the bisected
    distance there, NaN if none) or, with stop_up, until the ray rises above Z_TOP (flag).
    xi at distance t is amp * sum cos(phase0 + t phase1) over the features."""
    n = o.shape[0]
    hit_t = np.full(n, np.nan, np.float32)
    up = np.zeros(n, bool)
    live = np.arange(n)
    p0, p1 = xi_phase0, xi_phase1

    def f(idx, rows, tt):
        return o[idx, 2] + tt * d[idx, 2] + amp * np.cos(p0[rows] + tt[:, None] * p1[rows]).sum(1)

    while live.size:
        t[live] += h
        tl = t[live]
        rows = np.arange(live.size)
        neg = f(live, rows, tl) <= 0.0
        if neg.any():
            r = np.nonzero(neg)[0]
            lo, hi = tl[r] - h, tl[r].copy()
            for _ in range(24):
                mid = 0.5 * (lo + hi)
                below = f(live[r], r, mid) <= 0.0
                hi = np.where(below, mid, hi)
                lo = np.where(below, lo, mid)
            hit_t[live[r]] = hi
        z = o[live, 2] + tl * d[live, 2]
        out = (~neg) & (z > Z_TOP) if stop_up else np.zeros_like(neg)
        up[live[out]] = True
        keep = (~neg) & (~out) & (z > -8.0 * SIGMA) & (tl < 60.0 * SIGMA)
        live, p0, p1 = live[keep], p0[keep], p1[keep]
    return hit_t, up


def realization_image(alpha, height_field, spp=REAL_SPP, seed=0, chunk=8192):
    """Per-pixel escape fraction of single-scattered camera rays over fresh realizations."""
    ell = _lengthscale(alpha)
    h = np.float32(ell / STEPS_PER_L)
    amp = np.float32(SIGMA * math.sqrt(2.0 / N_FEATURES))
    rng = np.random.default_rng(seed)
    hits = np.zeros(W * H)
    count = np.zeros(W * H)
    order = np.repeat(np.arange(W * H), spp)
    rng.shuffle(order)
    for c0 in range(0, order.size, chunk):
        p = order[c0:c0 + chunk]
        n = p.size
        xs, ys = (p % W) + rng.random(n), (p // W) + rng.random(n)
        d = np.stack([refmath.pinhole_direction(EYE, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), FOV, W, H, a, b)
                      for a, b in zip(xs, ys)]).astype(np.float32)
        w = (rng.standard_normal((3, n, N_FEATURES)) / ell).astype(np.float32)
        if height_field:
            w[2] = 0.0
        b = (rng.random((n, N_FEATURES)) * 2.0 * math.pi).astype(np.float32)
        o = (EYE[None, :] + ((EYE[2] - Z_TOP) / -d[:, 2].astype(float))[:, None] * d).astype(np.float32)

        def phases(x, v):
            return (w[0] * x[:, :1] + w[1] * x[:, 1:2] + w[2] * x[:, 2:3] + b,
                    w[0] * v[:, :1] + w[1] * v[:, 1:2] + w[2] * v[:, 2:3])

        tc, _ = _march(o, d, np.zeros(n, np.float32), *phases(o, d), amp, h, stop_up=False)
        assert not np.isnan(tc).any(), "a camera ray passed the layer without meeting the surface"
        xc = o + tc[:, None] * d
        s = np.sin(phases(xc, d)[0])
        grad = np.stack([-amp * (s * w[0]).sum(1), -amp * (s * w[1]).sum(1), 1.0 - amp * (s * w[2]).sum(1)], 1)
        nrm = grad / np.linalg.norm(grad, axis=1, keepdims=True)
        wo = (d - 2.0 * np.sum(d * nrm, 1, keepdims=True) * nrm).astype(np.float32)
        _, up = _march(xc, wo, np.full(n, 1e-3 * h, np.float32), *phases(xc, wo), amp, h, stop_up=True)
        np.add.at(hits, p, up.astype(float))
        np.add.at(count, p, 1.0)
    return (hits / count).reshape(H, W), count.reshape(H, W)


def _compare(alpha, height_field, seed):
    o = orc.OracleScene(_scene(alpha, height_field)).render()
    m, var_o = o["mean"], o["var"] / ORACLE_SPP
    r, n = realization_image(alpha, height_field, seed=seed)
    # binomial variance under the oracle's value, plus the oracle's own estimate's
    var = np.clip(m * (1.0 - m), 1e-6, None) / n + var_o
    z = (r - m) / np.sqrt(var)
    se_mean = math.sqrt(var.sum()) / var.size
    return m, r, z, se_mean


@pytest.mark.parametrize("height_field", [True, False], ids=["height_field", "isotropic"])
def test_realization_image_agrees_at_low_roughness(height_field):
    m, r, z, se = _compare(0.3, height_field, seed=11 if height_field else 12)
    # the image has contrast (escape from 0.86 at grazing pixels to 0.99)
    assert m.max() - m.min() > 0.08
    gap = float(r.mean() - m.mean())
    assert abs(gap) < 4.0 * se, (gap, se)
    assert float(np.mean(z ** 2)) < 1.5, np.mean(z ** 2)
    assert float(np.abs(z).max()) < 5.0, np.abs(z).max()


def test_realization_image_gap_at_high_roughness_is_the_decorrelation_bias():
    """Isotropic kernel at roughness 1: the realizations' escape fraction exceeds the medium's
    (measured: +0.033 on a mean of 0.69, about 14 standard errors), and stays within the few
    percent of the paper's Fig. impact_independent."""
    m, r, z, se = _compare(1.0, False, seed=13)
    gap = float(r.mean() - m.mean())
    assert gap > 4.0 * se, (gap, se)
    assert gap < 0.06, gap
