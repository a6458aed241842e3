"""Independent reference mathematics for the oracle pins.

Everything here is written from definitions (Gaussian integrals, expectations,
quadrature) with SciPy/NumPy primitives; none of it reuses the oracle's formulas.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special, stats


def gauss_pdf3(g, mean, cov_diag):
    """Density of N(mean, diag(cov_diag)) at points g (n, 3)."""
    g = np.atleast_2d(g)
    z = (g - mean) ** 2 / cov_diag
    return np.exp(-0.5 * z.sum(-1)) / np.sqrt((2 * np.pi) ** 3 * np.prod(cov_diag))


def ndf_by_gdf(wm, mean, cov_diag):
    """Sec. 4.2.2 Eq. gdf_to_ndf: D(wm) = int_0^inf P(t wm) t^3 dt (1D quadrature)."""
    wm = np.asarray(wm, float)
    f = lambda t: gauss_pdf3(t * wm, mean, cov_diag)[0] * t ** 3
    val, _ = integrate.quad(f, 0.0, np.inf, epsabs=0.0, epsrel=1e-12, limit=400)
    return val


def projected_area_by_expectation(d, mean, cov_diag):
    """E[max(0, -d.g)] for g ~ N(mean, diag(cov)): -d.g is a 1D Gaussian."""
    d = np.asarray(d, float)
    m = -float(np.dot(d, mean))
    sd = math.sqrt(float(np.dot(d * d, cov_diag)))
    f = lambda x: x * stats.norm.pdf(x, m, sd)
    lo = 0.0
    hi = max(m, 0.0) + 40 * sd
    val, _ = integrate.quad(f, lo, hi, epsabs=0.0, epsrel=1e-12, limit=400, points=[max(m, 0.0)])
    return val


def rho_reference(mu, sigma):
    """phi(mu;0,s^2)/Phi(mu;0,s^2) via SciPy's log density and log CDF."""
    return math.exp(stats.norm.logpdf(mu, 0.0, sigma) - special.log_ndtr(mu / sigma))


def frame(axis):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    h = np.array([1.0, 0, 0]) if abs(axis[0]) < 0.9 else np.array([0, 1.0, 0])
    t = np.cross(axis, h)
    t /= np.linalg.norm(t)
    b = np.cross(axis, t)
    return t, b, axis


def sphere_grid(axis, n_theta=200, n_phi=256, hemisphere=False):
    """Gauss-Legendre in cos(theta) about `axis` x uniform phi; returns dirs (n,3), weights."""
    t, b, a = frame(axis)
    x, w = np.polynomial.legendre.leggauss(n_theta)
    if hemisphere:
        c = 0.5 * (x + 1.0)
        wc = 0.5 * w
    else:
        c, wc = x, w
    ph = (np.arange(n_phi) + 0.5) * 2 * np.pi / n_phi
    wp = 2 * np.pi / n_phi
    C, P = np.meshgrid(c, ph, indexing="ij")
    S = np.sqrt(np.maximum(0.0, 1 - C * C))
    dirs = (S * np.cos(P))[..., None] * t + (S * np.sin(P))[..., None] * b + C[..., None] * a
    W = (wc[:, None] * wp) * np.ones_like(P)
    return dirs.reshape(-1, 3), W.reshape(-1)


def beckmann_D(alpha, cos_m):
    """Textbook Beckmann NDF."""
    c2 = cos_m * cos_m
    tan2 = (1 - c2) / c2
    return math.exp(-tan2 / alpha ** 2) / (math.pi * alpha ** 2 * c2 * c2)


def beckmann_lambda(a):
    """Textbook Smith Lambda of the Beckmann distribution."""
    return 0.5 * (math.exp(-a * a) / (a * math.sqrt(math.pi)) - special.erfc(a))


def planar_transmittance(z0, z1, dz, sigma, proj):
    """Closed form of exp(-int sigma_t) along a ray crossing heights z0 -> z1 through the planar
    medium with density rho(z) = d/dz ln Phi(z/sigma): (Phi(z0/s)/Phi(z1/s))^(proj/dz)."""
    return math.exp(proj / dz * (special.log_ndtr(z0 / sigma) - special.log_ndtr(z1 / sigma)))


def aniso_cov(G, s, sn):
    """Sigma = s^2 (I - n n^T) + sn^2 n n^T about n = G/|G| (z when G = 0), as a 3x3 matrix."""
    G = np.asarray(G, float)
    g = np.linalg.norm(G)
    n = G / g if g > 0 else np.array([0.0, 0.0, 1.0])
    return s * s * (np.eye(3) - np.outer(n, n)) + sn * sn * np.outer(n, n)


def ndf_by_gdf_full(wm, mean, cov):
    """Eq. gdf_to_ndf for g ~ N(mean, cov) with a full covariance matrix (1D quadrature)."""
    wm = np.asarray(wm, float)
    mean = np.asarray(mean, float)
    inv = np.linalg.inv(cov)
    norm = 1.0 / math.sqrt((2 * np.pi) ** 3 * np.linalg.det(cov))

    def f(t):
        r = t * wm - mean
        return norm * math.exp(-0.5 * float(r @ inv @ r)) * t ** 3

    val, _ = integrate.quad(f, 0.0, np.inf, epsabs=0.0, epsrel=1e-12, limit=400)
    return val


def projected_area_full(d, mean, cov):
    """E[max(0, -d.g)] for g ~ N(mean, cov): -d.g ~ N(-d.mean, d^T cov d)."""
    d = np.asarray(d, float)
    m = -float(np.dot(d, mean))
    sd = math.sqrt(float(d @ cov @ d))
    f = lambda x: x * stats.norm.pdf(x, m, sd)
    hi = max(m, 0.0) + 40 * sd
    val, _ = integrate.quad(f, 0.0, hi, epsabs=0.0, epsrel=1e-12, limit=400, points=[max(m, 0.0)])
    return val


def ggx_D(alpha, cos_m):
    """Textbook GGX (Trowbridge-Reitz) NDF, zero below the horizon."""
    if cos_m <= 0.0:
        return 0.0
    c2 = cos_m * cos_m
    t2 = (1.0 - c2) / c2
    return alpha * alpha / (math.pi * c2 * c2 * (alpha * alpha + t2) ** 2)


def ggx_lambda(alpha, cos_t):
    """Textbook GGX Smith Lambda for a direction above the horizon."""
    t2 = (1.0 - cos_t * cos_t) / (cos_t * cos_t)
    return 0.5 * (-1.0 + math.sqrt(1.0 + alpha * alpha * t2))


def fresnel_conductor_snell(c, eta, k):
    """Unpolarized Fresnel reflectance for IOR n = eta + i k from Snell's law with complex
    angles: cos_t = sqrt(1 - sin^2 / n^2), r_s = (c - n cos_t)/(c + n cos_t),
    r_p = (n c - cos_t)/(n c + cos_t)."""
    n = complex(eta, k)
    sin2 = 1.0 - c * c
    cos_t = np.sqrt(1.0 - sin2 / (n * n) + 0j)
    rs = (c - n * cos_t) / (c + n * cos_t)
    rp = (n * c - cos_t) / (n * c + cos_t)
    return 0.5 * (abs(rs) ** 2 + abs(rp) ** 2)
