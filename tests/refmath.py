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


# ---------------------------------------------------------------------------
# Scene geometry written from definitions (camera, box, signed distances, grids).
# ---------------------------------------------------------------------------
def pinhole_direction(eye, target, up, vfov_deg, width, height, x_img, y_img):
    """Unit direction of the pinhole ray through image position (x_img, y_img) in pixel units
    (x to the right, y downward from the top-left corner).  The vertical field of view spans
    the image height; the horizontal extent follows from the aspect ratio width / height.
    The image plane sits at unit distance along the viewing direction."""
    eye, target, up = (np.asarray(v, float) for v in (eye, target, up))
    w = target - eye
    w /= np.linalg.norm(w)
    r = np.cross(w, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, w)
    half_h = math.tan(math.radians(vfov_deg) / 2.0)
    half_w = half_h * width / height
    # image-plane coordinates in [-half_w, half_w] x [-half_h, half_h], top row at +half_h
    px = (x_img / width * 2.0 - 1.0) * half_w
    py = (1.0 - y_img / height * 2.0) * half_h
    d = w + px * r + py * u
    return d / np.linalg.norm(d)


def box_chord(o, d, lo, hi, n_scan=4096, tmax=20.0):
    """Entry and exit distances of the ray o + t d through the box [lo, hi], found from the
    inside indicator: a fine scan for the transitions, then bisection to ~1e-13.  Returns
    None when the ray misses."""
    o, d, lo, hi = (np.asarray(v, float) for v in (o, d, lo, hi))
    inside = lambda t: bool(np.all(o + t * d >= lo) and np.all(o + t * d <= hi))
    ts = np.linspace(0.0, tmax, n_scan)
    pts = o[None, :] + ts[:, None] * d[None, :]
    ins = np.all((pts >= lo) & (pts <= hi), axis=1)
    if not ins.any():
        return None
    k0, k1 = int(np.argmax(ins)), len(ins) - 1 - int(np.argmax(ins[::-1]))

    def bisect(a, b, want_inside_at_b):
        for _ in range(80):
            m = 0.5 * (a + b)
            if inside(m) == want_inside_at_b:
                b = m
            else:
                a = m
        return 0.5 * (a + b)

    t0 = 0.0 if k0 == 0 else bisect(ts[k0 - 1], ts[k0], True)
    t1 = bisect(ts[k1 + 1], ts[k1], True) if k1 + 1 < len(ts) else tmax
    return t0, t1


def box_exit_distance(x, w, lo, hi):
    """Distance from a point x inside the box [lo, hi] to the box boundary along unit w:
    the smallest positive distance to the three planes the ray heads for."""
    x, w, lo, hi = (np.asarray(v, float) for v in (x, w, lo, hi))
    best = np.inf
    for a in range(3):
        if w[a] > 0:
            best = min(best, (hi[a] - x[a]) / w[a])
        elif w[a] < 0:
            best = min(best, (lo[a] - x[a]) / w[a])
    return best


def sdf_sphere_ref(x, c, r):
    v = np.asarray(x, float) - np.asarray(c, float)
    n = np.linalg.norm(v)
    return n - r, v / n


def sdf_box_ref(x, c, h):
    """Exact signed distance of an axis-aligned box (centre c, half extents h) by closest
    points: outside, the distance to the clamped point and the unit vector from it; inside,
    minus the distance to the nearest face and that face's outward normal.  Also returns the
    set of outward normals of all nearest faces (ties) for interior points."""
    x, c, h = (np.asarray(v, float) for v in (x, c, h))
    lo, hi = c - h, c + h
    p = np.minimum(np.maximum(x, lo), hi)
    if np.any(p != x):
        v = x - p
        n = np.linalg.norm(v)
        return n, v / n, [v / n]
    dist = np.concatenate([x - lo, hi - x])      # distances to the six faces
    m = dist.min()
    normals = []
    for k in np.flatnonzero(dist == m):
        nrm = np.zeros(3)
        nrm[k % 3] = -1.0 if k < 3 else 1.0
        normals.append(nrm)
    return -m, normals[0], normals


def union_sdf_ref(prims, x):
    """min over primitive rows [kind, cx, cy, cz, a, b, c, albedo] of their exact signed
    distances: value, gradient of the minimizing primitive, its index (lowest on ties), the
    valid gradients (ties inside boxes) and its albedo."""
    best = None
    for i, p in enumerate(np.asarray(prims, float)):
        if p[0] == 0:
            f, g = sdf_sphere_ref(x, p[1:4], p[4])
            gs = [g]
        else:
            f, g, gs = sdf_box_ref(x, p[1:4], p[4:7])
        if best is None or f < best[0]:
            best = (f, g, i, gs, p[7])
    return best


def trilinear_ref(grid_zyx, lo, hi, x):
    """Value and gradient of the trilinear interpolant of a node-centred grid (shape
    (nz, ny, nx), node k at lo + k / (n - 1) (hi - lo) per axis) at x, from SciPy's
    RegularGridInterpolator; the gradient along an axis is the difference of the
    interpolant on the two node planes bounding x, over their spacing (the interpolant is
    linear along each axis inside a cell)."""
    from scipy.interpolate import RegularGridInterpolator
    nz, ny, nx = grid_zyx.shape
    axes = [np.linspace(lo[2], hi[2], nz), np.linspace(lo[1], hi[1], ny), np.linspace(lo[0], hi[0], nx)]
    f = RegularGridInterpolator(axes, np.asarray(grid_zyx, float), method="linear")
    xz = np.array([x[2], x[1], x[0]], float)
    val = float(f(xz[None, :])[0])
    grad = np.zeros(3)
    for a_zyx, a_xyz in ((0, 2), (1, 1), (2, 0)):
        ax = axes[a_zyx]
        k = min(max(int(np.searchsorted(ax, xz[a_zyx], side="right")) - 1, 0), len(ax) - 2)
        p0, p1 = xz.copy(), xz.copy()
        p0[a_zyx], p1[a_zyx] = ax[k], ax[k + 1]
        grad[a_xyz] = (float(f(p1[None, :])[0]) - float(f(p0[None, :])[0])) / (ax[k + 1] - ax[k])
    return val, grad
