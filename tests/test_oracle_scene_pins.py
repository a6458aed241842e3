"""Pins of the oracle's scene-level parts that every curved-mean image depends on: the
pinhole camera, next-event estimation to a point light, the union of box and sphere signed
distances with per-primitive albedo, and trilinear interpolation of the offset and variance
grids.  Each is checked against an independent computation from definitions
(tests/refmath.py), never against the oracle's own formulas.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from gpss_inputs import scenes as sc
from oracle import oracle as orc
from tests import refmath as ref


def _f32(a):
    return np.asarray(a, np.float32)


# ---------------------------------------------------------------------------
# Pinhole camera and point light (Sec. 5 rendering of the classic medium): a homogeneous
# isotropic medium seen at depth 1.
# ---------------------------------------------------------------------------
def _homogeneous_point_scene(spp):
    return sc.Scene(
        name="homog_point", mean_kind=sc.MEAN_CONST, mean_const=0.05,
        prims=np.zeros((0, 8), np.float32), bounds=_f32([-0.5, -0.4, -0.3, 0.5, 0.4, 0.3]),
        variance=0.01, lengthscale=0.2, albedo=0.9, majorant_res=(4, 4, 4),
        point_light=_f32([1.2, 1.5, 0.8, 10.0]), env_radiance=0.0,
        cam_kind=sc.CAM_PINHOLE, cam_eye=(0.3, 0.4, 3.0), cam_target=(0.0, 0.0, 0.0),
        cam_up=(0.0, 1.0, 0.0), cam_fov_deg=30.0,
        width=48, height=32, spp=spp, max_depth=1, seed=17)


def _single_scatter_along(o, d, lo, hi, sig_t, albedo, light, I):
    """Expected depth-1 radiance of a ray through a homogeneous medium of extinction sig_t with
    the isotropic phase albedo / (4 pi), lit by a point light of intensity I outside the box:
    int sig_t e^{-sig_t (t - t_in)} albedo / (4 pi) e^{-sig_t l(x)} I / r(x)^2 dt over the
    chord, l(x) the shadow ray's length inside the box and r(x) the distance to the light."""
    ch = ref.box_chord(o, d, lo, hi)
    if ch is None:
        return 0.0
    t0, t1 = ch

    def f(t):
        x = o + t * d
        v = light - x
        r = np.linalg.norm(v)
        w = v / r
        ell = min(ref.box_exit_distance(x, w, lo, hi), r)
        return (sig_t * math.exp(-sig_t * (t - t0)) * albedo / (4 * math.pi)
                * math.exp(-sig_t * ell) * I / (r * r))

    val, _ = integrate.quad(f, t0, t1, epsabs=0.0, epsrel=1e-9, limit=400)
    return val


def test_pinhole_camera_and_point_light_single_scattering():
    """Each pixel's depth-1 value against a quadrature of the single-scattering integral over
    the pixel footprint (Gauss-Legendre in the jitter) and along each ray, with the rays built
    from the vertical-field-of-view definition and the light's inverse-square falloff.  The
    image is 48 x 32, so a horizontal field of view, a flipped row order or a 1/r falloff would
    each move the values by far more than the Monte Carlo error."""
    spp = 16000
    s = _homogeneous_point_scene(spp)
    o_s = orc.OracleScene(s)
    lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
    sigma = math.sqrt(orc.f32(s.variance))
    s0 = sigma / orc.f32(s.lengthscale)
    sig_t = ref.rho_reference(orc.f32(s.mean_const), sigma) * s0 / math.sqrt(2 * math.pi)
    albedo = orc.f32(s.albedo)
    light = s.point_light[:3].astype(float)
    I = float(s.point_light[3])
    eye = np.array([orc.f32(v) for v in s.cam_eye])
    # footprints inside the box's image, each entering and leaving through one pair of faces
    pixels = [(13, 9), (20, 12), (30, 10), (14, 20), (25, 18), (32, 15), (18, 23), (28, 24)]
    flat = np.array([j * s.width + i for i, j in pixels], np.int64)
    r = o_s.render_pixels(flat)
    xg, wg = np.polynomial.legendre.leggauss(6)
    ug, wu = 0.5 * (xg + 1.0), 0.5 * wg
    zs = []
    for k, (i, j) in enumerate(pixels):
        want = 0.0
        for a in range(6):
            for b in range(6):
                d = ref.pinhole_direction(eye, [orc.f32(v) for v in s.cam_target],
                                          [orc.f32(v) for v in s.cam_up], orc.f32(s.cam_fov_deg),
                                          s.width, s.height, i + ug[a], j + ug[b])
                want += wu[a] * wu[b] * _single_scatter_along(eye, d, lo, hi, sig_t, albedo, light, I)
        se = math.sqrt(r["var"][k] / spp)
        assert want > 0.0
        z = (r["mean"][k] - want) / se
        zs.append(z)
        assert abs(z) < 5.0, (pixels[k], r["mean"][k], want, se)
        assert r["mean"][k] == pytest.approx(want, rel=0.03)
    # the deviations behave like unit normals
    assert float(np.sum(np.square(zs))) < 26.1   # chi^2_8 upper 0.1 % quantile


def test_pinhole_misses_and_corners():
    """Pixels of the top and bottom rows whose whole footprint misses the box see only the
    (zero) environment."""
    s = _homogeneous_point_scene(64)
    o_s = orc.OracleScene(s)
    lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
    eye = np.array([orc.f32(v) for v in s.cam_eye])
    args = ([orc.f32(v) for v in s.cam_target], [orc.f32(v) for v in s.cam_up], orc.f32(s.cam_fov_deg),
            s.width, s.height)
    miss = []
    for j in (0, s.height - 1):
        for i in range(s.width):
            hit = any(ref.box_chord(eye, ref.pinhole_direction(eye, *args, i + du, j + dv), lo, hi) is not None
                      for du in (0.0, 1.0) for dv in (0.0, 1.0))
            if not hit:
                miss.append(j * s.width + i)
    assert len(miss) > 10
    r = o_s.render_pixels(np.array(miss, np.int64))
    assert np.all(r["mean"] == 0.0)
    # the reference rays through the middles of the top and bottom edges span the vertical
    # field of view
    mid_top = ref.pinhole_direction(eye, *args, s.width / 2.0, 0.0)
    mid_bot = ref.pinhole_direction(eye, *args, s.width / 2.0, float(s.height))
    assert math.degrees(math.acos(np.dot(mid_top, mid_bot))) == pytest.approx(orc.f32(s.cam_fov_deg), abs=1e-9)


# ---------------------------------------------------------------------------
# Union of signed distances with per-primitive albedo (the mixed-scene mean)
# ---------------------------------------------------------------------------
def _check_point(o_s, prims, x):
    f, g, idx, gs, alb = ref.union_sdf_ref(prims, x)
    q = o_s.eval_point(x)
    assert q["mu"] == pytest.approx(f, abs=1e-12)
    assert any(np.allclose(q["G"], gg, atol=1e-12) for gg in gs), (x, q["G"], gs)
    assert q["albedo"] == pytest.approx(float(np.float32(alb)), abs=0.0)
    return idx


def test_union_sdf_and_albedo_at_random_points():
    """mu, grad mu and albedo of the 16-primitive union against exact sphere and box distances
    by closest points: at random points of the box, inside every box primitive (interior
    distances are negative, the gradient the nearest face's normal) and on thin shells around
    every primitive."""
    s = sc.mixed_scene(var_res=8, width=8, height=8, spp=1, max_depth=1)
    o_s = orc.OracleScene(s)
    prims = s.prims.astype(float)
    rng = np.random.default_rng(21)
    lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
    seen = set()
    for x in lo + (hi - lo) * rng.random((1500, 3)):
        seen.add(_check_point(o_s, prims, x))
    n_box_inside = 0
    for p in prims:
        c = p[1:4]
        for _ in range(40):
            if p[0] == 1:
                x = c + (2 * rng.random(3) - 1) * p[4:7] * 0.98
                f, _, _, _, _ = ref.union_sdf_ref(prims, x)
                n_box_inside += f < 0
            else:
                v = rng.normal(size=3)
                x = c + v / np.linalg.norm(v) * p[4] * (1 + 0.05 * (2 * rng.random() - 1))
            seen.add(_check_point(o_s, prims, x))
    assert n_box_inside > 100
    assert len(seen) == len(prims)   # every primitive was the minimum somewhere


def test_union_sdf_ties_and_box_interior_ties():
    """Ties: two coincident spheres give the lower index's albedo; a point inside a box
    equidistant from two faces gets one of the two face normals; the box distance is exact at
    edge and corner regions (distance to the edge or corner point)."""
    prims = np.array([[1, 0.1, -0.2, 0.0, 0.3, 0.2, 0.25, 0.6],
                      [0, 0.8, 0.8, 0.8, 0.2, 0, 0, 0.7],
                      [0, 0.8, 0.8, 0.8, 0.2, 0, 0, 0.9]], np.float32)
    s = sc.mixed_scene(var_res=8, width=8, height=8, spp=1, max_depth=1).replace(prims=prims)
    o_s = orc.OracleScene(s)
    pf = prims.astype(float)
    # coincident spheres: the first one wins
    for x in ([0.8, 0.8, 1.1], [0.75, 0.9, 0.85], [1.0, 0.8, 0.6]):
        q = o_s.eval_point(x)
        assert q["albedo"] == pytest.approx(float(np.float32(0.7)), abs=0.0)
        assert q["mu"] == pytest.approx(np.linalg.norm(np.subtract(x, pf[1, 1:4])) - pf[1, 4], abs=1e-12)
    # inside the box on the plane equidistant from the +x and +y faces
    c, h = pf[0, 1:4], pf[0, 4:7]
    x = c + np.array([h[0] - 0.05, h[1] - 0.05, 0.0])
    q = o_s.eval_point(x)
    assert q["mu"] == pytest.approx(-0.05, abs=1e-7)
    assert any(np.allclose(q["G"], n) for n in ([1, 0, 0], [0, 1, 0]))
    # outside near an edge and a corner: Euclidean distance to the edge / corner
    edge = c + np.array([h[0] + 0.03, h[1] + 0.04, 0.0])
    corner = c + h + np.array([0.02, 0.03, 0.06])
    for x, want in ((edge, 0.05), (corner, 0.07)):
        _check_point(o_s, pf, x)
        assert o_s.eval_point(x)["mu"] == pytest.approx(want, abs=1e-7)


# ---------------------------------------------------------------------------
# Trilinear grids (offset added to the mean, variance of the kernel)
# ---------------------------------------------------------------------------
def test_trilinear_offset_and_variance_grids():
    """mu, grad mu and sigma on a sphere mean with an offset grid and a variance grid of
    different, non-cubic resolutions over a non-cubic box, against SciPy's
    RegularGridInterpolator (node k of each axis at lo + k / (n - 1) (hi - lo)) and the
    gradient of the interpolant from its values on the bounding node planes."""
    rng = np.random.default_rng(31)
    off = rng.normal(0.0, 0.02, (5, 7, 9)).astype(np.float32)        # (nz, ny, nx)
    var = rng.uniform(1e-4, 1e-2, (10, 8, 6)).astype(np.float32)
    s = sc.sphere_scene(0.05, width=8, height=8, spp=1, max_depth=1).replace(
        bounds=_f32([-1.2, -0.9, -1.1, 1.3, 1.0, 0.8]), offset_grid=off, variance_grid=var)
    o_s = orc.OracleScene(s)
    lo, hi = s.bounds[:3].astype(float), s.bounds[3:].astype(float)
    l = orc.f32(s.lengthscale)
    for x in lo + (hi - lo) * rng.random((400, 3)):
        q = o_s.eval_point(x)
        fo, go = ref.trilinear_ref(off, lo, hi, x)
        fv, _ = ref.trilinear_ref(var, lo, hi, x)
        f_s, g_s = ref.sdf_sphere_ref(x, [0, 0, 0], 1.0)
        assert q["mu"] == pytest.approx(f_s + fo, abs=1e-12)
        np.testing.assert_allclose(q["G"], g_s + go, rtol=0, atol=1e-9)
        assert q["sigma"] == pytest.approx(math.sqrt(fv), rel=1e-12)
        assert q["s"] == pytest.approx(math.sqrt(fv) / l, rel=1e-12)
    # exactly at grid nodes the interpolant is the node value
    for (kz, ky, kx) in ((0, 0, 0), (2, 3, 4), (4, 6, 8), (1, 5, 2)):
        x = lo + np.array([kx / 8, ky / 6, kz / 4]) * (hi - lo)
        f_s, _ = ref.sdf_sphere_ref(x, [0, 0, 0], 1.0)
        assert o_s.eval_point(x)["mu"] == pytest.approx(f_s + float(off[kz, ky, kx]), abs=1e-12)
