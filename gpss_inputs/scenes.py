"""Seeded scene descriptions for the five benchmark workloads.

A scene is the statement of the rendering problem for one Gaussian process
statistical surface (GPSS): a GP mean function (a plane or a union of signed
distance primitives, optionally plus a trilinear offset grid), a squared
exponential kernel (variance, scalar or gridded, and an isotropic lengthscale),
the medium's support box and albedo, delta lights, a constant environment, a
camera and the Monte Carlo sampler settings.

Grid conventions shared by every consumer:
  * every grid is node-centred over the scene's bounding box ``bounds``;
    node (i, j, k) sits at ``lo + (i, j, k) / (res - 1) * (hi - lo)``;
  * arrays are float32 with shape (nz, ny, nx), i.e. x varies fastest.

Primitive rows are ``[kind, cx, cy, cz, a, b, c, albedo]`` with kind 0 a sphere
of radius ``a`` and kind 1 an axis-aligned box of half extents ``(a, b, c)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PRIM_SPHERE = 0
PRIM_BOX = 1

MEAN_PLANE = 0      # mu(x) = z (+ offset)
MEAN_SDF = 1        # mu(x) = min_i sdf_i(x) (+ offset)
MEAN_CONST = 2      # mu(x) = mean_const (+ offset): a homogeneous medium

CAM_ORTHO = 0
CAM_PINHOLE = 1

NDF_GENERALIZED = 0   # Sec. 4.2: the GP macrofacet (Eqs. generalized_lambda, macro_ndf)
NDF_GGX = 1           # end of Sec. 4.1: GGX height-field macrofacet


@dataclasses.dataclass
class Scene:
    name: str
    mean_kind: int
    prims: np.ndarray                      # (n, 8) float32
    bounds: np.ndarray                     # (6,) float32: lo xyz, hi xyz
    variance: float
    lengthscale: float
    albedo: float
    albedo_per_prim: bool = False
    mean_const: float = 0.0                # constant mean value (MEAN_CONST)
    variance_grid: Optional[np.ndarray] = None   # (nz, ny, nx) float32
    offset_grid: Optional[np.ndarray] = None     # (nz, ny, nx) float32
    mix_R: float = 0.5
    majorant_res: tuple = (32, 32, 32)
    dir_light: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(4, np.float32))   # toward-light dir xyz, irradiance
    point_light: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(4, np.float32))   # position xyz, intensity
    env_radiance: float = 0.0
    cam_kind: int = CAM_PINHOLE
    cam_eye: tuple = (0.0, 0.0, 4.0)
    cam_target: tuple = (0.0, 0.0, 0.0)
    cam_up: tuple = (0.0, 1.0, 0.0)
    cam_fov_deg: float = 40.0              # pinhole vertical field of view
    cam_window: tuple = (1.0, 1.0)         # orthographic window width, height
    width: int = 64
    height: int = 64
    spp: int = 16
    max_depth: int = 8
    seed: int = 0
    scene_id: int = 0
    lengthscale_n: float = 0.0             # lengthscale along the local mean-gradient direction (0: isotropic)
    ndf_kind: int = 0                      # NDF_GENERALIZED (Eq. macro_ndf) or NDF_GGX (height field)
    fresnel_eta: float = 0.0               # conductor IOR eta + i k of the Fresnel term (eta = 0: F = albedo)
    fresnel_k: float = 0.0
    observations: Optional[np.ndarray] = None   # (n, 4) float32: x, y, z, observed value (Eq. condition_gp)
    obs_noise: float = 0.0                 # observation-noise variance (> 0 when observations are given)

    @property
    def n_pixels(self) -> int:
        return self.width * self.height

    @property
    def n_paths(self) -> int:
        return self.width * self.height * self.spp

    def replace(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _dir_from_angles(zenith_deg: float, azimuth_deg: float) -> np.ndarray:
    th, ph = math.radians(zenith_deg), math.radians(azimuth_deg)
    return np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


# ---------------------------------------------------------------------------
# Workload 1: planar GPSS, tiny.
# ---------------------------------------------------------------------------
def plane_scene(width: int = 64, height: int = 64, spp: int = 16, max_depth: int = 8,
                seed: int = 0, variance: float = 0.01, lengthscale: float = 0.05,
                albedo: float = 0.9, env: float = 0.0, light_E: float = 1.0,
                light_zenith: float = 30.0, light_azimuth: float = 180.0,
                cam_zenith: float = 45.0, cam_azimuth: float = 0.0,
                majorant_res=(1, 1, 64), half_thickness: float = 0.4) -> Scene:
    """Mean m(x) = z over the unit square, bounded to |z| < half_thickness."""
    ldir = _dir_from_angles(light_zenith, light_azimuth)
    cdir = _dir_from_angles(cam_zenith, cam_azimuth)
    target = np.array([0.5, 0.5, 0.0])
    eye = target + 2.0 * cdir
    return Scene(
        name="plane",
        mean_kind=MEAN_PLANE,
        prims=np.zeros((0, 8), np.float32),
        bounds=_f32([0.0, 0.0, -half_thickness, 1.0, 1.0, half_thickness]),
        variance=float(variance), lengthscale=float(lengthscale), albedo=float(albedo),
        majorant_res=tuple(int(v) for v in majorant_res),
        dir_light=_f32([ldir[0], ldir[1], ldir[2], light_E]),
        point_light=_f32([0, 0, 0, 0]),
        env_radiance=float(env),
        cam_kind=CAM_ORTHO, cam_eye=tuple(eye), cam_target=tuple(target),
        cam_up=(0.0, 0.0, 1.0), cam_window=(1.0, 1.0),
        width=width, height=height, spp=spp, max_depth=max_depth, seed=seed,
    )


# ---------------------------------------------------------------------------
# Workload 2: unit-sphere SDF mean, lengthscale sweep.
# ---------------------------------------------------------------------------
SPHERE_LENGTHSCALES = (0.005, 0.02, 0.1, 0.5)


def sphere_scene(lengthscale: float = 0.1, width: int = 512, height: int = 512,
                 spp: int = 64, max_depth: int = 32, seed: int = 2,
                 variance: float = 0.0025, albedo: float = 0.8,
                 majorant_res=(64, 64, 64), scene_id: int = 0) -> Scene:
    return Scene(
        name=f"sphere_l{lengthscale:g}",
        mean_kind=MEAN_SDF,
        prims=_f32([[PRIM_SPHERE, 0, 0, 0, 1.0, 0, 0, albedo]]),
        bounds=_f32([-1.25, -1.25, -1.25, 1.25, 1.25, 1.25]),
        variance=float(variance), lengthscale=float(lengthscale), albedo=float(albedo),
        majorant_res=tuple(int(v) for v in majorant_res),
        point_light=_f32([2.5, 3.0, 2.0, 20.0]),
        env_radiance=0.1,
        cam_kind=CAM_PINHOLE, cam_eye=(0.0, 0.5, 4.0), cam_target=(0.0, 0.0, 0.0),
        cam_up=(0.0, 1.0, 0.0), cam_fov_deg=40.0,
        width=width, height=height, spp=spp, max_depth=max_depth, seed=seed,
        scene_id=scene_id,
    )


# ---------------------------------------------------------------------------
# Anisotropic kernel (Fig. cmp_aniso): the sphere workload with roughness alpha = 0.8 across
# the local normal and alpha_z along it; alpha = sqrt(2) sigma / l (Eq. roughness).
# ---------------------------------------------------------------------------
ANISO_ALPHA_T = 0.8
ANISO_ALPHAS_Z = (0.01, 0.8)


def aniso_sphere_scene(alpha_z: float = 0.01, alpha_t: float = ANISO_ALPHA_T, **kw) -> Scene:
    variance = kw.pop("variance", 0.0025)
    sigma = float(np.sqrt(np.float32(variance)))
    s = sphere_scene(lengthscale=float(np.sqrt(2.0) * sigma / alpha_t), variance=variance, **kw)
    return s.replace(name=f"aniso_sphere_az{alpha_z:g}",
                     lengthscale_n=float(np.sqrt(2.0) * sigma / alpha_z))


# ---------------------------------------------------------------------------
# GGX height-field macrofacet (Fig. cmp_ggx): the sphere with a thin shell (variance 1e-4,
# sigma = 0.01, as in the paper's microfacet comparisons) and GGX roughness
# alpha = sqrt(2) sigma / l in 0.1 .. 1.0.
# ---------------------------------------------------------------------------
GGX_ALPHAS = (0.1, 0.5, 1.0)


def ggx_sphere_scene(alpha: float = 0.5, variance: float = 1e-4, **kw) -> Scene:
    # the thin shell (sigma = 0.01) wants cells near its thickness: 128^3 halves the tentative
    # collisions of 64^3 for twice the cell crossings
    kw.setdefault("majorant_res", (128, 128, 128))
    sigma = float(np.sqrt(np.float32(variance)))
    s = sphere_scene(lengthscale=float(np.sqrt(2.0) * sigma / alpha), variance=variance, **kw)
    return s.replace(name=f"ggx_sphere_a{alpha:g}", ndf_kind=NDF_GGX)


# ---------------------------------------------------------------------------
# Conductor Fresnel (the F of Eq. phase with a complex index of refraction), one channel per
# scene; an RGB image is three scenes (rendered together with gpss_render_batch).  Indices
# of refraction at about 650, 550 and 450 nm (eta, k per channel; approximate handbook values).
# ---------------------------------------------------------------------------
METAL_IOR = {
    "gold": ((0.18, 0.42, 1.37), (3.42, 2.35, 1.77)),
    "copper": ((0.27, 0.68, 1.22), (3.61, 2.63, 2.29)),
}


def fresnel_rgb_scenes(scene: Scene, metal: str = "gold") -> list:
    """The scene once per color channel with that channel's conductor IOR (albedo 1)."""
    etas, ks = METAL_IOR[metal]
    return [scene.replace(name=f"{scene.name}_{metal}_{c}", fresnel_eta=float(e), fresnel_k=float(k), albedo=1.0,
                          scene_id=scene.scene_id + i)
            for i, (c, e, k) in enumerate(zip("rgb", etas, ks))]


# ---------------------------------------------------------------------------
# GP conditioned on point observations (Eq. condition_gp), the surface-reconstruction use of
# GPISes: a seeded point cloud with observed SDF values.
#   cond_sphere_scene: the sphere prior (unit-sphere SDF mean) observed at n points whose
#     radii are jittered by U(-jitter, jitter) with observed value 0, i.e. the surface is
#     pulled through them; directions on a Fibonacci sphere.
#   cond_blob_scene: a constant prior mean (outside, one prior standard deviation) and a point
#     cloud on an ellipsoid (value 0) plus points at half the semi-axes inside (value -0.2).
# Observation noise is obs_noise_frac x the kernel variance.
# ---------------------------------------------------------------------------
MAX_OBSERVATIONS = 32
# The conditioned majorant is looser per cell than the unconditioned one (it bounds the
# posterior's mean, spread and gradient over the cell); a finer grid pays for itself because a
# posterior evaluation costs about a hundred cell crossings.
COND_MAJORANT_RES = (128, 128, 128)


def fibonacci_directions(n: int) -> np.ndarray:
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = math.pi * (3.0 - math.sqrt(5.0)) * i
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)


def cond_sphere_scene(n_obs: int = 32, jitter: float = 0.08, lengthscale: float = 0.25,
                      variance: float = 0.0025, obs_noise_frac: float = 0.05, obs_seed: int = 6,
                      **kw) -> Scene:
    kw.setdefault("majorant_res", COND_MAJORANT_RES)
    rng = np.random.default_rng(obs_seed)
    dirs = fibonacci_directions(n_obs)
    rad = 1.0 + rng.uniform(-jitter, jitter, n_obs)
    obs = np.concatenate([dirs * rad[:, None], np.zeros((n_obs, 1))], axis=1)
    s = sphere_scene(lengthscale=lengthscale, variance=variance, **kw)
    return s.replace(name=f"cond_sphere_n{n_obs}", observations=_f32(obs),
                     obs_noise=float(obs_noise_frac * variance))


def cond_blob_scene(n_surface: int = 26, axes=(0.6, 0.45, 0.35), lengthscale: float = 0.3,
                    variance: float = 0.04, obs_noise_frac: float = 0.05, width: int = 512,
                    height: int = 512, spp: int = 64, max_depth: int = 32, seed: int = 7,
                    majorant_res=COND_MAJORANT_RES) -> Scene:
    ax = np.asarray(axes, np.float64)
    surf = fibonacci_directions(n_surface) * ax
    inner = np.concatenate([np.diag(0.5 * ax), -np.diag(0.5 * ax)])
    obs = np.concatenate([np.concatenate([surf, np.zeros((n_surface, 1))], axis=1),
                          np.concatenate([inner, np.full((6, 1), -0.2)], axis=1)])
    sigma = math.sqrt(variance)
    s = sphere_scene(lengthscale=lengthscale, variance=variance, width=width, height=height, spp=spp,
                     max_depth=max_depth, seed=seed, majorant_res=majorant_res)
    return s.replace(name=f"cond_blob_n{obs.shape[0]}", mean_kind=MEAN_CONST, mean_const=float(sigma),
                     prims=np.zeros((0, 8), np.float32), bounds=_f32([-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]),
                     observations=_f32(obs), obs_noise=float(obs_noise_frac * variance))


# ---------------------------------------------------------------------------
# Workload 3: union of 16 seeded primitives, value-noise variance grid.
# ---------------------------------------------------------------------------
def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise_grid(res: int, lattice: int, rng: np.random.Generator) -> np.ndarray:
    """Smoothstep-interpolated lattice of U[0,1] values sampled on res^3 nodes."""
    lat = rng.random((lattice, lattice, lattice))
    u = np.linspace(0.0, lattice - 1.0, res)
    i0 = np.minimum(np.floor(u).astype(np.int64), lattice - 2)
    f = _smoothstep(u - i0)
    # separable interpolation along x, then y, then z (array axes z, y, x)
    a = lat[:, :, i0] * (1 - f) + lat[:, :, i0 + 1] * f
    a = a[:, i0, :] * (1 - f)[None, :, None] + a[:, i0 + 1, :] * f[None, :, None]
    a = a[i0, :, :] * (1 - f)[:, None, None] + a[i0 + 1, :, :] * f[:, None, None]
    return a


def mixed_scene(width: int = 1024, height: int = 1024, spp: int = 256, max_depth: int = 64,
                seed: int = 3, n_prims: int = 16, var_res: int = 128,
                lengthscale: float = 0.03, var_lo: float = 1e-4, var_hi: float = 1e-2,
                majorant_res=(80, 80, 80)) -> Scene:
    rng = np.random.default_rng(seed)
    prims = []
    for _ in range(n_prims):
        c = rng.uniform(-1.0, 1.0, 3)
        if rng.random() < 0.5:
            r = rng.uniform(0.15, 0.35)
            prims.append([PRIM_SPHERE, *c, r, 0.0, 0.0, rng.uniform(0.5, 0.95)])
        else:
            h = rng.uniform(0.1, 0.3, 3)
            prims.append([PRIM_BOX, *c, *h, rng.uniform(0.5, 0.95)])
    t = value_noise_grid(var_res, 9, rng)
    var = np.exp(math.log(var_lo) + t * (math.log(var_hi) - math.log(var_lo)))
    return Scene(
        name="mixed16",
        mean_kind=MEAN_SDF,
        prims=_f32(prims),
        bounds=_f32([-1.5, -1.5, -1.5, 1.5, 1.5, 1.5]),
        variance=float(var_hi), lengthscale=float(lengthscale), albedo=0.8,
        albedo_per_prim=True,
        variance_grid=_f32(var),
        majorant_res=tuple(int(v) for v in majorant_res),
        point_light=_f32([2.5, 3.0, 2.0, 20.0]),
        env_radiance=0.1,
        cam_kind=CAM_PINHOLE, cam_eye=(0.0, 1.0, 5.0), cam_target=(0.0, 0.0, 0.0),
        cam_up=(0.0, 1.0, 0.0), cam_fov_deg=40.0,
        width=width, height=height, spp=spp, max_depth=max_depth, seed=seed,
    )


# ---------------------------------------------------------------------------
# Workload 4: 64 sphere scenes of uneven size for the batched renderer.
# ---------------------------------------------------------------------------
def batch_scenes(n: int = 64, seed: int = 4, resolutions=(64, 128, 256, 512),
                 spps=(4, 16, 64), l_range=(0.005, 0.5), max_depth: int = 32,
                 majorant_res=(64, 64, 64)) -> List[Scene]:
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        res = int(rng.choice(resolutions))
        spp = int(rng.choice(spps))
        l = float(math.exp(rng.uniform(math.log(l_range[0]), math.log(l_range[1]))))
        s = sphere_scene(lengthscale=l, width=res, height=res, spp=spp, max_depth=max_depth,
                         seed=seed, majorant_res=majorant_res, scene_id=i)
        s.name = f"batch{i:02d}"
        out.append(s)
    return out


# ---------------------------------------------------------------------------
# Workload 5: sphere with a 64^3 mean-offset grid (differentiable form).
# ---------------------------------------------------------------------------
def offset_sphere_scene(target: bool, width: int = 256, height: int = 256, spp: int = 16,
                        max_depth: int = 16, seed: int = 5, grid_res: int = 64,
                        offset_std: float = 0.01, majorant_res=(64, 64, 64)) -> Scene:
    """target=True gives theta* (seeded N(0, offset_std^2) offsets, var 0.0025, l 0.1,
    albedo 0.8); target=False gives theta0 (zero offsets, var 0.003, l 0.12, albedo 0.7)."""
    if target:
        rng = np.random.default_rng(seed)
        off = rng.normal(0.0, offset_std, (grid_res, grid_res, grid_res))
        var, l, alb = 0.0025, 0.1, 0.8
    else:
        off = np.zeros((grid_res, grid_res, grid_res))
        var, l, alb = 0.0030, 0.12, 0.7
    s = sphere_scene(lengthscale=l, width=width, height=height, spp=spp, max_depth=max_depth,
                     seed=seed, variance=var, albedo=alb, majorant_res=majorant_res)
    s.name = "offset_sphere_target" if target else "offset_sphere_theta0"
    s.offset_grid = _f32(off)
    return s


def grad_param_indices(scene: Scene, n_nodes: int = 29, seed: int = 5,
                       band_sigmas: float = 3.0, facing: float = 0.3) -> np.ndarray:
    """Flat indices of offset-grid nodes for finite-difference checks: nodes within
    band_sigmas standard deviations of the unit sphere on the camera-facing side."""
    nz, ny, nx = scene.offset_grid.shape
    lo, hi = scene.bounds[:3].astype(np.float64), scene.bounds[3:].astype(np.float64)
    zs, ys, xs = np.meshgrid(*[np.linspace(lo[a], hi[a], n) for a, n in
                               ((2, nz), (1, ny), (0, nx))], indexing="ij")
    r = np.sqrt(xs ** 2 + ys ** 2 + zs ** 2)
    eye = np.asarray(scene.cam_eye, np.float64)
    eye = eye / np.linalg.norm(eye)
    face = (xs * eye[0] + ys * eye[1] + zs * eye[2]) / np.maximum(r, 1e-9)
    band = np.abs(r - 1.0) < band_sigmas * math.sqrt(scene.variance)
    cand = np.flatnonzero((band & (face > facing)).ravel())
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=min(n_nodes, cand.size), replace=False))


def config_scenes(name: str):
    """The full-size workload of one benchmark configuration."""
    if name == "plane":
        return [plane_scene()]
    if name == "sphere":
        return [sphere_scene(lengthscale=l) for l in SPHERE_LENGTHSCALES]
    if name == "mixed":
        return [mixed_scene()]
    if name == "batch":
        return batch_scenes()
    if name == "offset":
        return [offset_sphere_scene(True), offset_sphere_scene(False)]
    raise KeyError(name)
