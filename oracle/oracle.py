"""ctypes front end of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the CPU
baseline leg of the benchmark, never by the GPU library or its binding.

Scene scalars are rounded to float32 before they are handed over, so that the oracle
and the GPU library read bit-identical scene values.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the sanitized build (oracle/build.py) when GPSS_SANITIZED is "oracle"
LIB_PATH = os.path.join(HERE, "liboracle_san.so" if os.environ.get("GPSS_SANITIZED") == "oracle" else "liboracle.so")

C_TRACK_STEPS, C_REAL, C_NEE_STEPS, C_VIOLATIONS, C_CAPPED, C_ESCAPED, C_TRUNCATED, \
    C_CELLS, C_PHASE, C_NEE = range(10)
N_COUNTERS = 16
COUNTER_NAMES = ["track_steps", "real", "nee_steps", "violations", "capped", "escaped",
                 "truncated", "cells", "phase", "nee"]


class _Desc(C.Structure):
    _fields_ = [
        ("mean_kind", C.c_int32), ("mean_const", C.c_double),
        ("n_prims", C.c_int32), ("prims", C.POINTER(C.c_float)),
        ("offset", C.POINTER(C.c_float)), ("off_res", C.c_int32 * 3),
        ("variance", C.c_double), ("var_grid", C.POINTER(C.c_float)), ("var_res", C.c_int32 * 3),
        ("lengthscale", C.c_double), ("albedo", C.c_double), ("albedo_per_prim", C.c_int32),
        ("bounds", C.c_double * 6), ("mix_R", C.c_double), ("maj_res", C.c_int32 * 3),
        ("dir_light", C.c_double * 4), ("point_light", C.c_double * 4), ("env", C.c_double),
        ("cam_kind", C.c_int32), ("eye", C.c_double * 3), ("target", C.c_double * 3),
        ("up", C.c_double * 3), ("fov_deg", C.c_double), ("window", C.c_double * 2),
        ("width", C.c_int32), ("height", C.c_int32), ("spp", C.c_int32), ("max_depth", C.c_int32),
        ("seed", C.c_uint64), ("scene_id", C.c_uint32), ("lengthscale_n", C.c_double),
        ("ndf_kind", C.c_int32), ("fresnel_eta", C.c_double), ("fresnel_k", C.c_double),
        ("observations", C.POINTER(C.c_float)), ("n_obs", C.c_int32), ("obs_noise", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa
            _b.build(sanitize=LIB_PATH.endswith("_san.so"))
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.oracle_scene_create.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_void_p)]
        L.oracle_scene_destroy.argtypes = [C.c_void_p]
        L.oracle_majorants.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64]
        L.oracle_render.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp, dp, dp, dp,
                                    C.POINTER(C.c_int64), C.c_int32]
        L.oracle_render_pixels.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int64, C.c_int32,
                                           C.c_int32, dp, dp, C.POINTER(C.c_int64), C.c_int32]
        L.oracle_render_frozen.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, dp,
                                           C.POINTER(C.c_int64), C.c_int32]
        L.oracle_render_frozen_pixels.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.c_int64,
                                                  C.c_int32, C.c_int32, dp, C.c_int32]
        L.oracle_render_grad.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp, C.c_int32,
                                         C.POINTER(C.c_int64), dp, dp, C.c_int32]
        L.oracle_debug_trace.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int32, dp]
        L.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.oracle_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.c_uint32, C.c_int32, dp]
        for name in ("oracle_erfcx", "oracle_erfinv", "oracle_beckmann_lambda"):
            getattr(L, name).argtypes = [C.c_double]
            getattr(L, name).restype = C.c_double
        for name in ("oracle_ndf_aniso", "oracle_lambda_aniso"):
            getattr(L, name).argtypes = [C.c_double, C.c_double, C.c_double, dp]
            getattr(L, name).restype = C.c_double
        for name in ("oracle_sigma_proj_n", "oracle_ndf_n"):
            getattr(L, name).argtypes = [dp, C.c_double, C.c_double, dp]
            getattr(L, name).restype = C.c_double
        L.oracle_rho.argtypes = [C.c_double, C.c_double]
        L.oracle_rho.restype = C.c_double
        L.oracle_beckmann_ndf.argtypes = [C.c_double, C.c_double]
        L.oracle_beckmann_ndf.restype = C.c_double
        L.oracle_sigma_proj.argtypes = [dp, C.c_double, dp]
        L.oracle_sigma_proj.restype = C.c_double
        L.oracle_ndf.argtypes = [dp, C.c_double, dp]
        L.oracle_ndf.restype = C.c_double
        for sfx in ("", "_ggx"):
            getattr(L, "oracle_phase_eval" + sfx).argtypes = [dp, C.c_double, C.c_double, dp, dp]
            getattr(L, "oracle_phase_eval" + sfx).restype = C.c_double
            getattr(L, "oracle_mixture_pdf" + sfx).argtypes = [dp, C.c_double, C.c_double, dp, dp]
            getattr(L, "oracle_mixture_pdf" + sfx).restype = C.c_double
        L.oracle_phase_eval_at.argtypes = [C.c_void_p, dp, dp, dp]
        L.oracle_phase_eval_at.restype = C.c_double
        L.oracle_fresnel_conductor.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_fresnel_conductor.restype = C.c_double
        for name in ("oracle_sigma_proj_ggx", "oracle_ndf_ggx"):
            getattr(L, name).argtypes = [dp, C.c_double, dp]
            getattr(L, name).restype = C.c_double
        L.oracle_phase_sample.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp,
                                          dp, dp]
        L.oracle_phase_sample_ggx.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, dp, dp, dp,
                                          dp, dp]
        L.oracle_posterior.argtypes = [C.c_void_p, dp, dp]
        for name in ("oracle_sigma_proj_cov", "oracle_ndf_cov"):
            getattr(L, name).argtypes = [dp, dp, dp]
            getattr(L, name).restype = C.c_double
        L.oracle_eval_point.argtypes = [C.c_void_p, dp, dp]
        L.oracle_sigma_t.argtypes = [C.c_void_p, dp, dp]
        L.oracle_sigma_t.restype = C.c_double
        L.oracle_ratio_tracking.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_int32, dp]
        L.oracle_free_flight.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_int32, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def f32(x) -> float:
    return float(np.float32(x))


class OracleScene:
    """Oracle-side copy of a gpss_inputs.Scene (owns the C handle)."""

    def __init__(self, scene, **override):
        s = scene.replace(**override) if override else scene
        self.scene = s
        d = _Desc()
        d.mean_kind = int(s.mean_kind)
        d.mean_const = f32(getattr(s, "mean_const", 0.0))
        self._prims = np.ascontiguousarray(s.prims, np.float32).reshape(-1, 8)
        d.n_prims = self._prims.shape[0]
        d.prims = self._prims.ctypes.data_as(C.POINTER(C.c_float))
        self._off = None
        if s.offset_grid is not None:
            self._off = np.ascontiguousarray(s.offset_grid, np.float32)
            nz, ny, nx = self._off.shape
            d.offset = self._off.ctypes.data_as(C.POINTER(C.c_float))
            d.off_res[:] = [nx, ny, nz]
        self._var = None
        if s.variance_grid is not None:
            self._var = np.ascontiguousarray(s.variance_grid, np.float32)
            nz, ny, nx = self._var.shape
            d.var_grid = self._var.ctypes.data_as(C.POINTER(C.c_float))
            d.var_res[:] = [nx, ny, nz]
        d.variance = f32(s.variance)
        d.lengthscale = f32(s.lengthscale)
        d.albedo = f32(s.albedo)
        d.albedo_per_prim = int(bool(s.albedo_per_prim))
        d.bounds[:] = [f32(v) for v in s.bounds]
        d.mix_R = f32(s.mix_R)
        d.maj_res[:] = [int(v) for v in s.majorant_res]
        d.dir_light[:] = [f32(v) for v in s.dir_light]
        d.point_light[:] = [f32(v) for v in s.point_light]
        d.env = f32(s.env_radiance)
        d.cam_kind = int(s.cam_kind)
        d.eye[:] = [f32(v) for v in s.cam_eye]
        d.target[:] = [f32(v) for v in s.cam_target]
        d.up[:] = [f32(v) for v in s.cam_up]
        d.fov_deg = f32(s.cam_fov_deg)
        d.window[:] = [f32(v) for v in s.cam_window]
        d.width, d.height, d.spp, d.max_depth = s.width, s.height, s.spp, s.max_depth
        d.seed = int(s.seed)
        d.scene_id = int(s.scene_id)
        d.lengthscale_n = f32(s.lengthscale_n)
        d.ndf_kind = int(s.ndf_kind)
        d.fresnel_eta = f32(s.fresnel_eta)
        d.fresnel_k = f32(s.fresnel_k)
        obs = getattr(s, "observations", None)
        if obs is not None and len(obs):
            self._obs = np.ascontiguousarray(obs, np.float32).reshape(-1, 4)
            d.observations = self._obs.ctypes.data_as(C.POINTER(C.c_float))
            d.n_obs = self._obs.shape[0]
            d.obs_noise = f32(s.obs_noise)
        self._desc = d
        h = C.c_void_p()
        rc = lib().oracle_scene_create(C.byref(d), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_scene_create rejected the scene ({rc})")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib().oracle_scene_destroy(h)
            self.handle = None

    # ---- whole-image functions ----
    @property
    def n_majorant_cells(self) -> int:
        m = self.scene.majorant_res
        return int(m[0] * m[1] * m[2])

    def majorants(self) -> np.ndarray:
        n = self.n_majorant_cells
        out = np.zeros(n, np.float32)
        rc = lib().oracle_majorants(self.handle, out.ctypes.data_as(C.POINTER(C.c_float)), n)
        assert rc == 0
        return out

    def render(self, s0: int = 0, s1: Optional[int] = None, want_paths: bool = False,
               nthreads: int = 0):
        s = self.scene
        s1 = s.spp if s1 is None else s1
        npix = s.width * s.height
        mean = np.zeros(npix)
        var = np.zeros(npix)
        trunc = np.zeros(npix)
        paths = np.zeros(npix * (s1 - s0)) if want_paths else None
        cnt = np.zeros(N_COUNTERS, np.int64)
        rc = lib().oracle_render(self.handle, s0, s1, _dp(mean), _dp(var),
                                 _dp(paths) if want_paths else None, _dp(trunc),
                                 cnt.ctypes.data_as(C.POINTER(C.c_int64)), nthreads)
        assert rc == 0
        out = {"mean": mean.reshape(s.height, s.width), "var": var.reshape(s.height, s.width),
               "trunc": trunc.reshape(s.height, s.width),
               "counters": dict(zip(COUNTER_NAMES, cnt[:len(COUNTER_NAMES)].tolist()))}
        if want_paths:
            out["paths"] = paths.reshape(s.height, s.width, s1 - s0)
        return out

    def render_pixels(self, pixels, s0: int = 0, s1: Optional[int] = None, nthreads: int = 0):
        """Mean and variance of the listed pixels (flat indices) over samples [s0, s1)."""
        s = self.scene
        s1 = s.spp if s1 is None else s1
        px = np.ascontiguousarray(np.asarray(pixels, np.int64))
        mean, var = np.zeros(px.size), np.zeros(px.size)
        rc = lib().oracle_render_pixels(self.handle, px.ctypes.data_as(C.POINTER(C.c_int64)), px.size,
                                        s0, s1, _dp(mean), _dp(var), None, nthreads)
        assert rc == 0
        return {"mean": mean, "var": var}

    def render_frozen(self, weights: "OracleScene", s0: int = 0, s1: Optional[int] = None,
                      nthreads: int = 0) -> np.ndarray:
        s = self.scene
        s1 = s.spp if s1 is None else s1
        mean = np.zeros(s.width * s.height)
        rc = lib().oracle_render_frozen(self.handle, weights.handle, s0, s1, _dp(mean), None,
                                        nthreads)
        assert rc == 0
        return mean.reshape(s.height, s.width)

    def render_frozen_pixels(self, weights: "OracleScene", pixels, s0: int = 0, s1: Optional[int] = None,
                             nthreads: int = 0) -> np.ndarray:
        """Frozen-sampling render (decisions from this scene, weights from `weights`) of the
        listed pixels (flat indices) over samples [s0, s1)."""
        s = self.scene
        s1 = s.spp if s1 is None else s1
        px = np.ascontiguousarray(np.asarray(pixels, np.int64))
        mean = np.zeros(px.size)
        rc = lib().oracle_render_frozen_pixels(self.handle, weights.handle,
                                               px.ctypes.data_as(C.POINTER(C.c_int64)), px.size, s0, s1,
                                               _dp(mean), nthreads)
        assert rc == 0
        return mean

    def render_grad(self, dloss: np.ndarray, param_ids: Sequence[int], s0: int = 0,
                    s1: Optional[int] = None, nthreads: int = 0, want_image: bool = True):
        """Gradient of sum(dloss * image) at the selected parameters (and the image, unless
        want_image is False, in which case pixels with zero dloss are not traced)."""
        s = self.scene
        s1 = s.spp if s1 is None else s1
        dl = _vec(dloss).ravel()
        ids = np.ascontiguousarray(np.asarray(param_ids, np.int64))
        g = np.zeros(ids.size)
        mean = np.zeros(s.width * s.height) if want_image else None
        rc = lib().oracle_render_grad(self.handle, s0, s1, _dp(dl), int(ids.size),
                                      ids.ctypes.data_as(C.POINTER(C.c_int64)), _dp(g),
                                      _dp(mean) if want_image else None, nthreads)
        assert rc == 0
        return g, (mean.reshape(s.height, s.width) if want_image else None)

    def debug_trace(self, pixel: int, sample: int, kmax: int = 32):
        out = np.zeros(16 * kmax + 1)
        rc = lib().oracle_debug_trace(self.handle, pixel, sample, kmax, _dp(out))
        assert rc == 0
        return out[:-1].reshape(kmax, 16), out[-1]

    # ---- point functions ----
    def eval_point(self, x):
        out = np.zeros(8)
        lib().oracle_eval_point(self.handle, _dp(_vec(x)), _dp(out))
        return {"mu": out[0], "G": out[1:4].copy(), "sigma": out[4], "s": out[5],
                "albedo": out[6], "sn": out[7]}

    def posterior(self, x):
        """Conditioned scenes: posterior of (f(x), grad f(x)) (Eq. condition_gp) and the
        gradient distribution given f(x) = 0."""
        out = np.zeros(23)
        rc = lib().oracle_posterior(self.handle, _dp(_vec(x)), _dp(out))
        assert rc == 0, "not a conditioned scene"
        return {"mu": out[0], "grad": out[1:4].copy(), "var": out[4], "c": out[5:8].copy(),
                "Sgg": _sym(out[8:14]), "mg": out[14:17].copy(), "Sg": _sym(out[17:23])}

    def phase_eval_at(self, x, d, wi) -> float:
        return lib().oracle_phase_eval_at(self.handle, _dp(_vec(x)), _dp(_vec(d)), _dp(_vec(wi)))

    def sigma_t(self, x, d) -> float:
        return lib().oracle_sigma_t(self.handle, _dp(_vec(x)), _dp(_vec(d)))

    def ratio_tracking(self, o, d, tmax: float, n: int) -> np.ndarray:
        out = np.zeros(n)
        rc = lib().oracle_ratio_tracking(self.handle, _dp(_vec(o)), _dp(_vec(d)), float(tmax), n,
                                         _dp(out))
        assert rc == 0
        return out

    def free_flight(self, o, d, tmax: float, n: int) -> np.ndarray:
        out = np.zeros(n)
        lib().oracle_free_flight(self.handle, _dp(_vec(o)), _dp(_vec(d)), float(tmax), n, _dp(out))
        return out


# ---- free functions ----
def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return np.array(list(o), np.uint32)


def uniforms(seed, scene_id, pixel, sample, bounce, stream, n) -> np.ndarray:
    out = np.zeros(n)
    lib().oracle_uniforms(seed, scene_id, pixel, sample, bounce, stream, n, _dp(out))
    return out


def erfcx(x: float) -> float:
    return lib().oracle_erfcx(float(x))


def erfinv(y: float) -> float:
    return lib().oracle_erfinv(float(y))


def rho(mu: float, sigma: float) -> float:
    return lib().oracle_rho(float(mu), float(sigma))


def sigma_proj(G, s: float, d) -> float:
    return lib().oracle_sigma_proj(_dp(_vec(G)), float(s), _dp(_vec(d)))


def ndf(G, s: float, wm) -> float:
    return lib().oracle_ndf(_dp(_vec(G)), float(s), _dp(_vec(wm)))


def sigma_proj_n(G, s: float, sn: float, d) -> float:
    """Projected area with gradient std s across and sn along n = G/|G| (z if G = 0)."""
    return lib().oracle_sigma_proj_n(_dp(_vec(G)), float(s), float(sn), _dp(_vec(d)))


def ndf_n(G, s: float, sn: float, wm) -> float:
    """Generalized NDF with gradient std s across and sn along n = G/|G| (z if G = 0)."""
    return lib().oracle_ndf_n(_dp(_vec(G)), float(s), float(sn), _dp(_vec(wm)))


def beckmann_ndf(alpha: float, cos_m: float) -> float:
    return lib().oracle_beckmann_ndf(float(alpha), float(cos_m))


def ndf_aniso(ax, ay, az, wm) -> float:
    return lib().oracle_ndf_aniso(float(ax), float(ay), float(az), _dp(_vec(wm)))


def lambda_aniso(ax, ay, az, w) -> float:
    return lib().oracle_lambda_aniso(float(ax), float(ay), float(az), _dp(_vec(w)))


def beckmann_lambda(a: float) -> float:
    return lib().oracle_beckmann_lambda(float(a))


def phase_eval(G, s, albedo, d, wi, ggx: bool = False) -> float:
    f = lib().oracle_phase_eval_ggx if ggx else lib().oracle_phase_eval
    return f(_dp(_vec(G)), float(s), float(albedo), _dp(_vec(d)), _dp(_vec(wi)))


def mixture_pdf(G, s, R, d, wm, ggx: bool = False) -> float:
    f = lib().oracle_mixture_pdf_ggx if ggx else lib().oracle_mixture_pdf
    return f(_dp(_vec(G)), float(s), float(R), _dp(_vec(d)), _dp(_vec(wm)))


def phase_sample(G, s, albedo, R, d, u, ggx: bool = False):
    wi, wm = np.zeros(3), np.zeros(3)
    w, p = np.zeros(1), np.zeros(1)
    f = lib().oracle_phase_sample_ggx if ggx else lib().oracle_phase_sample
    f(_dp(_vec(G)), float(s), float(albedo), float(R), _dp(_vec(d)), _dp(_vec(u)), _dp(wi), _dp(wm),
      _dp(w), _dp(p))
    return wi, wm, float(w[0]), float(p[0])


def _sym(c6) -> np.ndarray:
    xx, xy, xz, yy, yz, zz = c6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def _six(S) -> np.ndarray:
    S = np.asarray(S, np.float64)
    return _vec([S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]])


def sigma_proj_cov(G, Sigma, d) -> float:
    """E[max(0, -d.g)] for g ~ N(G, Sigma) with a full 3x3 covariance."""
    return lib().oracle_sigma_proj_cov(_dp(_vec(G)), _dp(_six(Sigma)), _dp(_vec(d)))


def ndf_cov(G, Sigma, wm) -> float:
    """Generalized NDF int_0^inf r^3 N(r wm; G, Sigma) dr with a full 3x3 covariance."""
    return lib().oracle_ndf_cov(_dp(_vec(G)), _dp(_six(Sigma)), _dp(_vec(wm)))


def fresnel_conductor(c: float, eta: float, k: float) -> float:
    return lib().oracle_fresnel_conductor(float(c), float(eta), float(k))


def sigma_proj_ggx(G, s: float, d) -> float:
    """Projected area of the GGX height-field macrofacet (roughness sqrt(2) s / |G|)."""
    return lib().oracle_sigma_proj_ggx(_dp(_vec(G)), float(s), _dp(_vec(d)))


def ndf_ggx(G, s: float, wm) -> float:
    """GGX NDF about G/|G| with roughness sqrt(2) s / |G|, scaled by |G|."""
    return lib().oracle_ndf_ggx(_dp(_vec(G)), float(s), _dp(_vec(wm)))
