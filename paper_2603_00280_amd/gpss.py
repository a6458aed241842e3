"""Python binding of libgpss (argument marshalling only).

The functions below carry the C-ABI names of include/gpss.h; every rendering step runs in
the library's HIP kernels.  torch is used for device memory and streams.  Loading fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the host-sanitized build (build.py) when GPSS_SANITIZED is "abi"
LIB_PATH = os.path.join(HERE, "libgpss_san.so" if os.environ.get("GPSS_SANITIZED") == "abi" else "libgpss.so")

GPSS_OK = 0
GPSS_ERR_INVALID_ARG = -1
GPSS_ERR_HIP = -2
GPSS_ERR_OOM = -3
GPSS_ERR_UNSUPPORTED = -4
GPSS_NCOUNTERS = 16
COUNTER_NAMES = ["track_steps", "real", "nee_steps", "violations", "capped", "escaped",
                 "truncated", "cells", "phase", "nee", "nonfinite", "saturated"]

EXPORTED = ["gpss_scene_create", "gpss_scene_destroy", "gpss_scene_get_majorants", "gpss_render",
            "gpss_render_noalloc",
            "gpss_render_paths", "gpss_eval_medium", "gpss_debug_trace", "gpss_scene_set_kernel",
            "gpss_render_adjoint", "gpss_scene_set_params", "gpss_render_batch", "gpss_batch_autotune",
            "gpss_last_error"]
GPSS_KERNEL_AUTO, GPSS_KERNEL_MEGA, GPSS_KERNEL_WAVEFRONT, GPSS_KERNEL_PERSISTENT = 0, 1, 2, 3
KERNELS = {"auto": GPSS_KERNEL_AUTO, "mega": GPSS_KERNEL_MEGA, "wavefront": GPSS_KERNEL_WAVEFRONT,
           "persistent": GPSS_KERNEL_PERSISTENT}
REC_FIELDS = 16


class GpssError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpss error {code}: {msg}")
        self.code = code


class gpss_scene_desc(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("mean_kind", C.c_int32), ("mean_const", C.c_float),
        ("prims", C.POINTER(C.c_float)), ("n_prims", C.c_uint32),
        ("mean_offset", C.POINTER(C.c_float)), ("off_res", C.c_uint32 * 3),
        ("variance", C.c_float), ("variance_grid", C.POINTER(C.c_float)), ("var_res", C.c_uint32 * 3),
        ("lengthscale", C.c_float),
        ("albedo", C.c_float), ("albedo_per_prim", C.c_int32),
        ("bounds", C.c_float * 6), ("mix_R", C.c_float), ("majorant_res", C.c_uint32 * 3),
        ("dir_light", C.c_float * 4), ("point_light", C.c_float * 4), ("env_radiance", C.c_float),
        ("cam_kind", C.c_int32), ("cam_eye", C.c_float * 3), ("cam_target", C.c_float * 3),
        ("cam_up", C.c_float * 3), ("cam_fov_deg", C.c_float), ("cam_window", C.c_float * 2),
        ("width", C.c_uint32), ("height", C.c_uint32), ("spp", C.c_uint32), ("max_depth", C.c_uint32),
        ("seed", C.c_uint64), ("scene_id", C.c_uint32), ("lengthscale_n", C.c_float),
        ("ndf_kind", C.c_int32), ("fresnel_eta", C.c_float), ("fresnel_k", C.c_float),
        ("observations", C.POINTER(C.c_float)), ("n_obs", C.c_uint32), ("obs_noise", C.c_float),
    ]


_lib = None


def lib():
    """Load libgpss.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2603_00280_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, fp = C.c_void_p, C.POINTER(C.c_float)
        L.gpss_scene_create.argtypes = [C.POINTER(gpss_scene_desc), C.POINTER(vp)]
        L.gpss_scene_destroy.argtypes = [vp]
        L.gpss_scene_get_majorants.argtypes = [vp, fp, C.c_uint64]
        L.gpss_render.argtypes = [vp, vp, C.c_uint32, C.c_uint32, vp]
        L.gpss_render_noalloc.argtypes = [vp, vp, C.c_uint32, C.c_uint32, vp]
        L.gpss_render_paths.argtypes = [vp, vp, vp, C.c_uint32, C.c_uint32, vp]
        L.gpss_eval_medium.argtypes = [vp, vp, vp, vp, C.c_uint64, vp]
        L.gpss_debug_trace.argtypes = [vp, vp, C.c_uint32, vp, C.c_uint32, vp]
        L.gpss_scene_set_kernel.argtypes = [vp, C.c_int32]
        L.gpss_render_adjoint.argtypes = [vp, vp, vp, vp, C.c_uint32, C.c_uint32, vp]
        L.gpss_scene_set_params.argtypes = [vp, vp, C.c_float, C.c_float, C.c_float, vp]
        L.gpss_render_batch.argtypes = [C.POINTER(vp), C.c_uint32, C.POINTER(vp), vp]
        L.gpss_batch_autotune.argtypes = [C.POINTER(vp), C.c_uint32, C.POINTER(vp), vp,
                                          C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                          C.POINTER(C.c_float)]
        L.gpss_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name != "gpss_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def gpss_last_error() -> str:
    return lib().gpss_last_error().decode()


def _check(rc: int):
    if rc != GPSS_OK:
        raise GpssError(rc, gpss_last_error())


def _fp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def make_desc(scene):
    """gpss_scene_desc for a gpss_inputs.Scene; returns (desc, keepalive arrays)."""
    keep = []
    d = gpss_scene_desc()
    d.struct_size = C.sizeof(gpss_scene_desc)
    d.mean_kind = int(scene.mean_kind)
    d.mean_const = float(getattr(scene, "mean_const", 0.0))
    prims = np.ascontiguousarray(scene.prims, np.float32).reshape(-1, 8)
    keep.append(prims)
    d.prims = _fp(prims) if prims.size else None
    d.n_prims = prims.shape[0]
    if scene.offset_grid is not None:
        off = np.ascontiguousarray(scene.offset_grid, np.float32)
        keep.append(off)
        d.mean_offset = _fp(off)
        d.off_res[:] = [off.shape[2], off.shape[1], off.shape[0]]
    d.variance = float(scene.variance)
    if scene.variance_grid is not None:
        var = np.ascontiguousarray(scene.variance_grid, np.float32)
        keep.append(var)
        d.variance_grid = _fp(var)
        d.var_res[:] = [var.shape[2], var.shape[1], var.shape[0]]
    d.lengthscale = float(scene.lengthscale)
    d.albedo = float(scene.albedo)
    d.albedo_per_prim = int(bool(scene.albedo_per_prim))
    d.bounds[:] = [float(v) for v in scene.bounds]
    d.mix_R = float(scene.mix_R)
    d.majorant_res[:] = [int(v) for v in scene.majorant_res]
    d.dir_light[:] = [float(v) for v in scene.dir_light]
    d.point_light[:] = [float(v) for v in scene.point_light]
    d.env_radiance = float(scene.env_radiance)
    d.cam_kind = int(scene.cam_kind)
    d.cam_eye[:] = [float(v) for v in scene.cam_eye]
    d.cam_target[:] = [float(v) for v in scene.cam_target]
    d.cam_up[:] = [float(v) for v in scene.cam_up]
    d.cam_fov_deg = float(scene.cam_fov_deg)
    d.cam_window[:] = [float(v) for v in scene.cam_window]
    d.width, d.height, d.spp, d.max_depth = scene.width, scene.height, scene.spp, scene.max_depth
    d.seed = int(scene.seed)
    d.scene_id = int(scene.scene_id)
    d.lengthscale_n = float(getattr(scene, "lengthscale_n", 0.0))
    d.ndf_kind = int(getattr(scene, "ndf_kind", 0))
    d.fresnel_eta = float(getattr(scene, "fresnel_eta", 0.0))
    d.fresnel_k = float(getattr(scene, "fresnel_k", 0.0))
    obs = getattr(scene, "observations", None)
    if obs is not None and len(obs):
        obs = np.ascontiguousarray(obs, np.float32).reshape(-1, 4)
        keep.append(obs)
        d.observations = _fp(obs)
        d.n_obs = obs.shape[0]
        d.obs_noise = float(scene.obs_noise)
    return d, keep


# ---------------------------------------------------------------------------
# Thin wrappers with the C names
# ---------------------------------------------------------------------------
def gpss_scene_create(desc: gpss_scene_desc) -> int:
    h = C.c_void_p()
    _check(lib().gpss_scene_create(C.byref(desc), C.byref(h)))
    return h.value


def gpss_scene_destroy(handle: int) -> None:
    _check(lib().gpss_scene_destroy(handle))


def gpss_scene_get_majorants(handle: int, n: int) -> np.ndarray:
    out = np.zeros(n, np.float32)
    _check(lib().gpss_scene_get_majorants(handle, _fp(out), n))
    return out


def gpss_render(handle: int, image_ptr: int, s0: int, s1: int, stream=None) -> None:
    _check(lib().gpss_render(handle, image_ptr, s0, s1, _stream_ptr(stream)))


def gpss_render_noalloc(handle: int, image_ptr: int, s0: int, s1: int, stream=None) -> None:
    _check(lib().gpss_render_noalloc(handle, image_ptr, s0, s1, _stream_ptr(stream)))


def gpss_render_paths(handle: int, paths_ptr: int, counters_ptr: Optional[int], s0: int, s1: int,
                      stream=None) -> None:
    _check(lib().gpss_render_paths(handle, paths_ptr, counters_ptr, s0, s1, _stream_ptr(stream)))


def gpss_eval_medium(handle: int, pts_ptr: int, dirs_ptr: int, out_ptr: int, n: int, stream=None):
    _check(lib().gpss_eval_medium(handle, pts_ptr, dirs_ptr, out_ptr, n, _stream_ptr(stream)))


def gpss_render_adjoint(handle: int, dloss_ptr: int, grad_off_ptr: Optional[int], grad_sc_ptr: int,
                        s0: int, s1: int, stream=None) -> None:
    _check(lib().gpss_render_adjoint(handle, dloss_ptr, grad_off_ptr, grad_sc_ptr, s0, s1,
                                     _stream_ptr(stream)))


def gpss_scene_set_params(handle: int, offset_ptr: Optional[int], variance: float, lengthscale: float,
                          albedo: float, stream=None) -> None:
    _check(lib().gpss_scene_set_params(handle, offset_ptr, variance, lengthscale, albedo,
                                       _stream_ptr(stream)))


def gpss_render_batch(handles, image_ptrs, stream=None) -> None:
    n = len(handles)
    hs = (C.c_void_p * n)(*handles)
    ims = (C.c_void_p * n)(*image_ptrs)
    _check(lib().gpss_render_batch(hs, n, ims, _stream_ptr(stream)))


def gpss_batch_autotune(handles, image_ptrs, stream=None):
    n = len(handles)
    hs = (C.c_void_p * n)(*handles)
    ims = (C.c_void_p * n)(*image_ptrs)
    t, w, ms = C.c_uint32(), C.c_uint32(), C.c_float()
    _check(lib().gpss_batch_autotune(hs, n, ims, _stream_ptr(stream), C.byref(t), C.byref(w), C.byref(ms)))
    return {"tile": t.value, "waves_per_cu": w.value, "ms": ms.value}


def render_batch(scenes, outs=None, stream=None):
    """Render GpssScene objects in one persistent launch; returns their images."""
    import torch
    if outs is None:
        outs = [torch.empty(g.shape, dtype=torch.float32, device="cuda") for g in scenes]
    gpss_render_batch([g.handle for g in scenes], [o.data_ptr() for o in outs], stream)
    return outs


def gpss_scene_set_kernel(handle: int, kernel: int) -> None:
    _check(lib().gpss_scene_set_kernel(handle, kernel))


def gpss_debug_trace(handle: int, ids_ptr: int, n: int, out_ptr: int, kmax: int, stream=None):
    _check(lib().gpss_debug_trace(handle, ids_ptr, n, out_ptr, kmax, _stream_ptr(stream)))


# ---------------------------------------------------------------------------
# Scene object on torch device memory
# ---------------------------------------------------------------------------
class GpssScene:
    """A scene created in libgpss from a gpss_inputs.Scene."""

    def __init__(self, scene, kernel: str = "auto"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libgpss needs a HIP device")
        self.scene = scene
        desc, keep = make_desc(scene)
        self.handle = gpss_scene_create(desc)
        del keep
        self.set_kernel(kernel)

    def set_kernel(self, kernel: str) -> None:
        gpss_scene_set_kernel(self.handle, KERNELS[kernel])
        self.kernel = kernel

    def close(self):
        if getattr(self, "handle", None):
            gpss_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.scene.height, self.scene.width)

    def majorants(self) -> np.ndarray:
        m = self.scene.majorant_res
        return gpss_scene_get_majorants(self.handle, int(m[0] * m[1] * m[2]))

    def render(self, s0: int = 0, s1: Optional[int] = None, out=None, stream=None):
        import torch
        s1 = self.scene.spp if s1 is None else s1
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device="cuda")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert out.numel() == self.scene.n_pixels
        gpss_render(self.handle, out.data_ptr(), s0, s1, stream)
        return out

    def render_paths(self, s0: int = 0, s1: Optional[int] = None, counters: bool = False,
                     stream=None):
        import torch
        s1 = self.scene.spp if s1 is None else s1
        paths = torch.empty((self.scene.height, self.scene.width, s1 - s0), dtype=torch.float32,
                            device="cuda")
        cnt = torch.zeros(GPSS_NCOUNTERS, dtype=torch.int64, device="cuda") if counters else None
        gpss_render_paths(self.handle, paths.data_ptr(), cnt.data_ptr() if counters else None, s0,
                          s1, stream)
        if counters:
            return paths, cnt
        return paths

    def debug_trace(self, pixel_sample, kmax: int = 32, stream=None):
        """Per-vertex records of listed (pixel, sample) paths: (n, kmax, 16) and radiance (n,)."""
        import torch
        ids = torch.as_tensor(np.asarray(pixel_sample, np.uint32).reshape(-1, 2).astype(np.int32),
                              device="cuda").contiguous()
        n = ids.shape[0]
        out = torch.empty((n, kmax * REC_FIELDS + 1), dtype=torch.float32, device="cuda")
        gpss_debug_trace(self.handle, ids.data_ptr(), n, out.data_ptr(), kmax, stream)
        o = out.cpu().numpy()
        return o[:, :-1].reshape(n, kmax, REC_FIELDS), o[:, -1]

    def render_adjoint(self, dloss, s0: int = 0, s1: Optional[int] = None, stream=None):
        """(grad of the offset grid (nz, ny, nx) or None, grad of (variance, lengthscale, albedo))."""
        import torch
        s1 = self.scene.spp if s1 is None else s1
        dl = dloss.to(device="cuda", dtype=torch.float32).contiguous()
        assert dl.numel() == self.scene.n_pixels
        g_off = None
        if self.scene.offset_grid is not None:
            g_off = torch.empty(self.scene.offset_grid.shape, dtype=torch.float32, device="cuda")
        g_sc = torch.empty(3, dtype=torch.float32, device="cuda")
        gpss_render_adjoint(self.handle, dl.data_ptr(), g_off.data_ptr() if g_off is not None else None,
                            g_sc.data_ptr(), s0, s1, stream)
        return g_off, g_sc

    def set_params(self, offset=None, variance=None, lengthscale=None, albedo=None, stream=None):
        """Update the differentiable parameters (offset: device tensor of the grid's shape)."""
        import torch
        s = self.scene
        variance = float(s.variance if variance is None else variance)
        lengthscale = float(s.lengthscale if lengthscale is None else lengthscale)
        albedo = float(s.albedo if albedo is None else albedo)
        optr = None
        if offset is not None:
            off = offset.detach().to(device="cuda", dtype=torch.float32).contiguous()
            assert tuple(off.shape) == tuple(s.offset_grid.shape)
            optr = off.data_ptr()
            self._offset_keep = off
        gpss_scene_set_params(self.handle, optr, variance, lengthscale, albedo, stream)
        self.scene = s.replace(variance=variance, lengthscale=lengthscale, albedo=albedo)

    def eval_medium(self, points, dirs, stream=None):
        import torch
        pts = torch.as_tensor(np.asarray(points, np.float32), device="cuda").contiguous()
        drs = torch.as_tensor(np.asarray(dirs, np.float32), device="cuda").contiguous()
        n = pts.shape[0]
        out = torch.empty((n, 8), dtype=torch.float32, device="cuda")
        gpss_eval_medium(self.handle, pts.data_ptr(), drs.data_ptr(), out.data_ptr(), n, stream)
        return out


def counters_dict(cnt) -> dict:
    v = cnt.cpu().numpy() if hasattr(cnt, "cpu") else np.asarray(cnt)
    return dict(zip(COUNTER_NAMES, [int(x) for x in v[:len(COUNTER_NAMES)]]))
