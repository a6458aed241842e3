"""MI355X (gfx950) renderer for Gaussian process statistical surfaces under macrofacet
theory: HIP kernels behind the C-ABI of include/gpss.h, with a thin Python binding."""
from . import gpss  # noqa: F401  (ctypes binding; the library itself loads on first use)

__all__ = ["gpss"]
