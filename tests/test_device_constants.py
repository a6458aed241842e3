"""Constants compiled into the HIP kernels, checked on the host: the fitted scaled
complementary error function used by the density and the projected area."""
import os
import re
import importlib.util

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2603_00280_amd", "csrc")


def _fit_module():
    spec = importlib.util.spec_from_file_location("fit_erfcx", os.path.join(CSRC, "fit_erfcx.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _device_coefficients():
    """The Horner coefficients of erfcx_pos in gpss_device.hpp, highest degree first."""
    src = open(os.path.join(CSRC, "gpss_device.hpp")).read()
    body = src[src.index("float erfcx_pos(float y)"):]
    body = body[:body.index("return")]
    first = re.search(r"float p = ([-0-9.e+]+)f;", body)
    rest = re.findall(r"p = fmaf\(p, s, ([-0-9.e+]+)f\);", body)
    return [float(first.group(1))] + [float(v) for v in rest]


def test_device_erfcx_coefficients_are_the_fit():
    """The kernel's coefficients are the committed fit's (power basis, printed to 10
    significant digits)."""
    pytest.importorskip("scipy")
    fit = _fit_module()
    dev = _device_coefficients()
    assert len(dev) == fit.N + 1
    ref = fit.coefficients()[::-1]   # highest degree first, as Horner's scheme reads them
    np.testing.assert_allclose(dev, ref, rtol=1e-8, atol=1e-15)


def test_device_erfcx_float32_error():
    """Evaluated in float32 (Horner in s = 2t - 1, then exp), the device coefficients stay
    within 4e-7 relative error of SciPy's erfcx over y in [0, 1e7]."""
    pytest.importorskip("scipy")
    fit = _fit_module()
    dev = _device_coefficients()
    p = np.array(dev[::-1])   # lowest degree first, as float32_error expects
    assert fit.float32_error(p) < 4e-7
