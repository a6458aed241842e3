"""Constants compiled into the HIP kernels, checked on the host: the fitted scaled
complementary error function used by the density and the projected area, and the fitted
bracket q(y) = 1 - sqrt(pi) y erfcx(y) of the projected area and the density's
log-derivative."""
import os
import re
import importlib.util

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2603_00280_amd", "csrc")


def _fit_module(name="fit_erfcx"):
    spec = importlib.util.spec_from_file_location(name, os.path.join(CSRC, name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _device_coefficients(function="erfcx_pos"):
    """The Horner coefficients of `function` in gpss_device.hpp, highest degree first."""
    src = open(os.path.join(CSRC, "gpss_device.hpp")).read()
    body = src[src.index(f"float {function}(float y)"):]
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


def test_device_mills_q_coefficients_are_the_fit():
    pytest.importorskip("mpmath")
    fit = _fit_module("fit_mills")
    dev = _device_coefficients("mills_q")
    assert len(dev) == fit.N + 1
    np.testing.assert_allclose(dev, fit.coefficients()[::-1], rtol=1e-8, atol=1e-15)


def test_device_mills_q_float32_error():
    """Evaluated in float32, the bracket stays within 3e-7 relative error of the mpmath value
    over y in [0, 1e6], where 1 - sqrt(pi) y erfcx(y) formed from the erfcx fit in float32 loses
    digits in proportion to y^2 (checked: above 1e-4 relative error at y = 100)."""
    pytest.importorskip("mpmath")
    fit = _fit_module("fit_mills")
    p = np.array(_device_coefficients("mills_q")[::-1])
    assert fit.float32_error(p) < 3e-7
    # the cancelling form it replaces, with the erfcx fit evaluated in float32
    ef = _fit_module("fit_erfcx")
    pe = np.array(_device_coefficients("erfcx_pos")[::-1])
    y = np.float32(100.0)
    t = np.float32(1) / (np.float32(1) + np.float32(0.5) * y)
    s = np.float32(2) * t - np.float32(1)
    acc = np.float32(pe[-1])
    for k in range(len(pe) - 2, -1, -1):
        acc = acc * s + np.float32(pe[k])
    e32 = t * np.float32(np.exp(acc))
    naive = np.float32(1) - np.float32(np.sqrt(np.pi)) * y * e32
    exact = fit.q_exact(np.array([100.0]))[0]
    assert abs(float(naive) / exact - 1) > 1e-4
    assert ef.N == 12
