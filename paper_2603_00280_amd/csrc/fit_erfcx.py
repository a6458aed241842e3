"""Coefficients of the single-precision scaled complementary error function of
gpss_device.hpp (erfcx_pos): erfcx(y) = e^{y^2} erfc(y) for y >= 0 written as t e^{P(2t - 1)},
t = 1 / (1 + y / 2), with P the degree-12 least-squares Chebyshev fit of log(erfcx(y) / t)
over t in (0, 1], converted to the power basis.  Prints the coefficients and the largest
relative error of a float32 evaluation (Horner, then e^x) against SciPy's erfcx."""
import numpy as np
from scipy.special import erfcx

A, N = 0.5, 12


def coefficients():
    t = np.linspace(1e-5, 1.0, 40000)
    y = (1.0 / t - 1.0) / A
    c = np.polynomial.chebyshev.chebfit(2 * t - 1, np.log(erfcx(y) / t), N)
    return np.polynomial.chebyshev.cheb2poly(c)


def float32_error(p):
    f32 = np.float32
    y = np.concatenate([np.linspace(0, 5, 200001), np.geomspace(5, 1e7, 100000)]).astype(f32)
    t = f32(1) / (f32(1) + f32(A) * y)
    s = f32(2) * t - f32(1)
    acc = np.full_like(s, f32(p[-1]))
    for k in range(N - 1, -1, -1):
        acc = acc * s + f32(p[k])
    v = (t * np.exp(acc).astype(f32)).astype(np.float64)
    return float(np.max(np.abs(v / erfcx(y.astype(np.float64)) - 1)))


if __name__ == "__main__":
    p = coefficients()
    print("    " + ", ".join(f"{v:.9e}f" for v in p))
    print("max relative error (float32 evaluation):", f"{float32_error(p):.2e}")
