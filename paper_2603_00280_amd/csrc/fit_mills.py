"""Coefficients of the single-precision bracket q(y) = 1 - sqrt(pi) y erfcx(y), y >= 0, of
gpss_device.hpp (mills_q).

q is 1 - z R(z) with R the Mills ratio of the standard normal at z = sqrt(2) y.  It appears in
the projected area of a ray travelling up the mean gradient, s phi(z) q, and in the density's
log-derivative inside the medium, z + phi/Phi = sqrt(2/pi) q / erfcx.  Formed from erfcx as
written, it cancels to about 1 / (2 y^2) and loses digits in proportion to y^2.  Fitted
directly, it keeps its relative accuracy: q(y) = e^{P(2t - 1)} / (1 + 2 y + 2 y^2), t = 1 / (1 + y / 2)
(the variable of erfcx_pos), with P the least-squares Chebyshev fit of log(q (1 + 2 y + 2 y^2)) over
t in (0, 1], converted to the power basis.  The reference values come from mpmath at 40
digits.  The normalization behaves as q^-1 at both ends (q = 1 - sqrt(pi) y + 2 y^2 + ... near 0,
1 / (2 y^2) + ... for large y), which leaves a function of t that a degree-12 polynomial fits
to about 1e-7.  Prints the coefficients and the largest relative error of a float32
evaluation."""
import numpy as np

A, N = 0.5, 12


def q_exact(y):
    import mpmath as mp
    mp.mp.dps = 40
    out = np.empty(len(y))
    for i, v in enumerate(y):
        v = mp.mpf(float(v))
        out[i] = float(1 - mp.sqrt(mp.pi) * v * mp.erfc(v) * mp.exp(v * v))
    return out


def coefficients():
    t = np.linspace(1e-5, 1.0, 4000)
    y = (1.0 / t - 1.0) / A
    c = np.polynomial.chebyshev.chebfit(2 * t - 1, np.log(q_exact(y) * (1.0 + 2.0 * y + 2.0 * y * y)), N)
    return np.polynomial.chebyshev.cheb2poly(c)


def float32_eval(p, y):
    f32 = np.float32
    y = np.asarray(y, f32)
    t = f32(1) / (f32(1) + f32(A) * y)
    s = f32(2) * t - f32(1)
    acc = np.full_like(s, f32(p[-1]))
    for k in range(len(p) - 2, -1, -1):
        acc = acc * s + f32(p[k])
    den = f32(1) + f32(2) * y * (f32(1) + y)
    return (np.exp(acc).astype(f32) / den).astype(np.float64)


def float32_error(p):
    y = np.concatenate([np.linspace(0, 5, 2001), np.geomspace(5, 1e6, 1000)])
    y32 = y.astype(np.float32).astype(np.float64)
    return float(np.max(np.abs(float32_eval(p, y32) / q_exact(y32) - 1)))


if __name__ == "__main__":
    p = coefficients()
    print("    " + ", ".join(f"{v:.9e}f" for v in p))
    print("max relative error (float32 evaluation):", f"{float32_error(p):.2e}")
