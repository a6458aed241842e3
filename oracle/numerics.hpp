// Oracle numerics: Philox4x32-10, special functions and forward-mode dual numbers.
// TEST INFRASTRUCTURE ONLY (see oracle.h).  Double precision throughout.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>

namespace orc {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kSqrt2Pi = 2.50662827463100050242;

// ---------------------------------------------------------------------------
// Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
// 32x32->64 multiplications with the round key bumped by the Weyl constants
// between rounds.
// ---------------------------------------------------------------------------
inline void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// Random-number stream of one (pixel, sample, bounce, stream) address.  Draws are
// consumed in order; the fourth counter word counts blocks of four draws.  A uniform
// keeps the top 24 bits of a draw, so it is exact in single and double precision.
enum Stream : uint32_t { kCam = 0, kTrack = 1, kPhase = 2, kNee0 = 3 };

struct Rng {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int pos;
    Rng(const uint32_t k[2], uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t stream) {
        key[0] = k[0]; key[1] = k[1];
        ctr[0] = pixel; ctr[1] = sample; ctr[2] = (bounce & 0xFFFFu) | (stream << 16); ctr[3] = 0;
        pos = 4;
    }
    uint32_t next() {
        if (pos == 4) {
            philox4x32_10(ctr, key, buf);
            ctr[3] += 1;
            pos = 0;
        }
        return buf[pos++];
    }
    uint32_t next24() { return next() >> 8; }
    double uniform() { return (double)next24() * 0x1p-24; }
};

// ---------------------------------------------------------------------------
// Special functions.  erfc/erf/exp come from the C library; the scaled
// complementary error function erfcx(x) = exp(x^2) erfc(x) uses the direct
// product where erfc does not underflow and Laplace's continued fraction
//   erfc(x) = exp(-x^2)/sqrt(pi) * 1/(x + (1/2)/(x + 1/(x + (3/2)/(x + ...))))
// (evaluated bottom-up) in the far tail.
// ---------------------------------------------------------------------------
inline double erfcx_d(double x) {
    if (x < 0.0) {
        if (x < -26.0) return INFINITY;
        return 2.0 * std::exp(x * x) - erfcx_d(-x);
    }
    if (x < 5.0) return std::exp(x * x) * std::erfc(x);
    double f = x;
    for (int k = 120; k >= 1; --k) f = x + (0.5 * k) / f;
    return 1.0 / (kSqrtPi * f);
}

inline double Phi_d(double z) { return 0.5 * std::erfc(-z / kSqrt2); }
inline double phi_d(double z) { return std::exp(-0.5 * z * z) / kSqrt2Pi; }

// Inverse error function on (-1, 1): Newton iterations on erf, safeguarded by
// bisection on the bracket [-8, 8].
inline double erfinv_d(double y) {
    if (y <= -1.0) return -INFINITY;
    if (y >= 1.0) return INFINITY;
    // f(x) = erf(x) - y, written with erfc near |y| -> 1 so that it keeps its digits
    auto f = [y](double x) {
        if (y > 0.5) return (1.0 - y) - std::erfc(x);
        if (y < -0.5) return std::erfc(-x) - (1.0 + y);
        return std::erf(x) - y;
    };
    double lo = -8.0, hi = 8.0, x = 0.0;
    for (int it = 0; it < 200; ++it) {
        const double fx = f(x);
        if (fx == 0.0) break;
        if (fx > 0.0) hi = x; else lo = x;
        const double fp = 2.0 / kSqrtPi * std::exp(-x * x);
        double xn = x - fx / fp;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const double step = xn - x;
        x = xn;
        if (std::fabs(step) <= 4e-16 * std::fmax(1.0, std::fabs(x))) break;
    }
    return x;
}

// ---------------------------------------------------------------------------
// Forward-mode dual numbers with a fixed number of derivative slots.
// ---------------------------------------------------------------------------
struct Dual {
    static constexpr int N = 32;
    double v;
    double d[N];
    Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
    Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT: implicit from double
    static Dual var(double x, int slot) {
        Dual r(x);
        if (slot >= 0) r.d[slot] = 1.0;
        return r;
    }
};

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }

// y = f(x) with f'(x) = fp
inline Dual chain(const Dual& x, double fx, double fp) {
    Dual r(fx);
    for (int i = 0; i < Dual::N; ++i) r.d[i] = fp * x.d[i];
    return r;
}
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int i = 0; i < Dual::N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int i = 0; i < Dual::N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int i = 0; i < Dual::N; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int i = 0; i < Dual::N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
    Dual r(a.v / b.v);
    const double ib2 = 1.0 / (b.v * b.v);
    for (int i = 0; i < Dual::N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) * ib2;
    return r;
}
inline Dual operator+(const Dual& a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double a, const Dual& b) { return b + a; }
inline Dual operator-(const Dual& a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double a, const Dual& b) { return -b + a; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int i = 0; i < Dual::N; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator*=(Dual& a, const Dual& b) { a = a * b; return a; }

inline double t_exp(double x) { return std::exp(x); }
inline Dual t_exp(const Dual& x) { double e = std::exp(x.v); return chain(x, e, e); }
inline double t_sqrt(double x) { return std::sqrt(x); }
inline Dual t_sqrt(const Dual& x) { double s = std::sqrt(x.v); return chain(x, s, 0.5 / s); }
inline double t_erfc(double x) { return std::erfc(x); }
inline Dual t_erfc(const Dual& x) { return chain(x, std::erfc(x.v), -2.0 / kSqrtPi * std::exp(-x.v * x.v)); }
inline double t_erfcx(double x) { return erfcx_d(x); }
inline Dual t_erfcx(const Dual& x) { double e = erfcx_d(x.v); return chain(x, e, 2.0 * x.v * e - 2.0 / kSqrtPi); }
inline double t_pow(double x, double p) { return std::pow(x, p); }
inline Dual t_pow(const Dual& x, double p) { double y = std::pow(x.v, p); return chain(x, y, p * std::pow(x.v, p - 1.0)); }

}  // namespace orc
