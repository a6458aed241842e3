// FP64 CPU oracle: macrofacet rendering of Gaussian process statistical surfaces.
// TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain and slow on purpose: every
// quantity is evaluated from the paper's printed formula in double precision, one
// path at a time, with no blocking, caching or reordering.
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include <omp.h>

#include "numerics.hpp"

using namespace orc;

namespace {

struct Grid {
    int res[3] = {0, 0, 0};
    std::vector<double> v;
    bool empty() const { return v.empty(); }
};

struct Prim {
    int kind;
    double c[3];
    double h[3];
    double albedo;
};

}  // namespace

struct oracle_scene {
    int mean_kind;
    double mean_const;
    std::vector<Prim> prims;
    Grid offset, var;
    double variance, l, albedo;
    double l_n;            // lengthscale along the local mean-gradient direction (= l: isotropic)
    bool aniso;            // l_n != l
    bool ggx;              // GGX height-field macrofacet (NDF and Lambda of GGX) instead of Eq. macro_ndf
    double f_eta, f_k;     // conductor index of refraction eta + i k of the Fresnel term (eta = 0: F = albedo)
    bool albedo_per_prim;
    // GP conditioned on point observations (Eq. condition_gp): positions (3 per point),
    // observed values, noise variance, the Cholesky factor of kappa(C, C) + noise I (row-major,
    // lower) and the weights alpha = (kappa(C, C) + noise I)^-1 (m - mu(C)).
    bool cond;
    int n_obs;
    std::vector<double> obs_x, obs_m, obs_L, obs_alpha;
    double obs_noise;
    double lo[3], hi[3], ext[3];
    double R;
    int M[3];
    double cw[3];
    std::vector<double> maj;
    double dl[4], pl[4], env;
    int cam_kind;
    double eye[3], fwd[3], right[3], upc[3];
    double tan_half, aspect, win[2];
    int W, H, spp, max_depth;
    uint32_t key[2];
};

namespace {

using Scene = oracle_scene;

inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
inline void normalize3(double a[3]) {
    const double n = std::sqrt(dot3(a, a));
    a[0] /= n; a[1] /= n; a[2] /= n;
}

// Orthonormal basis around a unit vector n (Duff et al., "Building an orthonormal
// basis, revisited", JCGT 2017).
inline void onb(const double n[3], double t[3], double b[3]) {
    const double sign = std::copysign(1.0, n[2]);
    const double a = -1.0 / (sign + n[2]);
    const double bb = n[0] * n[1] * a;
    t[0] = 1.0 + sign * n[0] * n[0] * a; t[1] = sign * bb; t[2] = -sign * n[0];
    b[0] = bb; b[1] = sign + n[1] * n[1] * a; b[2] = -n[1];
}

struct Counters {
    int64_t c[ORC_C_COUNT] = {};
    void add(const Counters& o) { for (int i = 0; i < ORC_C_COUNT; ++i) c[i] += o.c[i]; }
};

// ---------------------------------------------------------------------------
// Mean function geometry (the parameter-free part of mu and grad mu).
// ---------------------------------------------------------------------------
void sdf_prim(const Prim& p, const double x[3], double& f, double g[3]) {
    if (p.kind == 0) {
        const double v[3] = {x[0] - p.c[0], x[1] - p.c[1], x[2] - p.c[2]};
        const double r = std::sqrt(dot3(v, v));
        f = r - p.h[0];
        if (r > 0.0) { g[0] = v[0] / r; g[1] = v[1] / r; g[2] = v[2] / r; }
        else { g[0] = 0.0; g[1] = 0.0; g[2] = 1.0; }
        return;
    }
    // axis-aligned box: exact signed distance
    double q[3], sg[3];
    for (int a = 0; a < 3; ++a) {
        const double dx = x[a] - p.c[a];
        sg[a] = dx < 0.0 ? -1.0 : 1.0;
        q[a] = std::fabs(dx) - p.h[a];
    }
    const double qmax = std::max(q[0], std::max(q[1], q[2]));
    if (qmax > 0.0) {
        double qp[3] = {std::max(q[0], 0.0), std::max(q[1], 0.0), std::max(q[2], 0.0)};
        const double n = std::sqrt(dot3(qp, qp));
        f = n;
        for (int a = 0; a < 3; ++a) g[a] = sg[a] * qp[a] / n;
    } else {
        f = qmax;
        int ax = 0;
        if (q[1] > q[ax]) ax = 1;
        if (q[2] > q[ax]) ax = 2;
        g[0] = g[1] = g[2] = 0.0;
        g[ax] = sg[ax];
    }
}

// Lower bound of a primitive's signed distance over the box [blo, bhi] (the majorant's mean
// bound; any lower bound keeps the majorant valid, a tight one keeps it small).  Sphere: the
// distance from its centre to the box, minus the radius (exact).  Box (centre c, half extents
// h): along each axis m_a is the smallest |x_a - c_a| - h_a over the box; the signed distance
// is never below max_a of |x_a - c_a| - h_a, and where some m_a > 0 the whole box lies outside
// the primitive, where the distance is the length of the positive parts.
double sdf_prim_min(const Prim& p, const double blo[3], const double bhi[3]) {
    double m[3];
    for (int a = 0; a < 3; ++a) {
        const double gap = p.c[a] < blo[a] ? blo[a] - p.c[a] : (p.c[a] > bhi[a] ? p.c[a] - bhi[a] : 0.0);
        m[a] = p.kind == 0 ? gap : gap - p.h[a];
    }
    if (p.kind == 0) return std::sqrt(dot3(m, m)) - p.h[0];
    const double mmax = std::max(m[0], std::max(m[1], m[2]));
    if (!(mmax > 0.0)) return mmax;
    const double mp[3] = {std::max(m[0], 0.0), std::max(m[1], 0.0), std::max(m[2], 0.0)};
    return std::sqrt(dot3(mp, mp));
}

double sdf_union(const Scene& S, const double x[3], double g[3], int& which) {
    double best = INFINITY;
    which = -1;
    for (size_t i = 0; i < S.prims.size(); ++i) {
        double f, gi[3];
        sdf_prim(S.prims[i], x, f, gi);
        if (f < best) { best = f; which = (int)i; g[0] = gi[0]; g[1] = gi[1]; g[2] = gi[2]; }
    }
    return best;
}

void mean_geom(const Scene& S, const double x[3], double& f, double g[3], int& which) {
    which = -1;
    if (S.mean_kind == 0) { f = x[2]; g[0] = 0; g[1] = 0; g[2] = 1; return; }
    if (S.mean_kind == 2) { f = S.mean_const; g[0] = g[1] = g[2] = 0; return; }
    f = sdf_union(S, x, g, which);
}

// Trilinear interpolation on a node-centred grid over the scene box.
struct Tri {
    int64_t idx[8];
    double w[8];
    double dw[8][3];
};

void trilinear(const Grid& G, const Scene& S, const double x[3], Tri& t) {
    int i0[3];
    double f[3], sc[3];
    for (int a = 0; a < 3; ++a) {
        double u = (x[a] - S.lo[a]) / S.ext[a] * (G.res[a] - 1);
        u = std::min(std::max(u, 0.0), (double)(G.res[a] - 1));
        int i = (int)std::floor(u);
        if (i > G.res[a] - 2) i = G.res[a] - 2;
        i0[a] = i;
        f[a] = u - i;
        sc[a] = (G.res[a] - 1) / S.ext[a];
    }
    int n = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx, ++n) {
                const double wx = dx ? f[0] : 1.0 - f[0];
                const double wy = dy ? f[1] : 1.0 - f[1];
                const double wz = dz ? f[2] : 1.0 - f[2];
                t.idx[n] = ((int64_t)(i0[2] + dz) * G.res[1] + (i0[1] + dy)) * G.res[0] + (i0[0] + dx);
                t.w[n] = wx * wy * wz;
                t.dw[n][0] = (dx ? 1.0 : -1.0) * sc[0] * wy * wz;
                t.dw[n][1] = (dy ? 1.0 : -1.0) * sc[1] * wx * wz;
                t.dw[n][2] = (dz ? 1.0 : -1.0) * sc[2] * wx * wy;
            }
}

// ---------------------------------------------------------------------------
// GP conditioned on point observations (Sec. 3.1, Eq. condition_gp).  The observations
// (C, m) carry independent Gaussian noise of variance s_n^2 > 0, which adds s_n^2 I to
// kappa(C, C); s_n -> 0 is the equation as printed.  The posterior of the value and the
// gradient at x follows from the same equation applied to the jointly Gaussian vector
// (f(x), grad f(x)) (Eq. joint_fg), whose covariances with f(C) are kappa(x, C) and
// grad_x kappa(x, C), and whose prior covariance at one point is diag(sigma^2, sigma^2/l^2 I)
// for the squared-exponential kernel (Eq. se_kernel).
// ---------------------------------------------------------------------------
double se_kernel(const Scene& S, const double x[3], const double y[3]) {
    const double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    return S.variance * std::exp(-dot3(d, d) / (2.0 * S.l * S.l));
}

// In-place Cholesky factor (lower, row-major) of a symmetric positive definite matrix.
bool cholesky(std::vector<double>& a, int n) {
    for (int j = 0; j < n; ++j) {
        double d = a[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        a[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = a[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
            a[(size_t)i * n + j] = v / d;
        }
        for (int i = 0; i < j; ++i) a[(size_t)i * n + j] = 0.0;
    }
    return true;
}

// Solve (L L^T) x = b in place.
void chol_solve(const std::vector<double>& L, int n, double* b) {
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * b[k];
        b[i] = v / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = b[i];
        for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * b[k];
        b[i] = v / L[(size_t)i * n + i];
    }
}

// Posterior of (f(x), grad f(x)) given the observations, for prior mean mu0 and gradient g0 at x.
struct Posterior {
    double mu, g[3];     // posterior mean of f(x) and of grad f(x)
    double var;          // posterior variance of f(x)
    double c[3];         // posterior covariance of grad f(x) with f(x)
    double Sgg[3][3];    // posterior covariance of grad f(x)
};

Posterior posterior_at(const Scene& S, const double x[3], double mu0, const double g0[3]) {
    const int n = S.n_obs;
    const double il2 = 1.0 / (S.l * S.l);
    // U: 4 x n covariances of (f(x), d f(x) / dx_a) with f(x_j)
    std::vector<double> U(4 * (size_t)n), Z;
    for (int j = 0; j < n; ++j) {
        const double* xj = &S.obs_x[3 * (size_t)j];
        const double k = se_kernel(S, x, xj);
        U[j] = k;
        for (int a = 0; a < 3; ++a) U[(size_t)(1 + a) * n + j] = -k * (x[a] - xj[a]) * il2;
    }
    Posterior P;
    P.mu = mu0;
    for (int a = 0; a < 3; ++a) P.g[a] = g0[a];
    for (int j = 0; j < n; ++j) {
        P.mu += U[j] * S.obs_alpha[j];
        for (int a = 0; a < 3; ++a) P.g[a] += U[(size_t)(1 + a) * n + j] * S.obs_alpha[j];
    }
    Z = U;
    for (int r = 0; r < 4; ++r) chol_solve(S.obs_L, n, &Z[(size_t)r * n]);
    double cov[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double v = r != c ? 0.0 : (r == 0 ? S.variance : S.variance * il2);
            for (int j = 0; j < n; ++j) v -= U[(size_t)r * n + j] * Z[(size_t)c * n + j];
            cov[r][c] = v;
        }
    P.var = cov[0][0];
    for (int a = 0; a < 3; ++a) {
        P.c[a] = cov[1 + a][0];
        for (int b = 0; b < 3; ++b) P.Sgg[a][b] = cov[1 + a][1 + b];
    }
    return P;
}

// Prior mean at x (mean function plus the trilinear offset grid).
double prior_mean(const Scene& S, const double x[3]) {
    double f, g[3];
    int which;
    mean_geom(S, x, f, g, which);
    if (!S.offset.empty()) {
        Tri t;
        trilinear(S.offset, S, x, t);
        for (int n = 0; n < 8; ++n) f += t.w[n] * S.offset.v[t.idx[n]];
    }
    return f;
}

// Projected area E[max(0, -d.g)] for g ~ N(G, Sigma) with a full covariance: -d.g is
// Gaussian with mean a = -d.G and variance d^T Sigma d.
double sigma_proj_cov(const double G[3], const double Sg[3][3], const double d[3]) {
    double v = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v += d[i] * Sg[i][j] * d[j];
    const double sd = std::sqrt(v);
    const double a = -dot3(d, G);
    return a * Phi_d(a / sd) + sd * phi_d(a / sd);
}

// Generalized NDF (Sec. 4.2.2) for g ~ N(G, Sigma) with a full covariance:
//   D(w) = int_0^inf r^3 N(r w; G, Sigma) dr.
// With A = w^T S^-1 w, B = w^T S^-1 G, C = G^T S^-1 G, b = B / sqrt(A), q = C - B^2/A the
// exponent is -(A/2)(r - B/A)^2 - q/2, and the moments of the truncated Gaussian give
//   D = [e^{-C/2} (b^2 + 2) + sqrt(2 pi) e^{-q/2} Phi(b) b (b^2 + 3)] / ((2 pi)^{3/2} |S|^{1/2} A^2).
double ndf_cov(const double G[3], const double Sg[3][3], const double w[3]) {
    const double det = Sg[0][0] * (Sg[1][1] * Sg[2][2] - Sg[1][2] * Sg[2][1]) -
                       Sg[0][1] * (Sg[1][0] * Sg[2][2] - Sg[1][2] * Sg[2][0]) +
                       Sg[0][2] * (Sg[1][0] * Sg[2][1] - Sg[1][1] * Sg[2][0]);
    double inv[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            // cofactor of (j, i) over the determinant
            const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            inv[i][j] = (Sg[r0][c0] * Sg[r1][c1] - Sg[r0][c1] * Sg[r1][c0]) / det;
        }
    auto quad = [&inv](const double u[3], const double v[3]) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) s += u[i] * inv[i][j] * v[j];
        return s;
    };
    const double A = quad(w, w), B = quad(w, G), C = quad(G, G);
    const double b = B / std::sqrt(A);
    const double q = std::max(C - B * B / A, 0.0);
    const double num = std::exp(-0.5 * C) * (b * b + 2.0) + kSqrt2Pi * std::exp(-0.5 * q) * Phi_d(b) * b * (b * b + 3.0);
    return num / (2.0 * kPi * kSqrt2Pi * std::sqrt(det) * A * A);
}

// ---------------------------------------------------------------------------
// GP statistics at a point (Sec. 3.1): f(x) ~ N(mu(x), sigma^2) and, independent of it
// at the same point (Eq. joint_fg), g(x) ~ N(grad mu(x), Sigma) with, for the
// squared-exponential kernel with lengthscale l across and l_n along the local
// mean-gradient direction n (Eq. se_kernel in that frame; n = z where grad mu = 0),
//   Sigma = (sigma / l)^2 (I - n n^T) + (sigma / l_n)^2 n n^T.
// ---------------------------------------------------------------------------
template <class T>
struct PointQ {
    T mu;
    T G[3];
    T sigma;
    T s;       // gradient standard deviation across n: sigma / l
    T sn;      // gradient standard deviation along n: sigma / l_n
    T albedo;
    bool ggx = false;   // GGX height-field macrofacet
    double f_eta = 0.0, f_k = 0.0;   // conductor Fresnel (eta = 0: none)
    // conditioned GP: G is the gradient mean given f(x) = 0 and cov its full covariance
    bool cond = false;
    double cov[3][3] = {};
};

template <class T>
struct Params {
    const Scene* S = nullptr;
    const std::unordered_map<int64_t, int>* node_slot = nullptr;
    int slot_var = -1, slot_l = -1, slot_alb = -1;
};

template <class T> inline T mk(double v, int slot);
template <> inline double mk<double>(double v, int) { return v; }
template <> inline Dual mk<Dual>(double v, int slot) { return Dual::var(v, slot); }

template <class T>
PointQ<T> eval_point(const Params<T>& P, const double x[3]) {
    const Scene& S = *P.S;
    PointQ<T> q;
    double f, g[3];
    int which;
    mean_geom(S, x, f, g, which);
    q.mu = T(f);
    for (int a = 0; a < 3; ++a) q.G[a] = T(g[a]);
    if (!S.offset.empty()) {
        Tri t;
        trilinear(S.offset, S, x, t);
        for (int n = 0; n < 8; ++n) {
            int slot = -1;
            if (P.node_slot) {
                auto it = P.node_slot->find(t.idx[n]);
                if (it != P.node_slot->end()) slot = it->second;
            }
            const T node = mk<T>(S.offset.v[t.idx[n]], slot);
            q.mu = q.mu + t.w[n] * node;
            for (int a = 0; a < 3; ++a) q.G[a] = q.G[a] + t.dw[n][a] * node;
        }
    }
    T variance;
    if (!S.var.empty()) {
        Tri t;
        trilinear(S.var, S, x, t);
        double v = 0.0;
        for (int n = 0; n < 8; ++n) v += t.w[n] * S.var.v[t.idx[n]];
        variance = T(v);
    } else {
        variance = mk<T>(S.variance, P.slot_var);
    }
    q.sigma = t_sqrt(variance);
    q.s = q.sigma / mk<T>(S.l, P.slot_l);
    q.sn = S.aniso ? q.sigma / T(S.l_n) : q.s;
    q.ggx = S.ggx;
    q.f_eta = S.f_eta;
    q.f_k = S.f_k;
    if (S.albedo_per_prim && which >= 0) q.albedo = T(S.prims[which].albedo);
    else q.albedo = mk<T>(S.albedo, P.slot_alb);
    if (S.cond) {
        // Conditioned GP: density from f(x) ~ N(mu_C, var_C); gradient distribution given
        // f(x) = 0 (the surface), by the same Gaussian conditioning applied to the posterior
        // pair (f(x), grad f(x)):  mean g_C - c mu_C / var_C, covariance Sgg - c c^T / var_C.
        const double g0[3] = {val(q.G[0]), val(q.G[1]), val(q.G[2])};
        const Posterior Q = posterior_at(S, x, val(q.mu), g0);
        q.cond = true;
        q.mu = T(Q.mu);
        q.sigma = T(std::sqrt(Q.var));
        double tr = 0.0;
        for (int a = 0; a < 3; ++a) {
            q.G[a] = T(Q.g[a] - Q.c[a] * Q.mu / Q.var);
            for (int b = 0; b < 3; ++b) q.cov[a][b] = Q.Sgg[a][b] - Q.c[a] * Q.c[b] / Q.var;
            tr += q.cov[a][a];
        }
        // isotropic gradient spread of the same total variance, used by the proposal only
        q.s = T(std::sqrt(tr / 3.0));
        q.sn = q.s;
    }
    return q;
}

// Density (Sec. 3.2 Eq. h_density with the height mapped to the SDF value, Sec. 4):
// rho = phi(f; 0, sigma^2) / Phi(f; 0, sigma^2) evaluated at the mean mu(x).
template <class T>
T rho_of(const T& mu, const T& sigma) {
    const T z = mu / sigma;
    if (val(z) > -30.0) {
        const T ph = t_exp(-0.5 * z * z) / (kSqrt2Pi * sigma);
        const T Ph = 0.5 * t_erfc(-z / kSqrt2);
        return ph / Ph;
    }
    // far tail: the same ratio written with erfcx so that Phi does not underflow
    return std::sqrt(2.0 / kPi) / (sigma * t_erfcx(-z / kSqrt2));
}

// Eq. generalized_lambda times cos(theta): the projected area of Eq. generalized_sigma_t in
// the frame of the geometric normal, for a direction with cos(theta) = c and squared
// tangent components tx2 = sin^2 cos^2 phi, ty2 = sin^2 sin^2 phi.
//   Lambda(a) c = c e^{-a^2}/(2 a sqrt(pi)) + (erf(a) - 1) c / 2,  a = c / den,
// written with c / a = den and erf(a) - 1 = -erfc(a).
template <class T>
T lambda_cos_general(const T& ax, const T& ay, const T& az, const T& c, const T& tx2, const T& ty2) {
    const T den = t_sqrt(ax * ax * tx2 + ay * ay * ty2 + az * az * c * c);
    const T a = c / den;
    return den * t_exp(-a * a) / (2.0 * kSqrtPi) - 0.5 * t_erfc(a) * c;
}

// Eq. macro_ndf (Appendix A), in the frame of the geometric normal, for a normal with
// cos(theta_m) = c and squared tangent components tx2, ty2.
template <class T>
T ndf_general(const T& ax, const T& ay, const T& az, const T& c, const T& tx2, const T& ty2) {
    const T A = tx2 / (ax * ax) + ty2 / (ay * ay) + c * c / (az * az);
    const T B = c / (az * az);
    const T C = 1.0 / (az * az);
    const T BA = B * B / A;
    const T pre = t_exp(-C + BA) / (kPi * kSqrtPi * ax * ay * az);
    const T t1 = (1.0 / (2.0 * A * A)) * (BA + 1.0) * t_exp(-BA);
    const T t2 = B * kSqrtPi / (2.0 * A * A * t_sqrt(A)) * (BA + 1.5) * t_erfc(-B / t_sqrt(A));
    return pre * (t1 + t2);
}

// Projected area for travel direction d at a point whose gradient is g ~ N(G, Sigma):
// the paper's Lambda(w) cos(theta) (Eq. generalized_lambda) about the local geometric
// normal n = G/|G| with roughnesses alpha_x = alpha_y = sqrt(2) s / |G| and
// alpha_z = sqrt(2) s_n / |G| (Eq. roughness), scaled by |G|, the length of the mean
// gradient.  Where grad mu = 0: E[max(0, -d.g)] = s_d / sqrt(2 pi), s_d^2 = d^T Sigma d.
// GGX height-field macrofacet (end of Sec. 4.1: any NDF may replace Beckmann under the
// Smith assumption).  About n = G/|G| with roughness alpha = sqrt(2) s / |G| (Eq. roughness)
// and scaled by |G| as the generalized forms are:
//   D(wm) = alpha^2 / (pi ((n.wm)^2 (alpha^2 - 1) + 1)^2) for n.wm > 0 (0 below),
//   sigma(d) = Lambda(w) cos(theta) over the microsurface, w = -d, cos = w.n of either sign:
//     cos (1 + Lambda(w)) entering from above, |cos| Lambda(-w) from below,
//     Lambda = (-1 + sqrt(1 + alpha^2 tan^2)) / 2,
//   which is (cos + sqrt(cos^2 + alpha^2 (1 - cos^2))) / 2 for both signs.
template <class T>
T ggx_lambda_cos(const T& alpha, const T& c) {
    const T e = alpha * alpha * (1.0 - c * c);
    const T r = t_sqrt(c * c + e);
    // (c + r) / 2; for c < 0 (from below) the same value as e / (2 (r - c)), free of cancellation
    return val(c) < 0.0 ? 0.5 * e / (r - c) : 0.5 * (c + r);
}
template <class T>
T ggx_D(const T& alpha, const T& c) {
    if (val(c) <= 0.0) return T(0.0);
    const T den = c * c * (alpha * alpha - 1.0) + 1.0;
    return alpha * alpha / (kPi * den * den);
}

template <class T>
T sigma_proj(const PointQ<T>& q, const double d[3]) {
    if (q.cond) {
        const double G[3] = {val(q.G[0]), val(q.G[1]), val(q.G[2])};
        return T(sigma_proj_cov(G, q.cov, d));
    }
    const T g2 = q.G[0] * q.G[0] + q.G[1] * q.G[1] + q.G[2] * q.G[2];
    if (q.ggx) {
        if (val(g2) == 0.0) return T(0.0);
        const T gn = t_sqrt(g2);
        const T c = -(q.G[0] * d[0] + q.G[1] * d[1] + q.G[2] * d[2]) / gn;
        return gn * ggx_lambda_cos(kSqrt2 * q.s / gn, c);
    }
    if (val(g2) == 0.0) {
        const T sd = t_sqrt(q.s * q.s * (1.0 - d[2] * d[2]) + q.sn * q.sn * (d[2] * d[2]));
        return sd / kSqrt2Pi;
    }
    const T gn = t_sqrt(g2);
    const T c = (q.G[0] * d[0] + q.G[1] * d[1] + q.G[2] * d[2]) / gn;
    const T alpha = kSqrt2 * q.s / gn, alpha_n = kSqrt2 * q.sn / gn;
    return gn * lambda_cos_general(alpha, alpha, alpha_n, c, 1.0 - c * c, T(0.0));
}

// Generalized NDF at normal wm for g ~ N(G, Sigma): Eq. macro_ndf with
// alpha_x = alpha_y = sqrt(2) s / |G|, alpha_z = sqrt(2) s_n / |G| about n = G/|G|, scaled
// by |G|.  Where grad mu = 0 (the B = C = 0 limit, n = z):
//   D = 2 / ((2 pi)^(3/2) s^2 s_n A^2),  A = (1 - c^2) / s^2 + c^2 / s_n^2,  c = wm_z.
template <class T>
T ndf(const PointQ<T>& q, const double wm[3]) {
    if (q.cond) {
        const double G[3] = {val(q.G[0]), val(q.G[1]), val(q.G[2])};
        return T(ndf_cov(G, q.cov, wm));
    }
    const T g2 = q.G[0] * q.G[0] + q.G[1] * q.G[1] + q.G[2] * q.G[2];
    if (q.ggx) {
        if (val(g2) == 0.0) return T(0.0);
        const T gn = t_sqrt(g2);
        const T c = (q.G[0] * wm[0] + q.G[1] * wm[1] + q.G[2] * wm[2]) / gn;
        return gn * ggx_D(kSqrt2 * q.s / gn, c);
    }
    if (val(g2) == 0.0) {
        const double c2 = wm[2] * wm[2];
        const T A = (1.0 - c2) / (q.s * q.s) + c2 / (q.sn * q.sn);
        return 2.0 / (2.0 * kPi * kSqrt2Pi * q.s * q.s * q.sn * A * A);
    }
    const T gn = t_sqrt(g2);
    const T c = (q.G[0] * wm[0] + q.G[1] * wm[1] + q.G[2] * wm[2]) / gn;
    const T alpha = kSqrt2 * q.s / gn, alpha_n = kSqrt2 * q.sn / gn;
    return gn * ndf_general(alpha, alpha, alpha_n, c, 1.0 - c * c, T(0.0));
}

// Beckmann NDF and Smith Lambda (the height-field limit used by the proposal).
double beckmann_D(double alpha, double cos_m, double sin2_m) {
    if (cos_m <= 0.0) return 0.0;
    const double c2 = cos_m * cos_m;
    return std::exp(-sin2_m / (c2 * alpha * alpha)) / (kPi * alpha * alpha * c2 * c2);
}
double beckmann_lambda(double a) {
    if (std::isinf(a)) return 0.0;
    return 0.5 * (std::exp(-a * a) / (a * kSqrtPi) - std::erfc(a));
}

// ---------------------------------------------------------------------------
// Proposal over half vectors (end of Sec. 4.2.2): with probability R the Beckmann
// distribution of visible normals (Heitz and d'Eon 2014, slope-space inversion) for
// alpha_B = sqrt(2) s / |G| about G/|G|; otherwise uniform over the hemisphere about
// v = -d.  The Beckmann part is used only while v is above the local horizon.
// ---------------------------------------------------------------------------
struct Proposal {
    bool beck;          // visible-normal component available (Beckmann, or GGX for a GGX macrofacet)
    bool ggx;
    double Reff;
    double N[3], T[3], B[3];
    double alpha, cosv, a;  // a = cot(theta_v) in the stretched configuration
};

Proposal make_proposal(const PointQ<double>& q, double R, const double v[3]) {
    Proposal p;
    const double gn = std::sqrt(dot3(q.G, q.G));
    p.beck = false;
    p.ggx = q.ggx;
    p.Reff = 0.0;
    if (gn > 0.0) {
        p.N[0] = q.G[0] / gn; p.N[1] = q.G[1] / gn; p.N[2] = q.G[2] / gn;
        p.cosv = dot3(v, p.N);
        if (p.cosv > 0.0) {
            p.beck = true;
            p.Reff = R;
            p.alpha = kSqrt2 * q.s / gn;
            double vt[3] = {v[0] - p.cosv * p.N[0], v[1] - p.cosv * p.N[1], v[2] - p.cosv * p.N[2]};
            const double st = std::sqrt(dot3(vt, vt));
            if (st > 1e-7) {
                p.T[0] = vt[0] / st; p.T[1] = vt[1] / st; p.T[2] = vt[2] / st;
                p.a = p.cosv / (p.alpha * st);
            } else {
                double b[3];
                onb(p.N, p.T, b);
                p.a = INFINITY;
            }
            cross3(p.N, p.T, p.B);
        }
    }
    return p;
}

double beckmann_vndf_pdf(const Proposal& p, const double v[3], const double wm[3]) {
    if (!p.beck) return 0.0;
    const double cm = dot3(wm, p.N);
    if (cm <= 0.0) return 0.0;
    if (p.ggx) {   // GGX visible normals: <v, wm> D(wm) / (cos_v (1 + Lambda(v)))
        const double vm = std::max(0.0, dot3(v, wm));
        return vm * ggx_D(p.alpha, cm) / ggx_lambda_cos(p.alpha, p.cosv);
    }
    double cr[3];
    cross3(wm, p.N, cr);
    const double D = beckmann_D(p.alpha, cm, dot3(cr, cr));
    const double vm = std::max(0.0, dot3(v, wm));
    return vm * D / ((1.0 + beckmann_lambda(p.a)) * p.cosv);
}

double mixture_pdf(const Proposal& p, const double v[3], const double wm[3]) {
    if (dot3(v, wm) <= 0.0) return 0.0;  // both components live on the hemisphere about v
    return p.Reff * beckmann_vndf_pdf(p, v, wm) + (1.0 - p.Reff) / (2.0 * kPi);
}

// Slope along the incidence plane for alpha = 1: solve F(x) = u F(a) on (-8, a] with
//   F(x) = erfc(-x)/2 + exp(-x^2)/(2 a sqrt(pi)),
// the unnormalized CDF of (1 - x/a)^+ exp(-x^2)/sqrt(pi).
double sample_slope_x(double a, double u) {
    const bool fin = !std::isinf(a);
    auto F = [a, fin](double x) {
        return 0.5 * std::erfc(-x) + (fin ? std::exp(-x * x) / (2.0 * a * kSqrtPi) : 0.0);
    };
    const double Fa = fin ? F(a) : 1.0;
    const double target = u * Fa;
    double lo = -8.0, hi = fin ? std::min(a, 8.0) : 8.0;
    if (target <= F(lo)) return lo;
    double x = std::min(std::max(0.0, lo), hi);
    for (int it = 0; it < 200; ++it) {
        const double fx = F(x) - target;
        if (fx == 0.0) break;
        if (fx > 0.0) hi = x; else lo = x;
        const double fp = std::exp(-x * x) / kSqrtPi * (fin ? (1.0 - x / a) : 1.0);
        double xn = (fp > 0.0) ? x - fx / fp : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const double step = xn - x;
        x = xn;
        if (std::fabs(step) <= 1e-15 * std::max(1.0, std::fabs(x))) break;
        if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(x))) break;
    }
    return x;
}

// Half vector from the selection uniform and two 24-bit uniforms.
void sample_half_vector(const Proposal& p, const double v[3], double u_sel, uint32_t ua24,
                        uint32_t ub24, double wm[3]) {
    const double ua = ua24 * 0x1p-24, ub = ub24 * 0x1p-24;
    if (u_sel < p.Reff && p.ggx) {
        // GGX visible normals (Heitz 2018): stretch v to the alpha = 1 configuration, sample
        // the projected hemisphere as a disk whose far half is foreshortened by the view,
        // lift the point to the hemisphere and unstretch.  Local frame (T, B, N).
        const double vx = dot3(v, p.T), vy = dot3(v, p.B), vz = p.cosv;
        double h[3] = {p.alpha * vx, p.alpha * vy, vz};
        const double hn = std::sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
        for (double& c : h) c /= hn;
        const double l2 = h[0] * h[0] + h[1] * h[1];
        double t1[3] = {1.0, 0.0, 0.0};
        if (l2 > 0.0) {
            const double il = 1.0 / std::sqrt(l2);
            t1[0] = -h[1] * il; t1[1] = h[0] * il; t1[2] = 0.0;
        }
        double t2[3];
        cross3(h, t1, t2);
        const double r = std::sqrt(ua), phi = 2.0 * kPi * ub;
        const double a1 = r * std::cos(phi);
        double a2 = r * std::sin(phi);
        const double sh = 0.5 * (1.0 + h[2]);
        a2 = (1.0 - sh) * std::sqrt(std::max(0.0, 1.0 - a1 * a1)) + sh * a2;
        const double a3 = std::sqrt(std::max(0.0, 1.0 - a1 * a1 - a2 * a2));
        double m[3];
        for (int k = 0; k < 3; ++k) m[k] = a1 * t1[k] + a2 * t2[k] + a3 * h[k];
        double e[3] = {p.alpha * m[0], p.alpha * m[1], std::max(0.0, m[2])};
        const double en = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        for (int k = 0; k < 3; ++k) wm[k] = (e[0] * p.T[k] + e[1] * p.B[k] + e[2] * p.N[k]) / en;
    } else if (u_sel < p.Reff) {
        const double xs = sample_slope_x(p.a, ua);
        const double ys = erfinv_d((2.0 * ub24 + 1.0) * 0x1p-24 - 1.0);
        const double x = p.alpha * xs, y = p.alpha * ys;
        const double n = std::sqrt(x * x + y * y + 1.0);
        for (int k = 0; k < 3; ++k) wm[k] = (-x * p.T[k] - y * p.B[k] + p.N[k]) / n;
    } else {
        double t[3], b[3];
        onb(v, t, b);
        const double ct = 1.0 - ua;
        const double st = std::sqrt(ua * (2.0 - ua));
        const double ph = 2.0 * kPi * ub;
        const double cp = std::cos(ph), sp = std::sin(ph);
        for (int k = 0; k < 3; ++k) wm[k] = st * cp * t[k] + st * sp * b[k] + ct * v[k];
    }
}

// ---------------------------------------------------------------------------
// Majorant grid: per cell an upper bound of sigma_t = rho * sigma_proj over the cell and
// all directions, rounded up to 5 significant bits so that independent double
// evaluations agree exactly.
//   rho(mu, sigma) = (1/sigma) r(mu/sigma), r = phi/Phi decreasing (Fig. monotonic_density)
//   sigma_proj <= E[max(0, X)], X ~ N(|G|max, smax^2) = g Phi(g/s) + s phi(g/s)
// ---------------------------------------------------------------------------
double r_ratio(double z) { return std::sqrt(2.0 / kPi) / erfcx_d(-z / kSqrt2); }

double quantize_majorant(double B) {
    if (std::isnan(B)) return INFINITY;
    const double Bp = B * (1.0 + 0x1p-10);
    if (!(Bp >= 0x1p-40)) return 0.0;
    if (std::isinf(Bp)) return INFINITY;
    int e;
    const double f = std::frexp(Bp, &e);
    const double m = std::ceil(f * 32.0);
    return std::ldexp(m, e - 5);
}

void node_range(int k, int M, int R, int& lo, int& hi) {
    lo = (int)(((int64_t)k * (R - 1)) / M);
    hi = (int)((((int64_t)(k + 1)) * (R - 1) + M - 1) / M);
    if (lo < 0) lo = 0;
    if (hi > R - 1) hi = R - 1;
}

// Where the prior mean is smooth over cell k (cell centre c, half diagonal h): its gradient
// at c and a bound H on the norm of its Hessian over the cell.  Plane and constant means
// have H = 0.  A mean of signed-distance primitives qualifies when one sphere is the
// minimum over the whole cell (its distance at c plus h stays below every other
// primitive's minus h, the distances being 1-Lipschitz) and its centre p lies outside the
// cell: the Hessian of |x - p| - R is (I - n n^T) / |x - p|, of norm 1 / |x - p|.
bool prior_smooth_on_cell(const Scene& S, const int k[3], const double cwv[3], double h, double g[3], double& H) {
    g[0] = g[1] = g[2] = 0.0;
    H = 0.0;
    if (S.mean_kind == 0) { g[2] = 1.0; return true; }
    if (S.mean_kind == 2) return true;
    double c[3];
    for (int a = 0; a < 3; ++a) c[a] = S.lo[a] + (k[a] + 0.5) * cwv[a];
    int best = -1;
    double fb = INFINITY, f2 = INFINITY;
    for (size_t i = 0; i < S.prims.size(); ++i) {
        double f, gi[3];
        sdf_prim(S.prims[i], c, f, gi);
        if (f < fb) { f2 = fb; fb = f; best = (int)i; g[0] = gi[0]; g[1] = gi[1]; g[2] = gi[2]; }
        else f2 = std::min(f2, f);
    }
    if (best < 0 || S.prims[best].kind != 0 || !(fb + h < f2 - h)) return false;
    double d2 = 0.0;   // squared distance from the sphere's centre to the cell
    for (int a = 0; a < 3; ++a) {
        const double c0 = S.lo[a] + k[a] * cwv[a], c1 = S.lo[a] + (k[a] + 1) * cwv[a];
        const double p = S.prims[best].c[a];
        const double d = p < c0 ? c0 - p : (p > c1 ? p - c1 : 0.0);
        d2 += d * d;
    }
    if (!(d2 > 0.0)) return false;
    H = 1.0 / std::sqrt(d2);
    return true;
}

// Bound for the conditioned GP (scalar prior variance s^2, isotropic kernel) over cell k
// (centre c, half extents e_a = cw_a / 2, half diagonal h), given the prior mean's minimum
// mu_min and gradient bound gmax over the cell.  With d_j the distances from observation j to
// the cell (nearest dmin_j, farthest dmax_j), kappa(d) = s^2 e^{-d^2/(2l^2)} and the
// posterior at c (mean mu_C(c), mean gradient grad mu_C(c), standard deviation s_C(c)):
//   mean:   mu_C >= mu_min + sum_j alpha_j kappa(d), taken at dmax_j for alpha_j > 0 and at
//           dmin_j otherwise;
//   slope:  |grad mu_C| <= G1 = gmax + sum_j |alpha_j| (s^2/l^2) d e^{-d^2/(2l^2)},
//           d = clamp(l, dmin_j, dmax_j) (the maximum of that profile over [dmin_j, dmax_j]);
//           where the prior mean is smooth on the cell (prior_smooth_on_cell, Hessian norm
//           at most H0) also |grad mu_C| <= Gb = |grad mu_C(c)| + h Hb with
//           Hb = H0 + sum_j |alpha_j| (s^2/l^2) e^{-dmin_j^2/(2l^2)} max(1, dmax_j^2/l^2 - 1)
//           (the Hessian of kappa(x - x_j) has eigenvalues (s^2/l^2) e^{-r^2/(2l^2)} times
//           r^2/l^2 - 1 and -1), and by Taylor's theorem
//           mu_C >= mu_C(c) - sum_a e_a |d mu_C(c) / dx_a| - Hb h^2 / 2;
//           G is the smaller slope bound, and mu_C >= mu_C(c) - h G in any case;
//   spread: s_C <= s (conditioning never adds variance); writing f(x_j) = r_j f(x) + e_j with
//           e_j independent of f(x) and the observation noise at least s_n^2 I,
//           1/s_C^2 <= 1/s^2 + sum_j r_j^2 / s_n^2, r_j^2 = e^{-d_j^2/l^2} <= e^{-dmin_j^2/l^2};
//           grad s_C = cov(grad f, f) / s_C has length at most s / l (Cauchy-Schwarz), so
//           s_C(c) - h s/l <= s_C <= s_C(c) + h s/l;
//   each of mu_lo, s_lo is the largest of its lower bounds, s_up the smaller upper bound.
// The gradient given f = 0 is N(m, Sigma) with Sigma <= (s/l)^2 I and |m| <= G + (s/l) |z|,
// z = mu_C / s_C (Cauchy-Schwarz again), so with sd = s/l and
// F(M, sd) = sd phi(M/sd) + M Phi(M/sd), increasing in both arguments and 1-Lipschitz in M,
//   sigma_proj <= F(G + sd |z|, sd),   rho = r(z) / s_C <= r(z) / s_lo,  r = phi/Phi decreasing,
// and z >= z_lo = mu_lo / (mu_lo > 0 ? s_up : s_lo).  Over z in [z_lo, 0) the product is at
// most r(z_lo) F(G + sd |z_lo|, sd) / s_lo; over z >= z0 = max(z_lo, 0) at most
// (r(z0) F(G, sd) + sd sup_{z >= z0} z r(z)) / s_lo, where z r(z) peaks at 0.29453 (z = 0.84)
// and decreases beyond, so the supremum is z0 r(z0) for z0 >= 0.9 and 0.2946 otherwise.
double cond_bound(const Scene& S, const int k[3], const double cwv[3], double mu_min, double gmax) {
    const double l = S.l, s2 = S.variance;
    double mu_c = 0.0, g_c = 0.0, prec = 1.0 / s2, hb = 0.0;
    for (int j = 0; j < S.n_obs; ++j) {
        const double* xj = &S.obs_x[3 * (size_t)j];
        double dn2 = 0.0, df2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double c0 = S.lo[a] + k[a] * cwv[a], c1 = S.lo[a] + (k[a] + 1) * cwv[a];
            const double dn = xj[a] < c0 ? c0 - xj[a] : (xj[a] > c1 ? xj[a] - c1 : 0.0);
            const double df = std::max(std::fabs(xj[a] - c0), std::fabs(xj[a] - c1));
            dn2 += dn * dn;
            df2 += df * df;
        }
        const double dmin = std::sqrt(dn2), dmax = std::sqrt(df2);
        const double al = S.obs_alpha[j];
        mu_c += al * s2 * std::exp(-(al > 0.0 ? df2 : dn2) / (2.0 * l * l));
        const double dd = std::min(std::max(l, dmin), dmax);
        g_c += std::fabs(al) * (s2 / (l * l)) * dd * std::exp(-dd * dd / (2.0 * l * l));
        prec += std::exp(-dn2 / (l * l)) / S.obs_noise;
        hb += std::fabs(al) * (s2 / (l * l)) * std::exp(-dn2 / (2.0 * l * l)) * std::max(1.0, df2 / (l * l) - 1.0);
    }
    const double s_hi = std::sqrt(s2), sl = s_hi / l;
    double c[3], g0[3], H0;
    for (int a = 0; a < 3; ++a) c[a] = S.lo[a] + (k[a] + 0.5) * cwv[a];
    const double hdiag = 0.5 * std::sqrt(cwv[0] * cwv[0] + cwv[1] * cwv[1] + cwv[2] * cwv[2]);
    const bool smooth = prior_smooth_on_cell(S, k, cwv, hdiag, g0, H0);
    const Posterior P = posterior_at(S, c, prior_mean(S, c), g0);
    double G = gmax + g_c;
    double mu_lo = mu_min + mu_c;
    if (smooth) {
        const double Hb = H0 + hb;
        G = std::min(G, std::sqrt(dot3(P.g, P.g)) + hdiag * Hb);
        double lin = 0.0;
        for (int a = 0; a < 3; ++a) lin += 0.5 * cwv[a] * std::fabs(P.g[a]);
        mu_lo = std::max(mu_lo, P.mu - lin - 0.5 * Hb * hdiag * hdiag);
    }
    mu_lo = std::max(mu_lo, P.mu - hdiag * G);
    const double s_c = std::sqrt(std::max(P.var, 0.0));
    const double s_lo = std::max(1.0 / std::sqrt(prec), s_c - hdiag * sl);
    const double s_up = std::min(s_hi, s_c + hdiag * sl);
    const double z_lo = mu_lo / (mu_lo > 0.0 ? s_up : s_lo);
    auto F = [&](double M) { return sl * phi_d(M / sl) + M * Phi_d(M / sl); };
    const double neg = r_ratio(z_lo) * F(G + sl * std::max(0.0, -z_lo));
    const double z0 = std::max(z_lo, 0.0);
    const double pos = r_ratio(z0) * F(G) + sl * (z0 >= 0.9 ? z0 * r_ratio(z0) : 0.2946);
    return std::max(neg, pos) / s_lo;
}

void build_majorants(Scene& S) {
    const int64_t n = (int64_t)S.M[0] * S.M[1] * S.M[2];
    S.maj.assign(n, 0.0);
    double cwv[3];
    for (int a = 0; a < 3; ++a) cwv[a] = S.ext[a] / S.M[a];
#pragma omp parallel for schedule(dynamic, 1)
    for (int kz = 0; kz < S.M[2]; ++kz)
        for (int ky = 0; ky < S.M[1]; ++ky)
            for (int kx = 0; kx < S.M[0]; ++kx) {
                const int k[3] = {kx, ky, kz};
                // offset grid: minimum and gradient bound over the nodes that reach the cell
                double off_min = 0.0, off_g = 0.0;
                if (!S.offset.empty()) {
                    int lo[3], hi[3];
                    for (int a = 0; a < 3; ++a) node_range(k[a], S.M[a], S.offset.res[a], lo[a], hi[a]);
                    off_min = INFINITY;
                    double md[3] = {0, 0, 0};
                    const int* r = S.offset.res;
                    for (int z = lo[2]; z <= hi[2]; ++z)
                        for (int y = lo[1]; y <= hi[1]; ++y)
                            for (int x = lo[0]; x <= hi[0]; ++x) {
                                const double v = S.offset.v[((int64_t)z * r[1] + y) * r[0] + x];
                                off_min = std::min(off_min, v);
                                if (x < hi[0]) md[0] = std::max(md[0], std::fabs(S.offset.v[((int64_t)z * r[1] + y) * r[0] + x + 1] - v));
                                if (y < hi[1]) md[1] = std::max(md[1], std::fabs(S.offset.v[((int64_t)z * r[1] + y + 1) * r[0] + x] - v));
                                if (z < hi[2]) md[2] = std::max(md[2], std::fabs(S.offset.v[((int64_t)(z + 1) * r[1] + y) * r[0] + x] - v));
                            }
                    double gs = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        const double g = md[a] / (S.ext[a] / (S.offset.res[a] - 1));
                        gs += g * g;
                    }
                    off_g = std::sqrt(gs);
                }
                double vmin = S.variance, vmax = S.variance;
                if (!S.var.empty()) {
                    int lo[3], hi[3];
                    for (int a = 0; a < 3; ++a) node_range(k[a], S.M[a], S.var.res[a], lo[a], hi[a]);
                    vmin = INFINITY; vmax = -INFINITY;
                    const int* r = S.var.res;
                    for (int z = lo[2]; z <= hi[2]; ++z)
                        for (int y = lo[1]; y <= hi[1]; ++y)
                            for (int x = lo[0]; x <= hi[0]; ++x) {
                                const double v = S.var.v[((int64_t)z * r[1] + y) * r[0] + x];
                                vmin = std::min(vmin, v);
                                vmax = std::max(vmax, v);
                            }
                }
                double mu_min, gmax;
                if (S.mean_kind == 0) {
                    mu_min = S.lo[2] + k[2] * cwv[2];
                    gmax = 1.0;
                } else if (S.mean_kind == 2) {
                    mu_min = S.mean_const;
                    gmax = 0.0;
                } else {
                    // the union's minimum over the cell: the smallest primitive bound
                    double blo[3], bhi[3];
                    for (int a = 0; a < 3; ++a) {
                        blo[a] = S.lo[a] + k[a] * cwv[a];
                        bhi[a] = S.lo[a] + (k[a] + 1) * cwv[a];
                    }
                    mu_min = INFINITY;
                    for (const Prim& p : S.prims) mu_min = std::min(mu_min, sdf_prim_min(p, blo, bhi));
                    gmax = 1.0;
                }
                mu_min += off_min;
                gmax += off_g;
                if (S.cond) {
                    S.maj[((int64_t)kz * S.M[1] + ky) * S.M[0] + kx] = quantize_majorant(cond_bound(S, k, cwv, mu_min, gmax));
                    continue;
                }
                const double smin_f = std::sqrt(vmin), smax_f = std::sqrt(vmax);
                const double s_max = smax_f / std::min(S.l, S.l_n);
                const double rho_max = r_ratio(mu_min / (mu_min > 0.0 ? smax_f : smin_f)) / smin_f;
                const double z = gmax / s_max;
                // GGX height field: sigma <= (|G| + sqrt(|G|^2 + 2 s^2)) / 2
                const double proj_max = S.ggx ? 0.5 * (gmax + std::sqrt(gmax * gmax + 2.0 * s_max * s_max))
                                              : gmax * Phi_d(z) + s_max * phi_d(z);
                S.maj[((int64_t)kz * S.M[1] + ky) * S.M[0] + kx] = quantize_majorant(rho_max * proj_max);
            }
}

// ---------------------------------------------------------------------------
// Ray / box and majorant-grid traversal.
// ---------------------------------------------------------------------------
bool clip_box(const Scene& S, const double o[3], const double d[3], double& t0, double& t1) {
    t0 = 0.0;
    t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < S.lo[a] || o[a] > S.hi[a]) return false;
            continue;
        }
        double ta = (S.lo[a] - o[a]) / d[a];
        double tb = (S.hi[a] - o[a]) / d[a];
        if (ta > tb) std::swap(ta, tb);
        t0 = std::max(t0, ta);
        t1 = std::min(t1, tb);
    }
    return t0 < t1;
}

struct Walker {
    const Scene* S;
    const double* o;
    const double* d;
    int idx[3];
    void init(double t) {
        for (int a = 0; a < 3; ++a) {
            const double p = o[a] + t * d[a];
            int i = (int)std::floor((p - S->lo[a]) / S->cw[a]);
            idx[a] = std::min(std::max(i, 0), S->M[a] - 1);
        }
    }
    double majorant() const { return S->maj[((int64_t)idx[2] * S->M[1] + idx[1]) * S->M[0] + idx[0]]; }
    // distance at which the ray leaves the current cell, and the axis it leaves through
    double exit(int& ax) const {
        double best = INFINITY;
        ax = 0;
        for (int a = 0; a < 3; ++a) {
            double tn = INFINITY;
            if (d[a] > 0.0) tn = (S->lo[a] + (idx[a] + 1) * S->cw[a] - o[a]) / d[a];
            else if (d[a] < 0.0) tn = (S->lo[a] + idx[a] * S->cw[a] - o[a]) / d[a];
            if (tn < best) { best = tn; ax = a; }
        }
        return best;
    }
    bool step(int ax) {
        idx[ax] += d[ax] > 0.0 ? 1 : -1;
        return idx[ax] >= 0 && idx[ax] < S->M[ax];
    }
};

constexpr int64_t kStepCap = 1 << 16;
// Russian roulette on shadow-ray transmittance (as in the null-scattering path tracer of
// the paper's implementation platform): below kRRThreshold the estimate survives with
// probability 1/2 and is doubled.
constexpr double kRRThreshold = 0.0625;

template <class T>
T sigma_t_of(const PointQ<T>& q, const double d[3]) { return rho_of(q.mu, q.sigma) * sigma_proj(q, d); }

enum TrackResult { kEscape = 0, kCollide = 1, kAbsorbed = 2 };

// Delta tracking (null-scattering, Sec. 5) of one segment [t0, t1] through the majorant
// grid.  Per tentative collision: optical depth tau = -ln(1 - u1) consumed cell by cell,
// then real iff u2 * majorant < sigma_t.  With `frozen`, decisions use P0 and the
// returned factor wfac carries the weight ratio of P1 to P0 (null: (m - st1)/(m - st0),
// real: st1/st0).
template <class T>
int delta_track(const Params<double>& P0, const Params<T>& P1, bool frozen, const double o[3],
                const double d[3], double t0, double t1, Rng& rng, double& t_hit, T& wfac,
                Counters& C) {
    Walker w{P0.S, o, d, {0, 0, 0}};
    w.init(t0);
    double t = t0;
    double tau = -std::log(1.0 - rng.uniform());
    int64_t steps = 0;
    C.c[ORC_C_CELLS]++;
    for (;;) {
        int ax;
        const double tn = w.exit(ax);
        const double tc = std::min(tn, t1);
        const double maj = w.majorant();
        const double seg = std::max(0.0, tc - t);
        if (maj > 0.0 && tau < maj * seg) {
            t += tau / maj;
            const double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
            C.c[ORC_C_TRACK_STEPS]++;
            if (++steps > kStepCap) { C.c[ORC_C_CAPPED]++; return kAbsorbed; }
            const double u2 = rng.uniform();
            const PointQ<double> q0 = eval_point(P0, x);
            const double st0 = sigma_t_of(q0, d);
            if (st0 > maj) C.c[ORC_C_VIOLATIONS]++;
            if (u2 * maj < st0) {
                if (frozen) {
                    const PointQ<T> q1 = eval_point(P1, x);
                    wfac = wfac * (sigma_t_of(q1, d) / st0);
                }
                t_hit = t;
                return kCollide;
            }
            if (frozen) {
                const PointQ<T> q1 = eval_point(P1, x);
                wfac = wfac * ((maj - sigma_t_of(q1, d)) / (maj - st0));
            }
            tau = -std::log(1.0 - rng.uniform());
            continue;
        }
        if (maj > 0.0) tau -= maj * seg;
        t = tc;
        if (tn >= t1) return kEscape;
        if (!w.step(ax)) return kEscape;
        C.c[ORC_C_CELLS]++;
    }
}

// Ratio tracking transmittance along [0, t1]: product of (1 - sigma_t / majorant) over
// tentative collisions (one uniform each for the free flight), with Russian roulette once
// the product falls below kRRThreshold (one more uniform).
template <class T>
T ratio_track(const Params<double>& P0, const Params<T>& P1, bool frozen, const double o[3],
              const double d[3], double t1, Rng& rng, Counters& C) {
    Walker w{P0.S, o, d, {0, 0, 0}};
    w.init(0.0);
    double t = 0.0;
    double Tr0 = 1.0;
    T Tr1 = T(1.0);
    double tau = -std::log(1.0 - rng.uniform());
    int64_t steps = 0;
    C.c[ORC_C_CELLS]++;
    for (;;) {
        int ax;
        const double tn = w.exit(ax);
        const double tc = std::min(tn, t1);
        const double maj = w.majorant();
        const double seg = std::max(0.0, tc - t);
        if (maj > 0.0 && tau < maj * seg) {
            t += tau / maj;
            const double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
            C.c[ORC_C_NEE_STEPS]++;
            if (++steps > kStepCap) { C.c[ORC_C_CAPPED]++; return T(0.0); }
            const PointQ<double> q0 = eval_point(P0, x);
            const double st0 = sigma_t_of(q0, d);
            if (st0 > maj) C.c[ORC_C_VIOLATIONS]++;
            Tr0 *= (1.0 - st0 / maj);
            if (frozen) {
                const PointQ<T> q1 = eval_point(P1, x);
                Tr1 = Tr1 * (1.0 - sigma_t_of(q1, d) / maj);
            }
            if (Tr0 < kRRThreshold) {
                if (rng.uniform() < 0.5) return T(0.0);
                Tr0 *= 2.0;
                Tr1 = Tr1 * 2.0;
            }
            tau = -std::log(1.0 - rng.uniform());
            continue;
        }
        if (maj > 0.0) tau -= maj * seg;
        t = tc;
        if (tn >= t1) break;
        if (!w.step(ax)) break;
        C.c[ORC_C_CELLS]++;
    }
    if (frozen) return Tr1;
    return T(Tr0);
}

void camera_ray(const Scene& S, uint32_t pixel, double ux, double uy, double o[3], double d[3]) {
    const int i = (int)(pixel % (uint32_t)S.W), j = (int)(pixel / (uint32_t)S.W);
    if (S.cam_kind == 0) {
        const double px = ((i + ux) / S.W - 0.5) * S.win[0];
        const double py = (0.5 - (j + uy) / S.H) * S.win[1];
        for (int k = 0; k < 3; ++k) {
            o[k] = S.eye[k] + px * S.right[k] + py * S.upc[k];
            d[k] = S.fwd[k];
        }
    } else {
        const double px = (2.0 * (i + ux) / S.W - 1.0) * S.tan_half * S.aspect;
        const double py = (1.0 - 2.0 * (j + uy) / S.H) * S.tan_half;
        for (int k = 0; k < 3; ++k) {
            o[k] = S.eye[k];
            d[k] = S.fwd[k] + px * S.right[k] + py * S.upc[k];
        }
        normalize3(d);
    }
}

// Conductor phase function (Eqs. phase and microfacet_vndf) with F = albedo, for travel
// direction d and scattered direction wi: albedo * D(wm) / (4 sigma_proj(d)), wm the half
// vector of v = -d and wi.
// Fresnel reflectance of a conductor with index of refraction n = eta + i k at incidence
// cosine c (the F of Eq. phase), from the Fresnel equations with complex amplitudes:
// w = n cos(theta_t) = sqrt(n^2 - sin^2), r_s = (c - w)/(c + w), r_p = (n^2 c - w)/(n^2 c + w),
// unpolarized F = (|r_s|^2 + |r_p|^2) / 2.
double fresnel_conductor(double c, double eta, double k) {
    c = std::min(std::max(c, 0.0), 1.0);
    const std::complex<double> n(eta, k);
    const std::complex<double> n2 = n * n;
    const std::complex<double> w = std::sqrt(n2 - (1.0 - c * c));
    const std::complex<double> rs = (c - w) / (c + w);
    const std::complex<double> rp = (n2 * c - w) / (n2 * c + w);
    return 0.5 * (std::norm(rs) + std::norm(rp));
}

// F(-w_o, w_m) of Eq. phase: the albedo, times the conductor Fresnel reflectance at the
// microflake when an index of refraction is given.
template <class T>
T fresnel_F(const PointQ<T>& q, double cos_d) {
    if (!(q.f_eta > 0.0)) return q.albedo;
    return q.albedo * fresnel_conductor(cos_d, q.f_eta, q.f_k);
}

template <class T>
T phase_eval(const PointQ<T>& q, const double d[3], const double wi[3]) {
    double h[3] = {wi[0] - d[0], wi[1] - d[1], wi[2] - d[2]};
    const double hn = std::sqrt(dot3(h, h));
    if (hn < 1e-7) return T(0.0);
    h[0] /= hn; h[1] /= hn; h[2] /= hn;
    const double cos_d = -dot3(d, h);   // <v, w_h>, v = -d
    return fresnel_F(q, cos_d) * ndf(q, h) / (4.0 * sigma_proj(q, d));
}

// One light path; returns its radiance estimate.
// With rec != nullptr, vertex k < kmax writes 16 values to rec[16 k ...]: position,
// distance along the segment, tentative collisions of the segment, (phase, Tr) per light,
// half vector, mixture pdf, throughput weight, throughput after the vertex, radiance after
// its next-event estimates.
template <class T>
T trace_path(const Params<double>& P0, const Params<T>& P1, bool frozen, uint32_t pixel,
             uint32_t sample, Counters& C, double& trunc_beta, double* rec = nullptr,
             int kmax = 0) {
    const Scene& S = *P0.S;
    Rng rc(S.key, pixel, sample, 0, kCam);
    const double ux = rc.uniform(), uy = rc.uniform();
    double o[3], d[3];
    camera_ray(S, pixel, ux, uy, o, d);
    T beta = T(1.0), L = T(0.0);
    int b = 0;
    for (;;) {
        double t0, t1;
        if (!clip_box(S, o, d, t0, t1)) {
            L = L + beta * S.env;
            C.c[ORC_C_ESCAPED]++;
            break;
        }
        Rng rt(S.key, pixel, sample, (uint32_t)b, kTrack);
        double th = 0.0;
        T wfac = T(1.0);
        const int64_t steps_before = C.c[ORC_C_TRACK_STEPS];
        const int res = delta_track(P0, P1, frozen, o, d, t0, t1, rt, th, wfac, C);
        double* r = (rec && b < kmax) ? rec + 16 * b : nullptr;
        if (frozen) beta = beta * wfac;
        if (res == kAbsorbed) break;
        if (res == kEscape) {
            L = L + beta * S.env;
            C.c[ORC_C_ESCAPED]++;
            break;
        }
        C.c[ORC_C_REAL]++;
        b += 1;
        if (b > S.max_depth) {
            trunc_beta += val(beta);
            C.c[ORC_C_TRUNCATED]++;
            break;
        }
        const double x[3] = {o[0] + th * d[0], o[1] + th * d[1], o[2] + th * d[2]};
        const PointQ<double> q0 = eval_point(P0, x);
        PointQ<T> q1;
        if (frozen) q1 = eval_point(P1, x);
        if (r) {
            r[0] = x[0]; r[1] = x[1]; r[2] = x[2]; r[3] = th;
            r[4] = (double)(C.c[ORC_C_TRACK_STEPS] - steps_before);
        }
        // next-event estimation to each delta light (directional = stream kNee0, point = kNee0+1)
        for (int li = 0; li < 2; ++li) {
            double wl[3], tend, Le;
            if (li == 0) {
                if (!(S.dl[3] > 0.0)) continue;
                wl[0] = S.dl[0]; wl[1] = S.dl[1]; wl[2] = S.dl[2];
                double a0, a1;
                if (!clip_box(S, x, wl, a0, a1)) a1 = 0.0;
                tend = a1;
                Le = S.dl[3];
            } else {
                if (!(S.pl[3] > 0.0)) continue;
                double dv[3] = {S.pl[0] - x[0], S.pl[1] - x[1], S.pl[2] - x[2]};
                const double r = std::sqrt(dot3(dv, dv));
                wl[0] = dv[0] / r; wl[1] = dv[1] / r; wl[2] = dv[2] / r;
                double a0, a1;
                if (!clip_box(S, x, wl, a0, a1)) a1 = 0.0;
                tend = std::min(a1, r);
                Le = S.pl[3] / (r * r);
            }
            C.c[ORC_C_NEE]++;
            T p;
            if (frozen) p = phase_eval(q1, d, wl);
            else p = T(phase_eval(q0, d, wl));
            Rng rn(S.key, pixel, sample, (uint32_t)b, kNee0 + (uint32_t)li);
            const T Tr = ratio_track(P0, P1, frozen, x, wl, tend, rn, C);
            L = L + beta * p * Tr * Le;
            if (r) { r[5 + 2 * li] = val(p); r[6 + 2 * li] = val(Tr); }
        }
        // phase sampling
        const double v[3] = {-d[0], -d[1], -d[2]};
        const Proposal prop = make_proposal(q0, S.R, v);
        Rng rp(S.key, pixel, sample, (uint32_t)b, kPhase);
        const double usel = rp.uniform();
        const uint32_t ua = rp.next24(), ub = rp.next24();
        double wm[3];
        sample_half_vector(prop, v, usel, ua, ub, wm);
        const double pdf = mixture_pdf(prop, v, wm);
        const double vm = dot3(v, wm);
        C.c[ORC_C_PHASE]++;
        if (!(pdf > 0.0) || !(vm > 0.0)) break;  // degenerate sample: the path ends
        double wi[3] = {2.0 * vm * wm[0] - v[0], 2.0 * vm * wm[1] - v[1], 2.0 * vm * wm[2] - v[2]};
        normalize3(wi);
        // beta *= albedo * D_{w_o}(wm) / pdf, D_{w_o}(wm) = <v, wm> D(wm) / sigma_proj(d)
        T wgt;
        if (frozen) wgt = fresnel_F(q1, vm) * vm * ndf(q1, wm) / (sigma_proj(q1, d) * pdf);
        else wgt = T(fresnel_F(q0, vm) * vm * ndf(q0, wm) / (sigma_proj(q0, d) * pdf));
        beta = beta * wgt;
        if (r) {
            r[9] = wm[0]; r[10] = wm[1]; r[11] = wm[2]; r[12] = pdf; r[13] = val(wgt);
            r[14] = val(beta); r[15] = val(L);
        }
        for (int k = 0; k < 3; ++k) { o[k] = x[k]; d[k] = wi[k]; }
    }
    return L;
}

Params<double> plain_params(const Scene* S) {
    Params<double> P;
    P.S = S;
    return P;
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

int oracle_scene_create(const oracle_scene_desc* D, oracle_scene** out) {
    if (!D || !out) return -1;
    if (D->width <= 0 || D->height <= 0 || D->spp <= 0 || D->max_depth < 0) return -1;
    if (!(D->lengthscale > 0.0) || !(D->albedo >= 0.0 && D->albedo <= 1.0)) return -1;
    if (!(D->lengthscale_n >= 0.0)) return -1;
    if (D->ndf_kind != 0 && D->ndf_kind != 1) return -1;
    if (D->ndf_kind == 1 && D->mean_kind == 2) return -1;   // GGX needs a macro-surface normal
    if (!(D->fresnel_eta >= 0.0) || !(D->fresnel_k >= 0.0)) return -1;
    if (!D->var_grid && !(D->variance > 0.0)) return -1;
    for (int a = 0; a < 3; ++a) {
        if (!(D->bounds[3 + a] > D->bounds[a])) return -1;
        if (D->maj_res[a] <= 0) return -1;
        if (D->offset && D->off_res[a] < 2) return -1;
        if (D->var_grid && D->var_res[a] < 2) return -1;
    }
    if (D->mean_kind == 1 && (D->n_prims <= 0 || !D->prims)) return -1;
    if (D->n_obs < 0 || (D->n_obs > 0 && !D->observations)) return -1;
    if (D->n_obs > 0) {
        // conditioning is defined here for a scalar-variance, isotropic, generalized macrofacet
        if (!(D->obs_noise > 0.0) || !std::isfinite(D->obs_noise) || D->var_grid || D->offset || D->ndf_kind != 0)
            return -1;
        if (D->lengthscale_n > 0.0 && D->lengthscale_n != D->lengthscale) return -1;
    }
    auto* S = new oracle_scene();
    S->mean_kind = D->mean_kind;
    S->mean_const = D->mean_const;
    for (int i = 0; i < (D->mean_kind == 1 ? D->n_prims : 0); ++i) {
        const float* p = D->prims + 8 * i;
        Prim q;
        q.kind = (int)p[0];
        for (int a = 0; a < 3; ++a) { q.c[a] = p[1 + a]; q.h[a] = p[4 + a]; }
        q.albedo = p[7];
        S->prims.push_back(q);
    }
    auto load = [](Grid& g, const float* src, const int32_t* res) {
        if (!src) return;
        for (int a = 0; a < 3; ++a) g.res[a] = res[a];
        const int64_t n = (int64_t)res[0] * res[1] * res[2];
        g.v.assign(src, src + n);
    };
    load(S->offset, D->offset, D->off_res);
    load(S->var, D->var_grid, D->var_res);
    S->variance = D->variance;
    S->l = D->lengthscale;
    S->l_n = D->lengthscale_n > 0.0 ? D->lengthscale_n : D->lengthscale;
    S->aniso = S->l_n != S->l;
    S->ggx = D->ndf_kind == 1;
    S->f_eta = D->fresnel_eta;
    S->f_k = D->fresnel_k;
    S->albedo = D->albedo;
    S->albedo_per_prim = D->albedo_per_prim != 0;
    for (int a = 0; a < 3; ++a) {
        S->lo[a] = D->bounds[a];
        S->hi[a] = D->bounds[3 + a];
        S->ext[a] = S->hi[a] - S->lo[a];
        S->M[a] = D->maj_res[a];
        S->cw[a] = S->ext[a] / S->M[a];
    }
    S->R = D->mix_R;
    for (int k = 0; k < 4; ++k) { S->dl[k] = D->dir_light[k]; S->pl[k] = D->point_light[k]; }
    S->env = D->env;
    S->cam_kind = D->cam_kind;
    for (int k = 0; k < 3; ++k) { S->eye[k] = D->eye[k]; S->fwd[k] = D->target[k] - D->eye[k]; }
    normalize3(S->fwd);
    cross3(S->fwd, D->up, S->right);
    normalize3(S->right);
    cross3(S->right, S->fwd, S->upc);
    S->tan_half = std::tan(0.5 * D->fov_deg * kPi / 180.0);
    S->aspect = (double)D->width / D->height;
    S->win[0] = D->window[0];
    S->win[1] = D->window[1];
    S->W = D->width; S->H = D->height; S->spp = D->spp; S->max_depth = D->max_depth;
    S->key[0] = (uint32_t)(D->seed & 0xFFFFFFFFu);
    S->key[1] = (uint32_t)(D->seed >> 32) ^ D->scene_id;
    S->cond = D->n_obs > 0;
    S->n_obs = D->n_obs;
    S->obs_noise = D->obs_noise;
    if (S->cond) {
        const int n = S->n_obs;
        for (int j = 0; j < n; ++j) {
            for (int a = 0; a < 3; ++a) S->obs_x.push_back(D->observations[4 * j + a]);
            S->obs_m.push_back(D->observations[4 * j + 3]);
        }
        // kappa(C, C) + s_n^2 I, its Cholesky factor, and alpha = (.)^-1 (m - mu(C))
        S->obs_L.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                S->obs_L[(size_t)i * n + j] = se_kernel(*S, &S->obs_x[3 * (size_t)i], &S->obs_x[3 * (size_t)j]) +
                                              (i == j ? S->obs_noise : 0.0);
        if (!cholesky(S->obs_L, n)) { delete S; return -1; }
        S->obs_alpha.resize(n);
        for (int j = 0; j < n; ++j) S->obs_alpha[j] = S->obs_m[j] - prior_mean(*S, &S->obs_x[3 * (size_t)j]);
        chol_solve(S->obs_L, n, S->obs_alpha.data());
    }
    build_majorants(*S);
    *out = S;
    return 0;
}

void oracle_scene_destroy(oracle_scene* s) { delete s; }

int oracle_majorants(const oracle_scene* s, float* out, int64_t n) {
    if (!s || !out || n != (int64_t)s->maj.size()) return -1;
    for (int64_t i = 0; i < n; ++i) out[i] = (float)s->maj[i];
    return 0;
}

static int render_impl(const oracle_scene* s_dec, const oracle_scene* s_w, bool frozen, int32_t s0,
                       int32_t s1, double* mean, double* var, double* paths, double* trunc,
                       int64_t* counters, int32_t nthreads) {
    if (!s_dec || !s_w || s1 <= s0 || s0 < 0 || !mean) return -1;
    const int64_t npix = (int64_t)s_dec->W * s_dec->H;
    const int ns = s1 - s0;
    Counters total;
    const Params<double> P0 = plain_params(s_dec);
    const Params<double> P1 = plain_params(s_w);
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        Counters C;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            double sum = 0.0, sq = 0.0, tb = 0.0;
            for (int sidx = s0; sidx < s1; ++sidx) {
                const double L = trace_path<double>(P0, P1, frozen, (uint32_t)p, (uint32_t)sidx, C, tb);
                sum += L;
                sq += L * L;
                if (paths) paths[p * ns + (sidx - s0)] = L;
            }
            mean[p] = sum / ns;
            if (var) var[p] = ns > 1 ? std::max(0.0, (sq - sum * sum / ns) / (ns - 1)) : 0.0;
            if (trunc) trunc[p] = tb / ns;
        }
#pragma omp critical
        total.add(C);
    }
    if (counters) for (int i = 0; i < ORC_C_COUNT; ++i) counters[i] = total.c[i];
    return 0;
}

static int render_pixels_impl(const oracle_scene* s, const oracle_scene* s_w, bool frozen, const int64_t* pixels,
                              int64_t n, int32_t s0, int32_t s1, double* mean, double* var, int64_t* counters,
                              int32_t nthreads) {
    if (!s || !s_w || !pixels || !mean || n < 0 || s1 <= s0 || s0 < 0) return -1;
    if (s->W != s_w->W || s->H != s_w->H) return -1;
    const int64_t npix = (int64_t)s->W * s->H;
    for (int64_t i = 0; i < n; ++i)
        if (pixels[i] < 0 || pixels[i] >= npix) return -1;
    const int ns = s1 - s0;
    Counters total;
    const Params<double> P = plain_params(s);
    const Params<double> Pw = plain_params(s_w);
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        Counters C;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i) {
            double sum = 0.0, sq = 0.0, tb = 0.0;
            for (int sidx = s0; sidx < s1; ++sidx) {
                const double L = trace_path<double>(P, Pw, frozen, (uint32_t)pixels[i], (uint32_t)sidx, C, tb);
                sum += L;
                sq += L * L;
            }
            mean[i] = sum / ns;
            if (var) var[i] = ns > 1 ? std::max(0.0, (sq - sum * sum / ns) / (ns - 1)) : 0.0;
        }
#pragma omp critical
        total.add(C);
    }
    if (counters) for (int i = 0; i < ORC_C_COUNT; ++i) counters[i] = total.c[i];
    return 0;
}

int oracle_render_pixels(const oracle_scene* s, const int64_t* pixels, int64_t n, int32_t s0, int32_t s1,
                         double* mean, double* var, int64_t* counters, int32_t nthreads) {
    return render_pixels_impl(s, s, false, pixels, n, s0, s1, mean, var, counters, nthreads);
}

int oracle_render_frozen_pixels(const oracle_scene* s_dec, const oracle_scene* s_w, const int64_t* pixels,
                                int64_t n, int32_t s0, int32_t s1, double* mean, int32_t nthreads) {
    return render_pixels_impl(s_dec, s_w, true, pixels, n, s0, s1, mean, nullptr, nullptr, nthreads);
}

int oracle_render(const oracle_scene* s, int32_t s0, int32_t s1, double* mean, double* var,
                  double* paths, double* trunc_beta, int64_t* counters, int32_t nthreads) {
    return render_impl(s, s, false, s0, s1, mean, var, paths, trunc_beta, counters, nthreads);
}

int oracle_render_frozen(const oracle_scene* s_dec, const oracle_scene* s_w, int32_t s0,
                         int32_t s1, double* mean, int64_t* counters, int32_t nthreads) {
    if (!s_dec || !s_w || s_dec->W != s_w->W || s_dec->H != s_w->H) return -1;
    return render_impl(s_dec, s_w, true, s0, s1, mean, nullptr, nullptr, nullptr, counters, nthreads);
}

int oracle_render_grad(const oracle_scene* s, int32_t s0, int32_t s1, const double* dloss,
                       int32_t n_params, const int64_t* param_ids, double* grad, double* mean,
                       int32_t nthreads) {
    if (!s || !dloss || !grad || n_params < 0 || n_params > Dual::N || s1 <= s0 || s0 < 0) return -1;
    if (s->cond) return -1;   // derivatives through the posterior are not carried
    std::unordered_map<int64_t, int> slots;
    Params<Dual> P1;
    P1.S = s;
    for (int j = 0; j < n_params; ++j) {
        const int64_t id = param_ids[j];
        if (id >= 0) {
            if (s->offset.empty() || id >= (int64_t)s->offset.v.size()) return -1;
            slots[id] = j;
        } else if (id == -1) P1.slot_var = j;
        else if (id == -2) P1.slot_l = j;
        else if (id == -3) P1.slot_alb = j;
        else return -1;
    }
    P1.node_slot = &slots;
    const Params<double> P0 = plain_params(s);
    const int64_t npix = (int64_t)s->W * s->H;
    const int ns = s1 - s0;
    std::vector<double> g(n_params, 0.0);
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        std::vector<double> gl(n_params, 0.0);
        Counters C;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            if (dloss[p] == 0.0 && !mean) continue;  // pixels without loss weight add nothing
            double tb = 0.0, sum = 0.0;
            Dual acc(0.0);
            for (int sidx = s0; sidx < s1; ++sidx) {
                const Dual L = trace_path<Dual>(P0, P1, true, (uint32_t)p, (uint32_t)sidx, C, tb);
                acc = acc + L;
                sum += L.v;
            }
            if (mean) mean[p] = sum / ns;
            for (int j = 0; j < n_params; ++j) gl[j] += dloss[p] * acc.d[j] / ns;
        }
#pragma omp critical
        for (int j = 0; j < n_params; ++j) g[j] += gl[j];
    }
    for (int j = 0; j < n_params; ++j) grad[j] = g[j];
    return 0;
}

int oracle_debug_trace(const oracle_scene* s, uint32_t pixel, uint32_t sample, int32_t kmax,
                       double* out) {
    if (!s || !out || kmax < 1) return -1;
    for (int k = 0; k < 16 * kmax + 1; ++k) out[k] = 0.0;
    Counters C;
    double tb = 0.0;
    const Params<double> P = plain_params(s);
    out[16 * kmax] = trace_path<double>(P, P, false, pixel, sample, C, tb, out, kmax);
    return 0;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    philox4x32_10(ctr, key, out);
}

void oracle_uniforms(uint64_t seed, uint32_t scene_id, uint32_t pixel, uint32_t sample,
                     uint32_t bounce, uint32_t stream, int32_t n, double* out) {
    const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32) ^ scene_id};
    Rng r(key, pixel, sample, bounce, stream);
    for (int i = 0; i < n; ++i) out[i] = r.uniform();
}

double oracle_erfcx(double x) { return erfcx_d(x); }
double oracle_fresnel_conductor(double c, double eta, double k) { return fresnel_conductor(c, eta, k); }
double oracle_erfinv(double y) { return erfinv_d(y); }
double oracle_rho(double mu, double sigma) { return rho_of(mu, sigma); }

static PointQ<double> point_from(const double G[3], double s, double albedo, double sn = 0.0, bool ggx = false) {
    PointQ<double> q;
    q.ggx = ggx;
    q.mu = 0.0;
    for (int a = 0; a < 3; ++a) q.G[a] = G[a];
    q.sigma = 0.0;
    q.s = s;
    q.sn = sn > 0.0 ? sn : s;
    q.albedo = albedo;
    return q;
}

double oracle_sigma_proj(const double G[3], double s, const double d[3]) {
    return sigma_proj(point_from(G, s, 1.0), d);
}
double oracle_ndf(const double G[3], double s, const double wm[3]) { return ndf(point_from(G, s, 1.0), wm); }
double oracle_sigma_proj_n(const double G[3], double s, double sn, const double d[3]) {
    return sigma_proj(point_from(G, s, 1.0, sn), d);
}
double oracle_ndf_n(const double G[3], double s, double sn, const double wm[3]) {
    return ndf(point_from(G, s, 1.0, sn), wm);
}
double oracle_beckmann_ndf(double alpha, double cos_m) {
    return beckmann_D(alpha, cos_m, std::max(0.0, 1.0 - cos_m * cos_m));
}
double oracle_beckmann_lambda(double a) { return beckmann_lambda(a); }
double oracle_ndf_aniso(double ax, double ay, double az, const double wm[3]) {
    return ndf_general<double>(ax, ay, az, wm[2], wm[0] * wm[0], wm[1] * wm[1]);
}
double oracle_lambda_aniso(double ax, double ay, double az, const double w[3]) {
    return lambda_cos_general<double>(ax, ay, az, w[2], w[0] * w[0], w[1] * w[1]) / w[2];
}
static double phase_eval_k(const double G[3], double s, double albedo, const double d[3], const double wi[3],
                           bool ggx) {
    return phase_eval(point_from(G, s, albedo, 0.0, ggx), d, wi);
}
static double mixture_pdf_k(const double G[3], double s, double R, const double d[3], const double wm[3],
                            bool ggx) {
    const double v[3] = {-d[0], -d[1], -d[2]};
    const Proposal p = make_proposal(point_from(G, s, 1.0, 0.0, ggx), R, v);
    return mixture_pdf(p, v, wm);
}
static int phase_sample_k(const double G[3], double s, double albedo, double R, const double d[3],
                          const double u[3], double* wi, double* wm, double* weight, double* pdf, bool ggx) {
    const PointQ<double> q = point_from(G, s, albedo, 0.0, ggx);
    const double v[3] = {-d[0], -d[1], -d[2]};
    const Proposal p = make_proposal(q, R, v);
    const uint32_t ua = (uint32_t)(u[1] * 0x1p24), ub = (uint32_t)(u[2] * 0x1p24);
    sample_half_vector(p, v, u[0], ua, ub, wm);
    *pdf = mixture_pdf(p, v, wm);
    const double vm = dot3(v, wm);
    for (int k = 0; k < 3; ++k) wi[k] = 2.0 * vm * wm[k] - v[k];
    normalize3(wi);
    *weight = fresnel_F(q, vm) * vm * ndf(q, wm) / (sigma_proj(q, d) * *pdf);
    return 0;
}
double oracle_phase_eval(const double G[3], double s, double albedo, const double d[3], const double wi[3]) {
    return phase_eval_k(G, s, albedo, d, wi, false);
}
double oracle_mixture_pdf(const double G[3], double s, double R, const double d[3], const double wm[3]) {
    return mixture_pdf_k(G, s, R, d, wm, false);
}
int oracle_phase_sample(const double G[3], double s, double albedo, double R, const double d[3],
                        const double u[3], double* wi, double* wm, double* weight, double* pdf) {
    return phase_sample_k(G, s, albedo, R, d, u, wi, wm, weight, pdf, false);
}
double oracle_sigma_proj_ggx(const double G[3], double s, const double d[3]) {
    return sigma_proj(point_from(G, s, 1.0, 0.0, true), d);
}
double oracle_ndf_ggx(const double G[3], double s, const double wm[3]) {
    return ndf(point_from(G, s, 1.0, 0.0, true), wm);
}
double oracle_phase_eval_ggx(const double G[3], double s, double albedo, const double d[3], const double wi[3]) {
    return phase_eval_k(G, s, albedo, d, wi, true);
}
double oracle_mixture_pdf_ggx(const double G[3], double s, double R, const double d[3], const double wm[3]) {
    return mixture_pdf_k(G, s, R, d, wm, true);
}
int oracle_phase_sample_ggx(const double G[3], double s, double albedo, double R, const double d[3],
                            const double u[3], double* wi, double* wm, double* weight, double* pdf) {
    return phase_sample_k(G, s, albedo, R, d, u, wi, wm, weight, pdf, true);
}

int oracle_eval_point(const oracle_scene* sc, const double x[3], double out[8]) {
    if (!sc) return -1;
    const PointQ<double> q = eval_point(plain_params(sc), x);
    out[0] = q.mu; out[1] = q.G[0]; out[2] = q.G[1]; out[3] = q.G[2];
    out[4] = q.sigma; out[5] = q.s; out[6] = q.albedo; out[7] = q.sn;
    return 0;
}

int oracle_posterior(const oracle_scene* sc, const double x[3], double out[23]) {
    if (!sc || !sc->cond) return -1;
    double f, g[3];
    int which;
    mean_geom(*sc, x, f, g, which);
    if (!sc->offset.empty()) {
        Tri t;
        trilinear(sc->offset, *sc, x, t);
        for (int n = 0; n < 8; ++n) {
            f += t.w[n] * sc->offset.v[t.idx[n]];
            for (int a = 0; a < 3; ++a) g[a] += t.dw[n][a] * sc->offset.v[t.idx[n]];
        }
    }
    const Posterior P = posterior_at(*sc, x, f, g);
    out[0] = P.mu;
    for (int a = 0; a < 3; ++a) out[1 + a] = P.g[a];
    out[4] = P.var;
    for (int a = 0; a < 3; ++a) out[5 + a] = P.c[a];
    const PointQ<double> q = eval_point(plain_params(sc), x);
    const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int e = 0; e < 6; ++e) out[8 + e] = P.Sgg[ij[e][0]][ij[e][1]];
    for (int a = 0; a < 3; ++a) out[14 + a] = q.G[a];
    for (int e = 0; e < 6; ++e) out[17 + e] = q.cov[ij[e][0]][ij[e][1]];
    return 0;
}

static void cov_from6(const double c6[6], double S[3][3]) {
    S[0][0] = c6[0]; S[0][1] = S[1][0] = c6[1]; S[0][2] = S[2][0] = c6[2];
    S[1][1] = c6[3]; S[1][2] = S[2][1] = c6[4]; S[2][2] = c6[5];
}
double oracle_sigma_proj_cov(const double G[3], const double cov6[6], const double d[3]) {
    double S[3][3];
    cov_from6(cov6, S);
    return sigma_proj_cov(G, S, d);
}
double oracle_ndf_cov(const double G[3], const double cov6[6], const double wm[3]) {
    double S[3][3];
    cov_from6(cov6, S);
    return ndf_cov(G, S, wm);
}

double oracle_phase_eval_at(const oracle_scene* sc, const double x[3], const double d[3], const double wi[3]) {
    return phase_eval(eval_point(plain_params(sc), x), d, wi);
}

double oracle_sigma_t(const oracle_scene* sc, const double x[3], const double d[3]) {
    return sigma_t_of(eval_point(plain_params(sc), x), d);
}

int oracle_ratio_tracking(const oracle_scene* sc, const double o[3], const double d[3],
                          double tmax, int32_t n, double* out_T) {
    if (!sc || !out_T || n < 0) return -1;
    const Params<double> P = plain_params(sc);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        Counters C;
        Rng r(sc->key, (uint32_t)i, 0, 0, kNee0);
        out_T[i] = ratio_track<double>(P, P, false, o, d, tmax, r, C);
    }
    return 0;
}

int oracle_free_flight(const oracle_scene* sc, const double o[3], const double d[3], double tmax,
                       int32_t n, double* out_t) {
    const Params<double> P = plain_params(sc);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        Counters C;
        Rng r(sc->key, (uint32_t)i, 0, 0, kTrack);
        double th = 0.0, wf = 1.0;
        const int res = delta_track<double>(P, P, false, o, d, 0.0, tmax, r, th, wf, C);
        out_t[i] = res == kCollide ? th : INFINITY;
    }
    return 0;
}

}  // extern "C"
