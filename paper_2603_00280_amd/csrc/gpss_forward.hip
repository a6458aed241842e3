// Forward kernels: majorant-grid construction, one-thread-per-path rendering, the per-pixel
// reduction and fixed-point accumulator kernels, and pointwise medium evaluation.
#include "gpss_accum.hpp"
#include "gpss_internal.hpp"
#include "gpss_trace.hpp"

namespace gpss {

// ---------------------------------------------------------------------------
// Majorant grid (double precision).  Per cell an upper bound of
// sigma_t = rho(mu, sigma) * sigma_proj over the cell and all directions:
//   rho(mu, sigma) = r(mu / sigma) / sigma with r = phi / Phi decreasing, so
//     rho <= r(mu_min / (mu_min > 0 ? sigma_max : sigma_min)) / sigma_min;
//   sigma_proj <= E[max(0, X)], X ~ N(gmax, s_max^2) = g Phi(g/s) + s phi(g/s);
//   mu_min = the smallest of the primitives' exact minima over the cell (sdf_prim_min_d;
//   exact for the plane),
//   plus the minimum offset node reaching the cell, gmax = |grad sdf| + bound of the
//   trilinear offset gradient.
// The bound times (1 + 2^-10) is rounded up to five significant bits; bounds below
// 2^-40 give 0 (the cell is skipped).
// ---------------------------------------------------------------------------
struct MajArgs {
    int mean_kind;
    float mean_const;
    int n_prims;
    const float4* prims;
    const float* offset;
    int off_res[3];
    const float* var_grid;
    int var_res[3];
    float variance;
    float lengthscale;
    int ggx;
    float lo[3], hi[3];
    int M[3];
    int n_obs;                  // conditioned GP: observations (0: none)
    const double* obs_d;        // 3 n positions, n weights alpha, n x n inverse Cholesky factor
    double obs_noise;
};

__device__ double sdf_prim_d(float4 a, float4 b, const double x[3]) {
    const double v[3] = {x[0] - (double)a.y, x[1] - (double)a.z, x[2] - (double)a.w};
    if (a.x < 0.5f) return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - (double)b.x;
    const double q[3] = {fabs(v[0]) - (double)b.x, fabs(v[1]) - (double)b.y, fabs(v[2]) - (double)b.z};
    const double qmax = fmax(q[0], fmax(q[1], q[2]));
    if (qmax > 0.0) {
        const double p0 = fmax(q[0], 0.0), p1 = fmax(q[1], 0.0), p2 = fmax(q[2], 0.0);
        return sqrt(p0 * p0 + p1 * p1 + p2 * p2);
    }
    return qmax;
}

// Lower bound of a primitive's signed distance over the box [blo, bhi]: for a sphere the
// distance from its centre to the box minus the radius; for a box, with m_a the smallest
// |x_a - c_a| - h_a over the box, the length of the positive m_a when one is positive (the
// cell lies outside the primitive), else max_a m_a (the distance is never below it).  The
// oracle's arithmetic, operation for operation (no contraction), so that both grids agree.
__device__ double sdf_prim_min_d(float4 a, float4 b, const double blo[3], const double bhi[3]) {
#pragma clang fp contract(off)
    const double c[3] = {(double)a.y, (double)a.z, (double)a.w};
    const double h[3] = {(double)b.x, (double)b.y, (double)b.z};
    const bool sphere = a.x < 0.5f;
    double m[3];
    for (int ax = 0; ax < 3; ++ax) {
        const double gap = c[ax] < blo[ax] ? blo[ax] - c[ax] : (c[ax] > bhi[ax] ? c[ax] - bhi[ax] : 0.0);
        m[ax] = sphere ? gap : gap - h[ax];
    }
    if (sphere) return sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) - h[0];
    const double mmax = fmax(m[0], fmax(m[1], m[2]));
    if (!(mmax > 0.0)) return mmax;
    const double p0 = fmax(m[0], 0.0), p1 = fmax(m[1], 0.0), p2 = fmax(m[2], 0.0);
    return sqrt(p0 * p0 + p1 * p1 + p2 * p2);
}

__device__ double quantize_majorant(double B) {
    if (isnan(B)) return INFINITY;
    const double Bp = B * (1.0 + 0x1p-10);
    if (!(Bp >= 0x1p-40)) return 0.0;
    if (isinf(Bp)) return INFINITY;
    int e;
    const double f = frexp(Bp, &e);
    return ldexp(ceil(f * 32.0), e - 5);
}

__device__ __forceinline__ void node_range(int k, int M, int R, int& lo, int& hi) {
    lo = (int)(((long long)k * (R - 1)) / M);
    hi = (int)((((long long)(k + 1)) * (R - 1) + M - 1) / M);
    lo = max(lo, 0);
    hi = min(hi, R - 1);
}

// Prior mean smooth over cell k (centre c, half diagonal h): its gradient g at c and a bound
// H of its Hessian norm over the cell.  Plane and constant means: H = 0.  Signed-distance
// primitives: only when one sphere is the minimum on the whole cell (its distance at c plus
// h below every other primitive's minus h; distances are 1-Lipschitz) and its centre p is
// outside the cell, where |x - p| - R has Hessian norm 1 / |x - p|.  Returns false otherwise.
__device__ bool prior_smooth(const MajArgs& A, const int k[3], const double cw[3], const double c[3], double h,
                             double g[3], double& H) {
    g[0] = g[1] = g[2] = 0.0;
    H = 0.0;
    if (A.mean_kind == 0) {
        g[2] = 1.0;
        return true;
    }
    if (A.mean_kind == 2) return true;
    int best = -1;
    double fb = INFINITY, f2 = INFINITY;
    for (int i = 0; i < A.n_prims; ++i) {
        const double f = sdf_prim_d(A.prims[2 * i], A.prims[2 * i + 1], c);
        if (f < fb) {
            f2 = fb;
            fb = f;
            best = i;
        } else {
            f2 = fmin(f2, f);
        }
    }
    if (best < 0 || A.prims[2 * best].x >= 0.5f || !(fb + h < f2 - h)) return false;
    const float4 P = A.prims[2 * best];
    const double p[3] = {(double)P.y, (double)P.z, (double)P.w};
    double d2 = 0.0, v2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double c0 = (double)A.lo[a] + k[a] * cw[a], c1 = (double)A.lo[a] + (k[a] + 1) * cw[a];
        const double d = p[a] < c0 ? c0 - p[a] : (p[a] > c1 ? p[a] - c1 : 0.0);
        d2 += d * d;
        v2 += (c[a] - p[a]) * (c[a] - p[a]);
    }
    if (!(d2 > 0.0)) return false;
    const double r = sqrt(v2);
    for (int a = 0; a < 3; ++a) g[a] = (c[a] - p[a]) / r;
    H = 1.0 / sqrt(d2);
    return true;
}

// Bound for the GP conditioned on point observations (scalar variance s^2, isotropic
// kernel) over cell k (centre c, half extents e_a, half diagonal h), from the prior mean's
// minimum mu_min, gradient bound gmax and value mu_c at c.  With dmin_j, dmax_j the nearest
// and farthest distances from observation j to the cell, kappa(d) = s^2 e^{-d^2/(2 l^2)} and
// the posterior mean, mean gradient and standard deviation at c:
//   mu_C >= mu_min + sum_j alpha_j kappa(alpha_j > 0 ? dmax_j : dmin_j);
//   |grad mu_C| <= gmax + sum_j |alpha_j| (s^2/l^2) d e^{-d^2/(2l^2)}, d = clamp(l, dmin_j, dmax_j);
//   where the prior mean is smooth on the cell (Hessian norm <= H0, prior_smooth), with
//   Hb = H0 + sum_j |alpha_j| (s^2/l^2) e^{-dmin_j^2/(2l^2)} max(1, dmax_j^2/l^2 - 1) bounding
//   the Hessian of mu_C: |grad mu_C| <= |grad mu_C(c)| + h Hb and (Taylor)
//   mu_C >= mu_C(c) - sum_a e_a |d mu_C(c)/dx_a| - Hb h^2 / 2;  G is the smaller slope bound;
//   mu_C >= mu_C(c) - h G;
//   s_C <= s;  1/s_C^2 <= 1/s^2 + sum_j e^{-dmin_j^2/l^2} / s_n^2 (f(x_j) = r_j f(x) + e_j with
//   e_j independent of f(x) and noise >= s_n^2 I), and |grad s_C| = |cov(grad f, f)| / s_C
//   <= s/l (Cauchy-Schwarz), so s_C(c) -+ h s/l bound s_C from both sides;
//   the conditioned gradient g ~ N(m, Sigma): Sigma <= (s/l)^2 I, |m| <= G + (s/l)|z|, so
//   sigma_proj <= F(G + (s/l)|z|, s/l) with F(M, sd) = sd phi(M/sd) + M Phi(M/sd) (increasing
//   in both, 1-Lipschitz in M);  rho = r(z)/s_C, r = phi/Phi decreasing,
//   z >= z_lo = mu_lo / (mu_lo > 0 ? s_up : s_lo).  Over z < 0: r(z_lo) F(G + (s/l)|z_lo|) / s_lo;
//   over z >= z0 = max(z_lo, 0): (r(z0) F(G) + (s/l) sup_{z >= z0} z r(z)) / s_lo, the supremum
//   being z0 r(z0) for z0 >= 0.9 (z r(z) peaks at 0.29453 near z = 0.84) and 0.2946 otherwise.
__device__ double cond_bound(const MajArgs& A, const int k[3], const double cw[3], double hdiag,
                             double mu_min, double gmax, double mu_c) {
    const int n = A.n_obs;
    const double* X = A.obs_d;
    const double* al = A.obs_d + 3 * n;
    const double* Li = A.obs_d + 4 * n;
    const double l = (double)A.lengthscale, s2 = (double)A.variance;
    const double il2 = 1.0 / (l * l);
    double c[3], lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = (double)A.lo[a] + k[a] * cw[a];
        hi[a] = (double)A.lo[a] + (k[a] + 1) * cw[a];
        c[a] = (double)A.lo[a] + (k[a] + 0.5) * cw[a];
    }
    double g0[3], H0;
    const bool smooth = prior_smooth(A, k, cw, c, hdiag, g0, H0);
    double mu_obs = 0.0, g_obs = 0.0, prec = 1.0 / s2, mu_p = mu_c, hb = 0.0;
    double gp[3] = {g0[0], g0[1], g0[2]};
    double kc[kMaxObs];
#pragma unroll
    for (int j = 0; j < kMaxObs; ++j) {
        kc[j] = 0.0;
        if (j < n) {
            double dn2 = 0.0, df2 = 0.0, dc2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double x = X[3 * j + a];
                const double dn = x < lo[a] ? lo[a] - x : (x > hi[a] ? x - hi[a] : 0.0);
                const double df = fmax(fabs(x - lo[a]), fabs(x - hi[a]));
                dn2 += dn * dn;
                df2 += df * df;
                dc2 += (c[a] - x) * (c[a] - x);
            }
            const double a_j = al[j];
            mu_obs += a_j * s2 * exp(-(a_j > 0.0 ? df2 : dn2) / (2.0 * l * l));
            const double dd = fmin(fmax(l, sqrt(dn2)), sqrt(df2));
            g_obs += fabs(a_j) * (s2 / (l * l)) * dd * exp(-dd * dd / (2.0 * l * l));
            prec += exp(-dn2 / (l * l)) / A.obs_noise;
            hb += fabs(a_j) * (s2 / (l * l)) * exp(-dn2 / (2.0 * l * l)) * fmax(1.0, df2 / (l * l) - 1.0);
            kc[j] = s2 * exp(-dc2 / (2.0 * l * l));
            mu_p += kc[j] * a_j;
            for (int a = 0; a < 3; ++a) gp[a] += -kc[j] * (c[a] - X[3 * j + a]) * il2 * a_j;
        }
    }
    double ww = 0.0;
    for (int i = 0; i < n; ++i) {
        double w = 0.0;
#pragma unroll
        for (int j = 0; j < kMaxObs; ++j) {
            if (j > i) break;
            w += Li[i * n + j] * kc[j];
        }
        ww += w * w;
    }
    const double s_hi = sqrt(s2), sl = s_hi / l;
    double G = gmax + g_obs;
    double mu_lo = mu_min + mu_obs;
    if (smooth) {
        const double Hb = H0 + hb;
        G = fmin(G, sqrt(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2]) + hdiag * Hb);
        double lin = 0.0;
        for (int a = 0; a < 3; ++a) lin += 0.5 * cw[a] * fabs(gp[a]);
        mu_lo = fmax(mu_lo, mu_p - lin - 0.5 * Hb * hdiag * hdiag);
    }
    mu_lo = fmax(mu_lo, mu_p - hdiag * G);
    const double s_c = sqrt(fmax(s2 - ww, 0.0));
    const double s_lo = fmax(1.0 / sqrt(prec), s_c - hdiag * sl);
    const double s_up = fmin(s_hi, s_c + hdiag * sl);
    const double z_lo = mu_lo / (mu_lo > 0.0 ? s_up : s_lo);
    const double kR = sqrt(2.0 / 3.14159265358979323846);
    const double kS2 = 1.41421356237309504880, kS2Pi = 2.50662827463100050242;
    // F(M, sl) with M >= 0
    auto F = [&](double M) {
        const double t = M / sl;
        return sl * (exp(-0.5 * t * t) / kS2Pi) + M * (0.5 * erfc(-t / kS2));
    };
    const double neg = kR / erfcx(-z_lo / kS2) * F(G + sl * fmax(0.0, -z_lo));
    const double z0 = fmax(z_lo, 0.0);
    const double r0 = kR / erfcx(-z0 / kS2);
    const double pos = r0 * F(G) + sl * (z0 >= 0.9 ? z0 * r0 : 0.2946);
    return fmax(neg, pos) / s_lo;
}

__global__ void majorant_kernel(MajArgs A, float* __restrict__ out) {
    const int n = A.M[0] * A.M[1] * A.M[2];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= n) return;
    const int k[3] = {cell % A.M[0], (cell / A.M[0]) % A.M[1], cell / (A.M[0] * A.M[1])};
    double ext[3], cw[3];
    for (int a = 0; a < 3; ++a) {
        ext[a] = (double)A.hi[a] - (double)A.lo[a];
        cw[a] = ext[a] / A.M[a];
    }
    const double hdiag = 0.5 * sqrt(cw[0] * cw[0] + cw[1] * cw[1] + cw[2] * cw[2]);
    double off_min = 0.0, off_g = 0.0;
    if (A.offset) {
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) node_range(k[a], A.M[a], A.off_res[a], lo[a], hi[a]);
        const int* r = A.off_res;
        off_min = INFINITY;
        double md[3] = {0.0, 0.0, 0.0};
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    const long long idx = ((long long)z * r[1] + y) * r[0] + x;
                    const double v = A.offset[idx];
                    off_min = fmin(off_min, v);
                    if (x < hi[0]) md[0] = fmax(md[0], fabs((double)A.offset[idx + 1] - v));
                    if (y < hi[1]) md[1] = fmax(md[1], fabs((double)A.offset[idx + r[0]] - v));
                    if (z < hi[2]) md[2] = fmax(md[2], fabs((double)A.offset[idx + (long long)r[0] * r[1]] - v));
                }
        double gs = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double g = md[a] / (ext[a] / (A.off_res[a] - 1));
            gs += g * g;
        }
        off_g = sqrt(gs);
    }
    double vmin = A.variance, vmax = A.variance;
    if (A.var_grid) {
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) node_range(k[a], A.M[a], A.var_res[a], lo[a], hi[a]);
        const int* r = A.var_res;
        vmin = INFINITY;
        vmax = -INFINITY;
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    const double v = A.var_grid[((long long)z * r[1] + y) * r[0] + x];
                    vmin = fmin(vmin, v);
                    vmax = fmax(vmax, v);
                }
    }
    double mu_min, gmax, mu_centre;
    if (A.mean_kind == 0) {
        mu_min = (double)A.lo[2] + k[2] * cw[2];
        mu_centre = (double)A.lo[2] + (k[2] + 0.5) * cw[2];
        gmax = 1.0;
    } else if (A.mean_kind == 2) {
        mu_min = (double)A.mean_const;
        mu_centre = mu_min;
        gmax = 0.0;
    } else {
        double c[3], blo[3], bhi[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (double)A.lo[a] + (k[a] + 0.5) * cw[a];
            blo[a] = __dadd_rn((double)A.lo[a], __dmul_rn((double)k[a], cw[a]));
            bhi[a] = __dadd_rn((double)A.lo[a], __dmul_rn((double)(k[a] + 1), cw[a]));
        }
        double best = INFINITY;
        mu_min = INFINITY;
        for (int i = 0; i < A.n_prims; ++i) {
            best = fmin(best, sdf_prim_d(A.prims[2 * i], A.prims[2 * i + 1], c));
            mu_min = fmin(mu_min, sdf_prim_min_d(A.prims[2 * i], A.prims[2 * i + 1], blo, bhi));
        }
        mu_centre = best;
        gmax = 1.0;
    }
    mu_min += off_min;
    gmax += off_g;
    if (A.n_obs > 0) {   // conditioned GP (no offset grid, scalar variance)
        out[cell] = (float)quantize_majorant(cond_bound(A, k, cw, hdiag, mu_min, gmax, mu_centre));
        return;
    }
    const double smin = sqrt(vmin), smax = sqrt(vmax);
    const double s_max = smax / (double)A.lengthscale;
    const double zr = mu_min / (mu_min > 0.0 ? smax : smin);
    const double rho_max = sqrt(2.0 / 3.14159265358979323846) / erfcx(-zr / 1.41421356237309504880) / smin;
    double proj_max;
    if (A.ggx) {   // GGX height field: sigma <= (|G| + sqrt(|G|^2 + 2 s^2)) / 2
        proj_max = 0.5 * (gmax + sqrt(gmax * gmax + 2.0 * s_max * s_max));
    } else {
        const double z = gmax / s_max;
        const double Phi = 0.5 * erfc(-z / 1.41421356237309504880);
        const double phi = exp(-0.5 * z * z) / 2.50662827463100050242;
        proj_max = gmax * Phi + s_max * phi;
    }
    out[cell] = (float)quantize_majorant(rho_max * proj_max);
}

// The walk's copy of the majorant grid (SceneDev::maj16): the top 16 bits of each float,
// exact because quantize_majorant keeps five significant bits (and 0 and infinity).
__global__ void majorant16_kernel(const float* __restrict__ maj, uint16_t* __restrict__ out, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) out[c] = (uint16_t)(__float_as_uint(maj[c]) >> 16);
}

int launch_majorants(gpss_scene* s, hipStream_t stream) {
    const gpss_scene_desc& D = s->desc;
    MajArgs A{};
    A.mean_kind = D.mean_kind;
    A.mean_const = D.mean_const;
    A.n_prims = (int)D.n_prims;
    A.prims = reinterpret_cast<const float4*>(s->d_prims);
    A.offset = s->d_offset;
    A.var_grid = s->d_var;
    for (int a = 0; a < 3; ++a) {
        A.off_res[a] = (int)D.off_res[a];
        A.var_res[a] = (int)D.var_res[a];
        A.lo[a] = D.bounds[a];
        A.hi[a] = D.bounds[3 + a];
        A.M[a] = (int)D.majorant_res[a];
    }
    A.variance = D.variance;
    // the largest gradient standard deviation: sigma over the smaller of the two lengthscales
    A.lengthscale = D.lengthscale_n > 0.0f ? fminf(D.lengthscale, D.lengthscale_n) : D.lengthscale;
    A.ggx = D.ndf_kind == GPSS_NDF_GGX;
    A.n_obs = (int)D.n_obs;
    A.obs_d = s->d_obs_d;
    A.obs_noise = D.obs_noise;
    const int n = A.M[0] * A.M[1] * A.M[2];
    hipLaunchKernelGGL(majorant_kernel, dim3((n + 127) / 128), dim3(128), 0, stream, A, s->d_maj);
    hipLaunchKernelGGL(majorant16_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, s->d_maj, s->d_maj16, n);
    return check_hip(hipGetLastError(), "majorant kernels launch");
}

// ---------------------------------------------------------------------------
// One thread per path: thread p renders (pixel p / ns, sample s0 + p % ns).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void flush_stats(const PathStats& st, unsigned long long* counters) {
    const uint32_t vals[12] = {st.track_steps, st.real, st.nee_steps, st.violations, st.capped,
                               st.escaped, st.truncated, st.cells, st.phase, st.nee, st.nonfinite, st.saturated};
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        const uint32_t t = wave_sum(vals[i]);
        if (lead && t) atomicAdd(&counters[i], (unsigned long long)t);
    }
}

// Minimum waves per SIMD the one-thread-per-path kernel is compiled for (register budget).
#ifndef GPSS_MEGA_MIN_WAVES
#define GPSS_MEGA_MIN_WAVES 4
#endif

template <bool STATS>
__global__ __launch_bounds__(256, GPSS_MEGA_MIN_WAVES) void render_paths_kernel(SceneDev S, float* __restrict__ paths,
                                                           unsigned long long* counters, uint32_t s0,
                                                           uint32_t ns, uint64_t npaths) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    PathStats st;
    st.clear();
    if (p < npaths) {
        const uint32_t pixel = (uint32_t)(p / ns);
        const uint32_t sample = s0 + (uint32_t)(p % ns);
        const float L = trace_path<STATS>(S, pixel, sample, st);
        if (STATS) {
            const int c = acc_class(L);
            st.nonfinite += c == kAccNonFinite;
            st.saturated += c == kAccSaturated;
        }
        paths[p] = L;
    }
    if (STATS) flush_stats(st, counters);
}

int mega_render(gpss_scene* s, float* paths, uint64_t* counters, uint32_t s0, uint32_t ns,
                hipStream_t stream) {
    const uint64_t npaths = s->n_pixels() * ns;
    const uint64_t blocks = (npaths + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return set_error(GPSS_ERR_INVALID_ARG, "too many paths in one launch");
    if (counters)
        hipLaunchKernelGGL(render_paths_kernel<true>, dim3((uint32_t)blocks), dim3(256), 0, stream, s->dev,
                           paths, reinterpret_cast<unsigned long long*>(counters), s0, ns, npaths);
    else
        hipLaunchKernelGGL(render_paths_kernel<false>, dim3((uint32_t)blocks), dim3(256), 0, stream, s->dev,
                           paths, nullptr, s0, ns, npaths);
    return check_hip(hipGetLastError(), "render_paths_kernel launch");
}

// Diagnostics: trace listed (pixel, sample) paths and keep their per-vertex records.
__global__ void debug_trace_kernel(SceneDev S, const uint32_t* __restrict__ ids, uint32_t n,
                                   float* __restrict__ out, int kmax) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    PathStats st;
    st.clear();
    float* rec = out + (size_t)i * (kmax * kRecFields + 1);
    for (int k = 0; k < kmax * kRecFields; ++k) rec[k] = 0.0f;
    rec[kmax * kRecFields] = trace_path<false, true>(S, ids[2 * i], ids[2 * i + 1], st, rec, kmax);
}

int launch_debug_trace(gpss_scene* s, const uint32_t* ids, uint32_t n, float* out, int kmax,
                       hipStream_t stream) {
    if (s->dev.n_obs > 0)
        return set_error(GPSS_ERR_UNSUPPORTED, "debug traces of a conditioned GP are not available");
    hipLaunchKernelGGL(debug_trace_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, s->dev, ids, n, out, kmax);
    return check_hip(hipGetLastError(), "debug_trace_kernel launch");
}

int launch_render_paths(gpss_scene* s, float* paths, uint64_t* counters, uint32_t s0, uint32_t ns,
                        hipStream_t stream) {
    if (s->dev.n_obs > 0 && (s->kernel == GPSS_KERNEL_MEGA || s->kernel == GPSS_KERNEL_WAVEFRONT))
        return set_error(GPSS_ERR_UNSUPPORTED, "a conditioned GP renders with the persistent kernel only");
    if (s->kernel == GPSS_KERNEL_MEGA) return mega_render(s, paths, counters, s0, ns, stream);
    if (s->kernel == GPSS_KERNEL_WAVEFRONT) return wf_render(s, paths, counters, s0, ns, stream);
    return sched_render(s, paths, nullptr, counters, s0, ns, stream);
}

// Per-pixel mean over the sample range from per-path radiances: the same fixed-point sums as
// the accumulating kernels (gpss_accum.hpp), hence the same image.
__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ paths, float* __restrict__ image,
                                                     uint32_t ns, uint64_t npix) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const float* src = paths + p * ns;
    unsigned long long lo = 0, hi = 0;
    for (uint32_t k = 0; k < ns; ++k) {
        const uint64_t v = acc_fixed(src[k]);
        lo += v & 0xFFFFFFFFull;
        hi += v >> 32;
    }
    image[p] = acc_mean(lo, hi, ns);
}

int launch_reduce(gpss_scene* s, const float* paths, float* image, uint32_t ns, hipStream_t stream) {
    const uint64_t npix = s->n_pixels();
    hipLaunchKernelGGL(reduce_kernel, dim3((uint32_t)((npix + 255) / 256)), dim3(256), 0, stream, paths, image,
                       ns, npix);
    return check_hip(hipGetLastError(), "reduce_kernel launch");
}

// Fixed-point accumulator of npix pixels (two words each): cleared before a launch adds to it,
// turned into the image after.  Kernels rather than memsets, so that they may be captured.
__global__ __launch_bounds__(256) void acc_clear_kernel(unsigned long long* __restrict__ acc, uint64_t nwords) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) acc[i] = 0ull;
}

__global__ __launch_bounds__(256) void acc_finalize_kernel(const unsigned long long* __restrict__ acc,
                                                           float* __restrict__ image, uint32_t ns, uint64_t npix) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    image[p] = acc_mean(acc[2 * p], acc[2 * p + 1], ns);
}

int launch_acc_clear(unsigned long long* acc, uint64_t npix, hipStream_t stream) {
    const uint64_t nw = 2 * npix;
    hipLaunchKernelGGL(acc_clear_kernel, dim3((uint32_t)((nw + 255) / 256)), dim3(256), 0, stream, acc, nw);
    return check_hip(hipGetLastError(), "acc_clear_kernel launch");
}

int launch_acc_finalize(const unsigned long long* acc, float* image, uint32_t ns, uint64_t npix,
                        hipStream_t stream) {
    hipLaunchKernelGGL(acc_finalize_kernel, dim3((uint32_t)((npix + 255) / 256)), dim3(256), 0, stream, acc, image,
                       ns, npix);
    return check_hip(hipGetLastError(), "acc_finalize_kernel launch");
}

// ---------------------------------------------------------------------------
// Pointwise medium evaluation.
// ---------------------------------------------------------------------------
template <bool COND>
__global__ void eval_kernel(SceneDev S, const float* __restrict__ pts, const float* __restrict__ dirs,
                            float* __restrict__ out, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float3 x = f3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
    const float3 d = f3(dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]);
    PointQ q = eval_point(S, x);
    if (COND) condition_point(S, x, q);
    const float r = rho_of(q.mu, q.sigma);
    const float sp = sigma_proj_at(q, d);
    float* o = out + 8 * i;
    o[0] = q.mu;
    o[1] = q.sigma;
    o[2] = q.s;
    o[3] = r;
    o[4] = sp;
    o[5] = r * sp;
    o[6] = ndf_at(q, d);
    o[7] = q.albedo;
}

int launch_eval(gpss_scene* s, const float* pts, const float* dirs, float* out, uint64_t n, hipStream_t stream) {
    if (s->dev.n_obs > 0)
        hipLaunchKernelGGL(eval_kernel<true>, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, stream, s->dev,
                           pts, dirs, out, n);
    else
        hipLaunchKernelGGL(eval_kernel<false>, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, stream, s->dev,
                           pts, dirs, out, n);
    return check_hip(hipGetLastError(), "eval_kernel launch");
}

}  // namespace gpss
