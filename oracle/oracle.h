/* FP64 CPU oracle for macrofacet rendering of Gaussian process statistical surfaces.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that the GPU
 * path is checked against; it is loaded by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg, and by nothing else.  It shares no code with the GPU
 * library.
 *
 * What it computes (paper sections / equations):
 *   - GP statistics at a point: value/gradient joint Gaussian (Sec. 3.1, Eq. joint_fg),
 *     roughness alpha = sqrt(2) sigma / l (Eq. roughness);
 *   - density rho = phi(f;0,s^2)/Phi(f;0,s^2) and projected area Lambda(w) cos(theta),
 *     extinction sigma_t = rho * sigma(w) (Sec. 4.2.1, Eqs. generalized_sigma_t and
 *     generalized_lambda);
 *   - the generalized NDF in closed form (Sec. 4.2.2, Eq. macro_ndf, Appendix A) and the
 *     conductor phase function built from it (Sec. 3.2, Eqs. phase, microfacet_vndf);
 *   - the R : (1-R) mixture of Beckmann visible-normal sampling and uniform hemisphere
 *     sampling about -w_o (end of Sec. 4.2.2);
 *   - null-scattering volumetric path tracing of the resulting classic exponential
 *     medium (Sec. 5): delta tracking, ratio tracking for next-event estimation.
 * All arithmetic is double precision.  Random numbers come from Philox4x32-10
 * (Salmon et al., SC'11) addressed by (pixel, sample, bounce, stream).
 *
 * Error behaviour: functions return 0 on success and a negative value on invalid
 * arguments; nothing is thrown across this interface.
 */
#ifndef GPSS_ORACLE_H
#define GPSS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t mean_kind;          /* 0 plane mu=z, 1 union SDF of prims, 2 constant mean */
    double mean_const;          /* constant mean value (mean_kind 2) */
    int32_t n_prims;
    const float* prims;         /* n_prims x 8: kind, cx, cy, cz, a, b, c, albedo */
    const float* offset;        /* nullable; off_res[2] x off_res[1] x off_res[0], x fastest */
    int32_t off_res[3];
    double variance;            /* scalar kernel variance (used when var_grid is NULL) */
    const float* var_grid;      /* nullable; var_res grid of variances */
    int32_t var_res[3];
    double lengthscale;
    double albedo;
    int32_t albedo_per_prim;
    double bounds[6];           /* lo xyz, hi xyz; every grid is node-centred over it */
    double mix_R;
    int32_t maj_res[3];
    double dir_light[4];        /* unit direction toward the light, irradiance E (0 = none) */
    double point_light[4];      /* position, intensity I (0 = none) */
    double env;                 /* constant environment radiance */
    int32_t cam_kind;           /* 0 orthographic, 1 pinhole */
    double eye[3], target[3], up[3];
    double fov_deg;             /* pinhole vertical field of view */
    double window[2];           /* orthographic window width, height */
    int32_t width, height, spp, max_depth;
    uint64_t seed;
    uint32_t scene_id;
    double lengthscale_n;       /* lengthscale along the local mean-gradient direction (0: = lengthscale) */
    int32_t ndf_kind;           /* 0: generalized macrofacet (Eq. macro_ndf); 1: GGX height field */
    double fresnel_eta, fresnel_k;  /* conductor IOR eta + i k of the Fresnel term; eta = 0: F = albedo */
    /* GP conditioning (Eq. condition_gp): n_obs x 4 (x, y, z, observed value), with
     * observation-noise variance obs_noise > 0; needs a scalar variance, the isotropic
     * kernel and the generalized NDF.  n_obs = 0: the unconditioned GP. */
    const float* observations;
    int32_t n_obs;
    double obs_noise;
} oracle_scene_desc;

typedef struct oracle_scene oracle_scene;

/* counters[] layout (int64): */
enum {
    ORC_C_TRACK_STEPS = 0,  /* tentative collisions during free-flight sampling */
    ORC_C_REAL = 1,         /* real collisions (scattering events, incl. the truncating one) */
    ORC_C_NEE_STEPS = 2,    /* tentative collisions during ratio tracking */
    ORC_C_VIOLATIONS = 3,   /* sigma_t above the cell majorant (must be 0) */
    ORC_C_CAPPED = 4,       /* segments that hit the step cap */
    ORC_C_ESCAPED = 5,      /* paths that left the medium */
    ORC_C_TRUNCATED = 6,    /* paths stopped by the depth limit */
    ORC_C_CELLS = 7,        /* majorant cells visited by delta and ratio tracking */
    ORC_C_PHASE = 8,        /* phase-function samples */
    ORC_C_NEE = 9,          /* next-event estimates (light connections) */
    ORC_C_COUNT = 16
};

int oracle_scene_create(const oracle_scene_desc* desc, oracle_scene** out);
void oracle_scene_destroy(oracle_scene* s);

/* Majorant grid, maj_res[0]*maj_res[1]*maj_res[2] float values, x fastest. */
int oracle_majorants(const oracle_scene* s, float* out, int64_t n);

/* Forward render of samples [s0, s1).  mean/var: width*height (var = unbiased sample
 * variance of the per-path radiance, 0 when fewer than 2 samples); paths (nullable):
 * width*height*(s1-s0), pixel-major; trunc_beta (nullable): per-pixel mean throughput
 * of depth-truncated paths; counters: ORC_C_COUNT int64. */
int oracle_render(const oracle_scene* s, int32_t s0, int32_t s1, double* mean, double* var,
                  double* paths, double* trunc_beta, int64_t* counters, int32_t nthreads);

/* Forward render of listed pixels only (flat indices): mean/var of n entries. */
int oracle_render_pixels(const oracle_scene* s, const int64_t* pixels, int64_t n, int32_t s0,
                         int32_t s1, double* mean, double* var, int64_t* counters, int32_t nthreads);

/* Frozen-sampling render: every sampling decision is taken with scene s_dec, every
 * weight is evaluated with scene s_w (same geometry, different parameters). With
 * s_w == s_dec it equals oracle_render. */
int oracle_render_frozen(const oracle_scene* s_dec, const oracle_scene* s_w, int32_t s0,
                         int32_t s1, double* mean, int64_t* counters, int32_t nthreads);
/* The same for listed pixels only (flat indices): mean of n entries. */
int oracle_render_frozen_pixels(const oracle_scene* s_dec, const oracle_scene* s_w, const int64_t* pixels,
                                int64_t n, int32_t s0, int32_t s1, double* mean, int32_t nthreads);

/* Gradient of sum_p dloss[p] * I_p w.r.t. the selected parameters, by forward-mode
 * dual numbers through the frozen-sampling estimator at the scene's parameters.
 * param_ids[j] >= 0 selects offset-grid node j (flat index), -1 the kernel variance,
 * -2 the lengthscale, -3 the albedo.  n_params <= 32. Also writes the image (nullable);
 * when mean is NULL, pixels with dloss == 0 are skipped. */
int oracle_render_grad(const oracle_scene* s, int32_t s0, int32_t s1, const double* dloss,
                       int32_t n_params, const int64_t* param_ids, double* grad,
                       double* mean, int32_t nthreads);

/* Per-vertex record of one path (16 doubles per real collision k < kmax, then the path
 * radiance at out[16 kmax]); same fields as the GPU library's debug trace. */
int oracle_debug_trace(const oracle_scene* s, uint32_t pixel, uint32_t sample, int32_t kmax,
                       double* out);

/* ---- point functions (used by the closed-form pins) ---- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_uniforms(uint64_t seed, uint32_t scene_id, uint32_t pixel, uint32_t sample,
                     uint32_t bounce, uint32_t stream, int32_t n, double* out);
double oracle_erfcx(double x);
double oracle_erfinv(double y);
double oracle_rho(double mu, double sigma);
double oracle_sigma_proj(const double G[3], double s, const double d[3]);
double oracle_ndf(const double G[3], double s, const double wm[3]);
double oracle_beckmann_ndf(double alpha, double cos_m);
double oracle_beckmann_lambda(double a);
/* Eqs. macro_ndf and generalized_lambda with separate roughnesses, local frame (z = normal) */
/* sigma(d) and D(wm) for g ~ N(G, s^2 (I - n n^T) + sn^2 n n^T), n = G/|G| (z if G = 0) */
double oracle_sigma_proj_n(const double G[3], double s, double sn, const double d[3]);
double oracle_ndf_n(const double G[3], double s, double sn, const double wm[3]);
double oracle_ndf_aniso(double ax, double ay, double az, const double wm[3]);
double oracle_lambda_aniso(double ax, double ay, double az, const double w[3]);
double oracle_phase_eval(const double G[3], double s, double albedo, const double d[3],
                         const double wi[3]);
/* pdf of the mixture proposal over half vectors */
double oracle_mixture_pdf(const double G[3], double s, double R, const double d[3],
                          const double wm[3]);
/* one phase sample from uniforms u[3] = (select, a, b): out wi[3], wm[3], weight, pdf */
int oracle_phase_sample(const double G[3], double s, double albedo, double R,
                        const double d[3], const double u[3], double* wi, double* wm,
                        double* weight, double* pdf);
/* unpolarized Fresnel reflectance of a conductor (IOR eta + i k) at incidence cosine c */
double oracle_fresnel_conductor(double c, double eta, double k);
/* the same for the GGX height-field macrofacet (NDF kind 1) */
double oracle_sigma_proj_ggx(const double G[3], double s, const double d[3]);
double oracle_ndf_ggx(const double G[3], double s, const double wm[3]);
double oracle_phase_eval_ggx(const double G[3], double s, double albedo, const double d[3], const double wi[3]);
double oracle_mixture_pdf_ggx(const double G[3], double s, double R, const double d[3], const double wm[3]);
int oracle_phase_sample_ggx(const double G[3], double s, double albedo, double R, const double d[3],
                            const double u[3], double* wi, double* wm, double* weight, double* pdf);
/* Conditioned scenes: posterior at x, 23 doubles: mu_C, grad mu_C[3], var_C, c[3] = cov(grad f,
 * f), Sgg[6] = cov(grad f) (xx xy xz yy yz zz), then the gradient distribution given f(x) = 0:
 * mean[3], covariance[6].  -1 for an unconditioned scene. */
int oracle_posterior(const oracle_scene* sc, const double x[3], double out[23]);
/* projected area and NDF for g ~ N(G, Sigma), Sigma given as xx xy xz yy yz zz */
double oracle_sigma_proj_cov(const double G[3], const double cov6[6], const double d[3]);
double oracle_ndf_cov(const double G[3], const double cov6[6], const double wm[3]);
/* mu, G[3], sigma, s (across n), albedo, s_n (along n) at a point */
int oracle_eval_point(const oracle_scene* sc, const double x[3], double out[8]);
double oracle_sigma_t(const oracle_scene* sc, const double x[3], const double d[3]);
/* phase function of the scene's medium at x for travel direction d, scattered direction wi */
double oracle_phase_eval_at(const oracle_scene* sc, const double x[3], const double d[3], const double wi[3]);
/* ratio-tracking transmittance estimates of n independent streams (pixel index = i) */
int oracle_ratio_tracking(const oracle_scene* sc, const double o[3], const double d[3],
                          double tmax, int32_t n, double* out_T);
/* first real collision distance by delta tracking for n streams (INFINITY on escape) */
int oracle_free_flight(const oracle_scene* sc, const double o[3], const double d[3],
                       double tmax, int32_t n, double* out_t);

#ifdef __cplusplus
}
#endif
#endif
