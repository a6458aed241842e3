/* gpss: MI355X (gfx950) renderer for Gaussian process statistical surfaces (GPSSes)
 * under macrofacet theory.
 *
 * A GPSS is a Gaussian process f ~ GP(mu, kappa) with a squared-exponential kernel
 * (Sec. 3.1, Eq. se_kernel) whose zero level set is the surface.  Macrofacet theory
 * renders it, without realizations, as a classic exponential participating medium with
 *   extinction  sigma_t(x, w) = rho(x) sigma(w),
 *               rho = phi(mu; 0, s^2) / Phi(mu; 0, s^2)            (Sec. 4.2.1, Eq. generalized_sigma_t)
 *               sigma(w) = Lambda(w) cos(theta)                    (Eq. generalized_lambda)
 *   phase       p(w_o, w_i) = F D_{w_o}(w_m) / (4 |w_o . w_m|)     (Sec. 3.2, Eqs. phase, microfacet_vndf)
 *               with the generalized NDF D of Sec. 4.2.2 (Eq. macro_ndf) and F = albedo,
 * and is rendered by null-scattering volumetric path tracing (Sec. 5).
 *
 * Conventions used by every entry point
 *   - All calls return GPSS_OK (0) or a negative GPSS_ERR_* code; gpss_last_error() gives a
 *     thread-local message for the last failure on the calling thread.  Invalid arguments
 *     are rejected before any device work is enqueued.  No C++ exception crosses the ABI.
 *   - "host" pointers are read during the call only; "device" pointers are device memory
 *     owned by the caller, which must stay valid until the enqueued work completes.
 *   - Rendering calls are asynchronous and ordered on the given HIP stream (NULL = the
 *     default stream); the caller synchronizes.  A scene must not be used by two
 *     overlapping calls at once (it owns per-scene scratch memory).
 *   - Random numbers: Philox4x32-10 with key (seed_lo32, seed_hi32 ^ scene_id) and counter
 *     (pixel, sample, bounce | stream << 16, block); results are a deterministic function
 *     of the scene and the sample range.
 */
#ifndef GPSS_H
#define GPSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gpss_scene* gpss_scene_t;
typedef struct ihipStream_t* gpss_stream_t; /* hipStream_t */

enum {
    GPSS_OK = 0,
    GPSS_ERR_INVALID_ARG = -1,
    GPSS_ERR_HIP = -2,
    GPSS_ERR_OOM = -3,
    GPSS_ERR_UNSUPPORTED = -4
};

enum { GPSS_MEAN_PLANE = 0, GPSS_MEAN_SDF = 1, GPSS_MEAN_CONST = 2 };
enum { GPSS_PRIM_SPHERE = 0, GPSS_PRIM_BOX = 1 };
enum { GPSS_CAM_ORTHO = 0, GPSS_CAM_PINHOLE = 1 };
enum { GPSS_NDF_GENERALIZED = 0, GPSS_NDF_GGX = 1 };

/* Statement of one rendering problem (all host memory, copied by gpss_scene_create).
 * Grids are float32, x fastest, node-centred over `bounds` (node i at lo + i/(res-1)*ext). */
typedef struct {
    uint32_t struct_size;          /* sizeof(gpss_scene_desc): ABI version check */
    /* GP mean mu(x) (Sec. 3.1) */
    int32_t mean_kind;             /* GPSS_MEAN_*: plane mu = z, union of SDF primitives, constant */
    float mean_const;              /* value of the constant mean */
    const float* prims;            /* n_prims x 8: kind, cx, cy, cz, a (radius | half x), b, c, albedo */
    uint32_t n_prims;              /* 1..64 for GPSS_MEAN_SDF */
    const float* mean_offset;      /* nullable: trilinear offset grid added to mu */
    uint32_t off_res[3];
    /* squared-exponential kernel (Eq. se_kernel, isotropic) */
    float variance;                /* sigma^2 > 0, used when variance_grid is NULL */
    const float* variance_grid;    /* nullable: trilinear grid of sigma^2 (locally stationary) */
    uint32_t var_res[3];
    float lengthscale;             /* l > 0; gradient std is sigma / l (Eq. roughness); see lengthscale_n */
    /* medium */
    float albedo;                  /* F of the conductor phase function, in [0, 1] */
    int32_t albedo_per_prim;       /* nonzero: albedo of the primitive with the smallest SDF */
    float bounds[6];               /* support box lo xyz, hi xyz */
    float mix_R;                   /* probability of the Beckmann visible-normal proposal */
    uint32_t majorant_res[3];      /* majorant grid cells per axis (1..256) */
    /* lights */
    float dir_light[4];            /* unit direction toward the light, irradiance E (0 = none) */
    float point_light[4];          /* position, intensity I (0 = none) */
    float env_radiance;            /* constant environment radiance (escaped paths) */
    /* camera */
    int32_t cam_kind;              /* GPSS_CAM_* */
    float cam_eye[3], cam_target[3], cam_up[3];
    float cam_fov_deg;             /* pinhole vertical field of view, degrees */
    float cam_window[2];           /* orthographic window width, height */
    /* sampler */
    uint32_t width, height;        /* pixels; row 0 at the top */
    uint32_t spp;                  /* samples per pixel of a full render */
    uint32_t max_depth;            /* maximum number of real scattering events per path */
    uint64_t seed;
    uint32_t scene_id;
    /* kernel anisotropy (Eq. se_kernel in the frame of the local geometric normal, i.e. the
     * mean-gradient direction, z where grad mu = 0): lengthscale along that direction;
     * `lengthscale` applies across it.  0 = isotropic (l_n = l).  Sec. 4.2.1: alpha_z =
     * sqrt(2) sigma / l_n in Eqs. generalized_lambda and macro_ndf. */
    float lengthscale_n;
    /* NDF of the macrofacet: GPSS_NDF_GENERALIZED (the GP macrofacet of Sec. 4.2, Eqs.
     * generalized_lambda and macro_ndf) or GPSS_NDF_GGX (height-field macrofacet with the GGX
     * NDF and Smith Lambda about the mean gradient, roughness sqrt(2) sigma / l; end of
     * Sec. 4.1, Fig. cmp_ggx).  GGX needs a mean with a gradient (not GPSS_MEAN_CONST) and
     * the isotropic kernel. */
    int32_t ndf_kind;
    /* conductor Fresnel term (Eq. phase): index of refraction eta + i k of the microflakes;
     * F = albedo x Fresnel reflectance at the half vector.  eta = 0: F = albedo. */
    float fresnel_eta, fresnel_k;
    /* GP conditioned on point observations (Sec. 3.1, Eq. condition_gp): n_obs (0..32) rows of
     * (x, y, z, observed value) taken with independent Gaussian noise of variance obs_noise
     * (at least 1e-4 x variance, so that single precision resolves the posterior variance),
     * which adds obs_noise I to kappa(C, C) (a zero noise, the equation as printed, would let
     * the posterior variance vanish at the observations and the density become singular).
     * The medium is then the conditioned GP's: f(x) ~ N(mu_C, kappa_C(x, x)), and the gradient
     * given f(x) = 0 has the posterior's full 3x3 covariance (Eq. joint_fg conditioned the same
     * way).  Needs a scalar variance, no mean offset grid, the isotropic kernel and the
     * generalized NDF.  Rendered by the persistent kernel; GPSS_KERNEL_MEGA and _WAVEFRONT,
     * gpss_render_batch, gpss_render_adjoint, gpss_scene_set_params and gpss_debug_trace return
     * GPSS_ERR_UNSUPPORTED for such a scene.  n_obs = 0: the unconditioned GP. */
    const float* observations;
    uint32_t n_obs;
    float obs_noise;
} gpss_scene_desc;

/* Create a scene: validates `desc`, uploads primitives and grids, and builds the
 * conservative majorant grid on the device (double precision, rounded up to five
 * significant bits; the tracer reads a 16-bit copy, which holds every such value exactly).
 * For a union of 4 to 16 primitives it also lists, per majorant cell, the primitives that can
 * be the union's minimum there (2 bytes per cell), so that a medium evaluation visits only
 * those; the results equal the full union's bit for bit.  Device memory beyond the inputs:
 * 6 bytes per majorant cell (8 with such a union), and a ~0.5 KiB scene record.
 * Synchronous.  *out receives the handle. */
int gpss_scene_create(const gpss_scene_desc* desc, gpss_scene_t* out);
int gpss_scene_destroy(gpss_scene_t scene);

/* Implementation used by gpss_render / gpss_render_paths.  All give bit-identical path
 * radiances.  AUTO (default) = PERSISTENT: persistent waves that take paths in chunks and
 * schedule each path's operations (cell steps, medium evaluations, phase sampling, segment
 * starts) so that every operation runs for many lanes of a wave at once; WAVEFRONT:
 * per-bounce track / scatter / light-connection kernels over queues of structure-of-arrays
 * path state; MEGA: one thread per path. */
enum { GPSS_KERNEL_AUTO = 0, GPSS_KERNEL_MEGA = 1, GPSS_KERNEL_WAVEFRONT = 2, GPSS_KERNEL_PERSISTENT = 3 };
int gpss_scene_set_kernel(gpss_scene_t scene, int32_t kernel);

/* Copy the majorant grid (majorant_res[0]*[1]*[2] floats, x fastest) to host memory `out`
 * of capacity n floats.  Synchronous. */
int gpss_scene_get_majorants(gpss_scene_t scene, float* out, uint64_t n);

/* Forward render (Sec. 5, null-scattering path tracing) of samples [s0, s1) of every
 * pixel into image_dev (device, width*height floats, overwritten with the mean radiance
 * over those samples).  0 <= s0 < s1, and width*height*(s1-s0) < 2^31 paths per call (as for
 * every rendering call; split larger ranges, the chunks reproduce the same paths).
 * Each pixel's paths are summed exactly in fixed point (path radiance rounded to a multiple of
 * 2^-32, values from 2^24 on saturate, invalid ones add 0; see GPSS_CNT_NONFINITE), so the
 * image does not depend on the order in which paths finish and every kernel form gives the
 * same image.  The persistent form (default) keeps one 16-byte sum per pixel, allocated by
 * the scene's first render; the wavefront and one-thread forms also keep every path's
 * radiance (4 bytes per path of the call). */
int gpss_render(gpss_scene_t scene, float* image_dev, uint32_t s0, uint32_t s1,
                gpss_stream_t stream);

/* For callers that cannot allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid allocation): gpss_render by the persistent kernel, with its scratch
 * memory (the per-pixel fixed-point sums, 16 bytes per pixel, and the path counter) in a
 * fixed array of the library on each device instead of memory of the scene.  The call
 * allocates and frees nothing (it reads the scene record uploaded as gpss_render would).
 * At most 1048576 pixels (1024 x 1024); larger images return GPSS_ERR_INVALID_ARG.  The
 * array (16 MiB per device) is held until the process ends and is shared by every call on a
 * device: calls that overlap on one device race (each clears the array on its own stream
 * before rendering).  The scene's device must be current.  Same image as gpss_render. */
int gpss_render_noalloc(gpss_scene_t scene, float* image_dev, uint32_t s0, uint32_t s1,
                        gpss_stream_t stream);

/* As gpss_render but writes the per-path radiance to paths_dev (device,
 * width*height*(s1-s0) floats, pixel-major, then sample).  counters_dev (device, nullable)
 * receives GPSS_NCOUNTERS uint64 event counts added to its current contents. */
enum {
    GPSS_CNT_TRACK_STEPS = 0, GPSS_CNT_REAL = 1, GPSS_CNT_NEE_STEPS = 2,
    GPSS_CNT_VIOLATIONS = 3, GPSS_CNT_CAPPED = 4, GPSS_CNT_ESCAPED = 5,
    GPSS_CNT_TRUNCATED = 6, GPSS_CNT_CELLS = 7, GPSS_CNT_PHASE = 8, GPSS_CNT_NEE = 9,
    /* path radiances that are not a valid estimate: NaN, infinite or negative (an image adds
     * them as 0), and finite ones of at least 2^24 (an image adds them as 2^24) */
    GPSS_CNT_NONFINITE = 10, GPSS_CNT_SATURATED = 11,
    GPSS_NCOUNTERS = 16
};
int gpss_render_paths(gpss_scene_t scene, float* paths_dev, uint64_t* counters_dev,
                      uint32_t s0, uint32_t s1, gpss_stream_t stream);

/* Gradient of a scalar image loss (Sec. 5 estimator, differentiated by path replay).
 * dloss_dimage_dev: device, width*height floats, d loss / d image for the image of
 * gpss_render over [s0, s1).  grad_offset_dev: device, off_res[0]*[1]*[2] floats,
 * overwritten with d loss / d (mean-offset grid nodes); required iff the scene has an offset
 * grid.  grad_scalars_dev: device, 3 floats, overwritten with d loss / d (kernel variance,
 * lengthscale, albedo); the variance entry is 0 when the scene has a variance grid and the
 * albedo entry when albedo is per primitive.  The estimator is the forward one with every
 * sampling decision frozen at the current parameters; each path is traced (primal pass), then
 * replayed from its random-number streams by the same lane, which keeps the path's radiance
 * and its first light connections' contributions in registers and LDS: nothing is stored
 * per path in device memory, the call allocates nothing.  Gradients are accumulated with
 * floating-point atomics, so their last bits depend on scheduling. */
int gpss_render_adjoint(gpss_scene_t scene, const float* dloss_dimage_dev, float* grad_offset_dev,
                        float* grad_scalars_dev, uint32_t s0, uint32_t s1, gpss_stream_t stream);

/* Render n scenes of uneven size and sample count in one persistent launch, each over its
 * full [0, spp) into images_dev[i] (host array of device pointers, width*height floats
 * each; the array is read during the call only).  Images are identical to gpss_render's.
 * The work table (tiles of one scene's paths), a 16-byte fixed-point sum per pixel of the
 * batch and a hipGraph of [cursor reset, sum clear, persistent kernel, image kernel] are
 * built on the first call for a given scene list (which allocates and synchronizes) and
 * replayed afterwards; tile size and persistent grid come from the tuning cache written by
 * gpss_batch_autotune (file $GPSS_TUNE_CACHE, else ~/.cache/gpss_batch_tuning.txt), else 4096
 * paths and 12 waves per CU.  Later calls are asynchronous and ordered on `stream`: changed
 * scene records and image pointers are copied on `stream` from pinned staging, which waits
 * only when four earlier uploads of this list are still queued.  Calls on one scene list
 * must not overlap on different streams.  All scenes must live on one device. */
int gpss_render_batch(const gpss_scene_t* scenes, uint32_t n, float* const* images_dev,
                      gpss_stream_t stream);

/* Time every (tile size, waves per CU) candidate on this batch, keep the fastest for later
 * gpss_render_batch calls and append it to the tuning cache.  Outputs (nullable): the
 * chosen tile size, waves per CU and the batch time in ms. */
int gpss_batch_autotune(const gpss_scene_t* scenes, uint32_t n, float* const* images_dev,
                        gpss_stream_t stream, uint32_t* tile, uint32_t* waves_per_cu, float* ms);

/* Replace the differentiable parameters: mean-offset grid (device, nullable = unchanged),
 * kernel variance (> 0), lengthscale (> 0), albedo (in [0, 1]); rebuilds the majorant grid.
 * Asynchronous on `stream`. */
int gpss_scene_set_params(gpss_scene_t scene, const float* mean_offset_dev, float variance,
                          float lengthscale, float albedo, gpss_stream_t stream);

/* Evaluate the medium at n points for n directions (diagnostics and tests).
 * points_dev, dirs_dev: device, n x 3 floats.  out_dev: device, n x 8 floats:
 * mu, sigma (std), s = sigma/l, rho, sigma_proj(dir), sigma_t, ndf(dir as normal), albedo.
 * For a conditioned GP, mu and sigma are the posterior's and s is the isotropic spread the
 * proposal uses (root of a third of the trace of the gradient covariance given f = 0). */
int gpss_eval_medium(gpss_scene_t scene, const float* points_dev, const float* dirs_dev,
                     float* out_dev, uint64_t n, gpss_stream_t stream);

/* Trace n listed paths (diagnostics).  ids_dev: device, n x 2 uint32 (pixel, sample).
 * out_dev: device, n x (kmax * 16 + 1) floats; per real collision k < kmax, 16 floats:
 * position xyz, distance along the segment, tentative collisions of the segment,
 * (phase value, transmittance) for the directional then the point light, sampled half
 * vector xyz, its mixture pdf, the throughput weight, throughput after the vertex and
 * radiance after its next-event estimates; the last float is the path radiance. */
int gpss_debug_trace(gpss_scene_t scene, const uint32_t* ids_dev, uint32_t n, float* out_dev,
                     uint32_t kmax, gpss_stream_t stream);

const char* gpss_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GPSS_H */
