// C-ABI entry points of libgpss: argument validation, scene upload, scratch management and
// the host side of every call.  No exception leaves this file.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "gpss_internal.hpp"

namespace {
thread_local std::string g_last_error;

bool finite3(const float* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}
}  // namespace

namespace gpss {

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return GPSS_OK;
    if (e == hipErrorOutOfMemory) return set_error(GPSS_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return set_error(GPSS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int ensure_wavefront(gpss_scene* s, uint64_t npaths) {
    if (s->wf_cap >= npaths && s->wf_mem) return GPSS_OK;
    if (s->wf_mem) {
        int rc = check_hip(hipFree(s->wf_mem), "hipFree(wavefront)");
        s->wf_mem = nullptr;
        s->wf_cap = 0;
        if (rc) return rc;
    }
    // 6 doubles + 3 floats + 1 word + 6 floats + 5 queue words per path, plus counters
    const uint64_t n = npaths;
    const size_t bytes = n * (6 * 8 + 3 * 4 + 4 + 6 * 4 + 5 * 4) + 256 + 64 * 16;
    int rc = check_hip(hipMalloc(&s->wf_mem, bytes), "hipMalloc(wavefront)");
    if (rc) return rc;
    char* m = static_cast<char*>(s->wf_mem);
    auto take = [&m](size_t b) {
        char* r = m;
        m += (b + 255) & ~size_t(255);
        return r;
    };
    WfState& W = s->wf;
    W.ox = reinterpret_cast<double*>(take(8 * n));
    W.oy = reinterpret_cast<double*>(take(8 * n));
    W.oz = reinterpret_cast<double*>(take(8 * n));
    W.dx = reinterpret_cast<double*>(take(8 * n));
    W.dy = reinterpret_cast<double*>(take(8 * n));
    W.dz = reinterpret_cast<double*>(take(8 * n));
    W.beta = reinterpret_cast<float*>(take(4 * n));
    W.L = reinterpret_cast<float*>(take(4 * n));
    W.bounce = reinterpret_cast<uint32_t*>(take(4 * n));
    W.nee_c = reinterpret_cast<float*>(take(8 * n));
    W.nee_bp = reinterpret_cast<float*>(take(8 * n));
    W.nee_le = reinterpret_cast<float*>(take(8 * n));
    W.q_a = reinterpret_cast<uint32_t*>(take(4 * n));
    W.q_b = reinterpret_cast<uint32_t*>(take(4 * n));
    W.q_scatter = reinterpret_cast<uint32_t*>(take(4 * n));
    W.q_nee = reinterpret_cast<uint32_t*>(take(8 * n));
    W.cnt = reinterpret_cast<uint32_t*>(take(4 * kQNum));
    W.out = nullptr;
    s->wf_cap = npaths;
    if (!s->wf_grid) {
        int cus = 0;
        rc = device_cus(s->device, &cus);
        if (rc) return rc;
        s->wf_grid = (uint32_t)cus * 4u;
    }
    return GPSS_OK;
}

int device_cus(int device, int* cus) {
    int n = 0;
    int rc = check_hip(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device),
                       "hipDeviceGetAttribute");
    if (rc) return rc;
    *cus = n > 0 ? n : 1;
    return GPSS_OK;
}

// Device copy of the scene record read by the persistent kernels (through a pointer, which
// keeps the kernels' scalar registers free): re-uploaded after every change of `dev`, ordered
// on `stream` after the work already queued there.  The copy goes from a pinned staging
// record; the staging is rewritten only once its previous copy has completed (an event
// wait that blocks only when the previous upload is still queued).  The path counter, the
// record and the staging are allocated with the scene.
int ensure_sched(gpss_scene* s, hipStream_t stream) {
    if (s->dev_uploaded != s->dev_version) {
        int rc = check_hip(hipEventSynchronize(s->rec_event), "hipEventSynchronize(scene record)");
        if (rc) return rc;
        *s->h_rec = s->dev;
        rc = check_hip(hipMemcpyAsync(s->d_dev, s->h_rec, sizeof(SceneDev), hipMemcpyHostToDevice, stream),
                       "hipMemcpyAsync(scene record)");
        if (!rc) rc = check_hip(hipEventRecord(s->rec_event, stream), "hipEventRecord(scene record)");
        if (rc) return rc;
        s->dev_uploaded = s->dev_version;
    }
    return GPSS_OK;
}

// Per-pixel fixed-point accumulator of gpss_render (two 64-bit words per pixel), allocated on
// the scene's first render.
int ensure_acc(gpss_scene* s) {
    if (s->d_acc) return GPSS_OK;
    return check_hip(hipMalloc(&s->d_acc, 2 * s->n_pixels() * sizeof(unsigned long long)), "hipMalloc(accumulator)");
}

int ensure_scratch(gpss_scene* s, size_t floats) {
    if (s->scratch_floats >= floats) return GPSS_OK;
    if (s->d_scratch) {
        int rc = check_hip(hipFree(s->d_scratch), "hipFree(scratch)");
        s->d_scratch = nullptr;
        s->scratch_floats = 0;
        if (rc) return rc;
    }
    int rc = check_hip(hipMalloc(&s->d_scratch, floats * sizeof(float)), "hipMalloc(scratch)");
    if (rc) return rc;
    s->scratch_floats = floats;
    return GPSS_OK;
}

}  // namespace gpss

using gpss::check_hip;
using gpss::set_error;
using gpss::WfState;
using gpss::kQNum;

namespace {

int upload(const float* src, size_t n, float** dst);

int validate_desc(const gpss_scene_desc* D) {
    if (!D) return set_error(GPSS_ERR_INVALID_ARG, "desc is NULL");
    if (D->struct_size != sizeof(gpss_scene_desc))
        return set_error(GPSS_ERR_INVALID_ARG, "desc.struct_size %u != %zu", D->struct_size, sizeof(gpss_scene_desc));
    if (D->mean_kind < 0 || D->mean_kind > 2) return set_error(GPSS_ERR_INVALID_ARG, "mean_kind %d", D->mean_kind);
    if (D->mean_kind == GPSS_MEAN_SDF) {
        if (!D->prims || D->n_prims < 1 || D->n_prims > (uint32_t)gpss::kMaxPrims)
            return set_error(GPSS_ERR_INVALID_ARG, "SDF mean needs 1..%d primitives", gpss::kMaxPrims);
        for (uint32_t i = 0; i < D->n_prims; ++i) {
            const float* p = D->prims + 8 * i;
            if (!finite3(p, 8)) return set_error(GPSS_ERR_INVALID_ARG, "primitive %u not finite", i);
            if (p[0] != 0.0f && p[0] != 1.0f) return set_error(GPSS_ERR_INVALID_ARG, "primitive %u kind", i);
            const int nr = p[0] == 0.0f ? 1 : 3;
            for (int k = 0; k < nr; ++k)
                if (!(p[4 + k] > 0.0f)) return set_error(GPSS_ERR_INVALID_ARG, "primitive %u size", i);
            if (!(p[7] >= 0.0f && p[7] <= 1.0f)) return set_error(GPSS_ERR_INVALID_ARG, "primitive %u albedo", i);
        }
    }
    if (!std::isfinite(D->mean_const)) return set_error(GPSS_ERR_INVALID_ARG, "mean_const");
    auto grid_ok = [](const float* g, const uint32_t* res, bool positive, const char* name) -> int {
        for (int a = 0; a < 3; ++a)
            if (res[a] < 2 || res[a] > 1024) return set_error(GPSS_ERR_INVALID_ARG, "%s resolution", name);
        const uint64_t n = (uint64_t)res[0] * res[1] * res[2];
        for (uint64_t i = 0; i < n; ++i)
            if (!std::isfinite(g[i]) || (positive && !(g[i] > 0.0f)))
                return set_error(GPSS_ERR_INVALID_ARG, "%s value %llu", name, (unsigned long long)i);
        return GPSS_OK;
    };
    if (D->mean_offset) {
        int rc = grid_ok(D->mean_offset, D->off_res, false, "mean_offset");
        if (rc) return rc;
    }
    if (D->variance_grid) {
        int rc = grid_ok(D->variance_grid, D->var_res, true, "variance_grid");
        if (rc) return rc;
    } else if (!(D->variance > 0.0f) || !std::isfinite(D->variance)) {
        return set_error(GPSS_ERR_INVALID_ARG, "variance must be > 0");
    }
    if (!(D->lengthscale > 0.0f) || !std::isfinite(D->lengthscale))
        return set_error(GPSS_ERR_INVALID_ARG, "lengthscale must be > 0");
    if (!(D->lengthscale_n >= 0.0f) || !std::isfinite(D->lengthscale_n))
        return set_error(GPSS_ERR_INVALID_ARG, "lengthscale_n must be >= 0 (0: isotropic)");
    if (!(D->fresnel_eta >= 0.0f) || !(D->fresnel_k >= 0.0f) || !std::isfinite(D->fresnel_eta) ||
        !std::isfinite(D->fresnel_k))
        return set_error(GPSS_ERR_INVALID_ARG, "fresnel_eta and fresnel_k must be finite and >= 0");
    if (D->ndf_kind != GPSS_NDF_GENERALIZED && D->ndf_kind != GPSS_NDF_GGX)
        return set_error(GPSS_ERR_INVALID_ARG, "unknown ndf_kind %d", D->ndf_kind);
    if (D->ndf_kind == GPSS_NDF_GGX && D->mean_kind == GPSS_MEAN_CONST)
        return set_error(GPSS_ERR_INVALID_ARG, "the GGX macrofacet needs a mean with a gradient");
    if (D->ndf_kind == GPSS_NDF_GGX && D->lengthscale_n > 0.0f && D->lengthscale_n != D->lengthscale)
        return set_error(GPSS_ERR_INVALID_ARG, "the GGX macrofacet takes the isotropic kernel");
    if (!(D->albedo >= 0.0f && D->albedo <= 1.0f)) return set_error(GPSS_ERR_INVALID_ARG, "albedo not in [0,1]");
    if (!(D->mix_R >= 0.0f && D->mix_R <= 1.0f)) return set_error(GPSS_ERR_INVALID_ARG, "mix_R not in [0,1]");
    if (!finite3(D->bounds, 6)) return set_error(GPSS_ERR_INVALID_ARG, "bounds not finite");
    for (int a = 0; a < 3; ++a) {
        if (!(D->bounds[3 + a] > D->bounds[a])) return set_error(GPSS_ERR_INVALID_ARG, "empty bounds");
        if (D->majorant_res[a] < 1 || D->majorant_res[a] > 256)
            return set_error(GPSS_ERR_INVALID_ARG, "majorant_res must be 1..256");
    }
    if (!finite3(D->dir_light, 4) || !finite3(D->point_light, 4) || !std::isfinite(D->env_radiance))
        return set_error(GPSS_ERR_INVALID_ARG, "light values not finite");
    if (D->dir_light[3] < 0.0f || D->point_light[3] < 0.0f || D->env_radiance < 0.0f)
        return set_error(GPSS_ERR_INVALID_ARG, "negative light");
    if (D->dir_light[3] > 0.0f) {
        const float n = std::sqrt(D->dir_light[0] * D->dir_light[0] + D->dir_light[1] * D->dir_light[1] +
                                  D->dir_light[2] * D->dir_light[2]);
        if (std::fabs(n - 1.0f) > 1e-3f) return set_error(GPSS_ERR_INVALID_ARG, "dir_light direction not unit");
    }
    if (D->cam_kind != GPSS_CAM_ORTHO && D->cam_kind != GPSS_CAM_PINHOLE)
        return set_error(GPSS_ERR_INVALID_ARG, "cam_kind");
    if (!finite3(D->cam_eye, 3) || !finite3(D->cam_target, 3) || !finite3(D->cam_up, 3))
        return set_error(GPSS_ERR_INVALID_ARG, "camera not finite");
    if (D->cam_kind == GPSS_CAM_PINHOLE && !(D->cam_fov_deg > 0.0f && D->cam_fov_deg < 180.0f))
        return set_error(GPSS_ERR_INVALID_ARG, "cam_fov_deg");
    if (D->cam_kind == GPSS_CAM_ORTHO && !(D->cam_window[0] > 0.0f && D->cam_window[1] > 0.0f))
        return set_error(GPSS_ERR_INVALID_ARG, "cam_window");
    if (D->width < 1 || D->height < 1 || D->width > 16384 || D->height > 16384)
        return set_error(GPSS_ERR_INVALID_ARG, "resolution");
    if (D->spp < 1) return set_error(GPSS_ERR_INVALID_ARG, "spp must be >= 1");
    if (D->max_depth > 65534) return set_error(GPSS_ERR_INVALID_ARG, "max_depth > 65534");
    if (D->n_obs > 0) {
        if (D->n_obs > (uint32_t)gpss::kMaxObs)
            return set_error(GPSS_ERR_INVALID_ARG, "n_obs %u > %d", D->n_obs, gpss::kMaxObs);
        if (!D->observations) return set_error(GPSS_ERR_INVALID_ARG, "observations is NULL");
        if (!finite3(D->observations, 4 * (int)D->n_obs)) return set_error(GPSS_ERR_INVALID_ARG, "observations not finite");
        if (!(D->obs_noise > 0.0f) || !std::isfinite(D->obs_noise))
            return set_error(GPSS_ERR_INVALID_ARG, "obs_noise must be > 0");
        // below this the single-precision posterior variance sigma^2 - |L^-1 k|^2 at an
        // observation (about obs_noise) would be lost in the cancellation
        if (!D->variance_grid && D->obs_noise < 1e-4f * D->variance)
            return set_error(GPSS_ERR_INVALID_ARG, "obs_noise must be >= 1e-4 x variance");
        if (D->variance_grid || D->mean_offset || D->ndf_kind != GPSS_NDF_GENERALIZED ||
            (D->lengthscale_n > 0.0f && D->lengthscale_n != D->lengthscale))
            return set_error(GPSS_ERR_UNSUPPORTED, "conditioning takes a scalar variance, no mean offset grid, the "
                                                   "isotropic kernel and the generalized NDF");
    }
    return GPSS_OK;
}

// Host SDF of one primitive row (kind, cx, cy, cz, a, b, c, albedo) in double.
double sdf_prim_host(const float* p, const double x[3]) {
    const double v[3] = {x[0] - (double)p[1], x[1] - (double)p[2], x[2] - (double)p[3]};
    if (p[0] == 0.0f) return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - (double)p[4];
    const double q[3] = {std::fabs(v[0]) - (double)p[4], std::fabs(v[1]) - (double)p[5], std::fabs(v[2]) - (double)p[6]};
    const double qmax = std::fmax(q[0], std::fmax(q[1], q[2]));
    if (qmax > 0.0) {
        const double a = std::fmax(q[0], 0.0), b = std::fmax(q[1], 0.0), c = std::fmax(q[2], 0.0);
        return std::sqrt(a * a + b * b + c * c);
    }
    return qmax;
}

// Conditioning on point observations (Eq. condition_gp), prepared once in double:
// K = kappa(C, C) + s_n^2 I = L L^T, alpha = K^-1 (m - mu(C)) and L^-1.  The device takes
// (position - origin, alpha) and L^-1 (padded to kMaxObs x kMaxObs) in single precision, the
// majorant kernel positions, alpha and L^-1 in double.
int prepare_observations(gpss_scene* s, const gpss_scene_desc& D) {
    const int n = (int)D.n_obs;
    const double s2 = D.variance, l = D.lengthscale, noise = D.obs_noise;
    std::vector<double> X(3 * n), m(n), K((size_t)n * n), Li((size_t)n * n, 0.0), alpha(n);
    for (int j = 0; j < n; ++j) {
        for (int a = 0; a < 3; ++a) X[3 * j + a] = D.observations[4 * j + a];
        m[j] = D.observations[4 * j + 3];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) d2 += (X[3 * i + a] - X[3 * j + a]) * (X[3 * i + a] - X[3 * j + a]);
            K[(size_t)i * n + j] = s2 * std::exp(-d2 / (2.0 * l * l)) + (i == j ? noise : 0.0);
        }
    // Cholesky (lower) in place
    for (int j = 0; j < n; ++j) {
        double d = K[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= K[(size_t)j * n + k] * K[(size_t)j * n + k];
        if (!(d > 0.0)) return set_error(GPSS_ERR_INVALID_ARG, "observation covariance not positive definite");
        d = std::sqrt(d);
        K[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = K[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= K[(size_t)i * n + k] * K[(size_t)j * n + k];
            K[(size_t)i * n + j] = v / d;
        }
    }
    // L^-1 column by column (forward substitution on unit vectors)
    for (int c = 0; c < n; ++c)
        for (int i = c; i < n; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) v -= K[(size_t)i * n + k] * Li[(size_t)k * n + c];
            Li[(size_t)i * n + c] = v / K[(size_t)i * n + i];
        }
    // residuals m - mu(C) of the prior mean, then alpha = L^-T L^-1 r
    for (int j = 0; j < n; ++j) {
        const double* x = &X[3 * j];
        double mu = 0.0;
        if (D.mean_kind == GPSS_MEAN_PLANE) {
            mu = x[2];
        } else if (D.mean_kind == GPSS_MEAN_CONST) {
            mu = D.mean_const;
        } else {
            mu = INFINITY;
            for (uint32_t i = 0; i < D.n_prims; ++i) mu = std::fmin(mu, sdf_prim_host(D.prims + 8 * i, x));
        }
        alpha[j] = m[j] - mu;
    }
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) {
        double v = 0.0;
        for (int k = 0; k <= i; ++k) v += Li[(size_t)i * n + k] * alpha[k];
        y[i] = v;
    }
    for (int i = 0; i < n; ++i) {
        double v = 0.0;
        for (int k = i; k < n; ++k) v += Li[(size_t)k * n + i] * y[k];
        alpha[i] = v;
    }
    float origin[3];
    for (int a = 0; a < 3; ++a) origin[a] = 0.5f * (D.bounds[a] + D.bounds[3 + a]);
    // kMaxObs float4 (position - origin, alpha; zeros beyond n), then the lower triangle of
    // L^-1 row by row as float4 (L^-1_ij, L^-1_ij (x_j - origin)), formed in double and
    // rounded once, each row zero-padded to 4 cond_row_blocks(i) entries
    std::vector<float> F(4 * gpss::kMaxObs + 4 * (size_t)gpss::kCondTriEntries, 0.0f);
    for (int j = 0; j < n; ++j) {
        for (int a = 0; a < 3; ++a) F[4 * j + a] = D.observations[4 * j + a] - origin[a];
        F[4 * j + 3] = (float)alpha[j];
    }
    size_t e = 4 * gpss::kMaxObs;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 4 * gpss::cond_row_blocks(i); ++j, e += 4) {
            if (j > i) continue;   // padding stays zero
            const double v = Li[(size_t)i * n + j];
            F[e] = (float)v;
            for (int a = 0; a < 3; ++a) F[e + 1 + a] = (float)(v * ((double)D.observations[4 * j + a] - (double)origin[a]));
        }
    std::vector<double> Dd;
    Dd.insert(Dd.end(), X.begin(), X.end());
    Dd.insert(Dd.end(), alpha.begin(), alpha.end());
    Dd.insert(Dd.end(), Li.begin(), Li.end());
    int rc = upload(F.data(), F.size(), &s->d_obs);
    if (!rc) rc = check_hip(hipMalloc(&s->d_obs_d, Dd.size() * sizeof(double)), "hipMalloc(observations)");
    if (!rc)
        rc = check_hip(hipMemcpy(s->d_obs_d, Dd.data(), Dd.size() * sizeof(double), hipMemcpyHostToDevice),
                       "hipMemcpy observations");
    for (int a = 0; a < 3; ++a) s->dev.obs_c[a] = origin[a];
    return rc;
}

int upload(const float* src, size_t n, float** dst) {
    int rc = check_hip(hipMalloc(dst, n * sizeof(float)), "hipMalloc");
    if (rc) return rc;
    return check_hip(hipMemcpy(*dst, src, n * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy H2D");
}

void free_scene(gpss_scene* s) {
    if (!s) return;
    (void)hipFree(s->d_prims);
    (void)hipFree(s->d_cand);
    (void)hipFree(s->d_maj16);
    (void)hipFree(s->d_offset);
    (void)hipFree(s->d_var);
    (void)hipFree(s->d_maj);
    (void)hipFree(s->d_obs);
    (void)hipFree(s->d_obs_d);
    (void)hipFree(s->d_scratch);
    (void)hipFree(s->wf_mem);
    (void)hipFree(s->d_head);
    (void)hipFree(s->d_dev);
    (void)hipFree(s->d_acc);
    if (s->h_rec) (void)hipHostFree(s->h_rec);
    if (s->rec_event) (void)hipEventDestroy(s->rec_event);
    delete s;
}

// (l / l_n)^2 - 1: the kernel's anisotropy as the scene record carries it (0: isotropic).
float aniso_k(const gpss_scene_desc& D) {
    if (!(D.lengthscale_n > 0.0f) || D.lengthscale_n == D.lengthscale) return 0.0f;
    const float r = D.lengthscale / D.lengthscale_n;
    return r * r - 1.0f;
}

// Scheduling policy from the scene's typical gradient spread sigma / l: the variance, or the
// median node of the variance grid (where most of a grid's medium is; its largest node picked
// the rough policy for the 1024^2 mixed scene, 4 % slower there than the smooth one), over the
// shorter of the two lengthscales.
void set_policy(gpss_scene* s) {
    const gpss_scene_desc& D = s->desc;
    float v = D.variance;
    if (!s->var_h.empty()) {
        std::vector<float> t(s->var_h);
        std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
        v = t[t.size() / 2];
    }
    const float l = D.lengthscale_n > 0.0f ? std::min(D.lengthscale, D.lengthscale_n) : D.lengthscale;
    const gpss::SchedPolicy p = gpss::sched_policy(std::sqrt(v) / l);
    s->dev.walk_steps = p.walk_steps;
    s->dev.scatter_min = p.scatter_min;
}

// Per majorant cell, the primitives that can be the union's minimum somewhere in the cell
// (SceneDev::prim_cand).  Each primitive's SDF is 1-Lipschitz, so over the cell widened by a
// margin it stays within r of its value at the centre (r: half the widened cell's diagonal).
// A primitive whose lower bound d_p - r exceeds the smallest upper bound min_q d_q + r by more
// than the margin is above the minimum everywhere in the cell, so it can neither be the
// minimum nor tie with it.  The margins (1e-4 of the box) are far above the single-precision
// rounding of a point's cell index and of its distances.  Cells with more than three
// candidates, and unions of fewer than four or more than sixteen primitives, take all.
constexpr uint32_t kCandMinPrims = 4, kCandMaxPrims = 16, kCandMax = 3;

static double sdf_host(const float* p, const double x[3]) {
    double v[3], q[3];
    for (int a = 0; a < 3; ++a) v[a] = x[a] - (double)p[1 + a];
    if (p[0] < 0.5f) return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - (double)p[4];
    double out = 0.0, qmax = -INFINITY;
    for (int a = 0; a < 3; ++a) {
        q[a] = std::fabs(v[a]) - (double)p[4 + a];
        qmax = std::max(qmax, q[a]);
        out += q[a] > 0.0 ? q[a] * q[a] : 0.0;
    }
    return qmax > 0.0 ? std::sqrt(out) : qmax;
}

static int build_candidates(gpss_scene* s) {
    const gpss_scene_desc& D = s->desc;
    const uint32_t n = D.n_prims;
    if (D.mean_kind != GPSS_MEAN_SDF || n < kCandMinPrims || n > kCandMaxPrims) return GPSS_OK;
    const uint32_t M[3] = {D.majorant_res[0], D.majorant_res[1], D.majorant_res[2]};
    double lo[3], cw[3], ext_max = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double ext = (double)D.bounds[3 + a] - (double)D.bounds[a];
        lo[a] = D.bounds[a];
        cw[a] = ext / M[a];
        ext_max = std::max(ext_max, ext);
    }
    const double margin = 1e-4 * ext_max;
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) r2 += (0.5 * cw[a] + margin) * (0.5 * cw[a] + margin);
    const double r = std::sqrt(r2);
    std::vector<uint16_t> tab((size_t)M[0] * M[1] * M[2]);
    std::vector<double> d(n);
    size_t cell = 0;
    for (uint32_t iz = 0; iz < M[2]; ++iz)
        for (uint32_t iy = 0; iy < M[1]; ++iy)
            for (uint32_t ix = 0; ix < M[0]; ++ix, ++cell) {
                const double c[3] = {lo[0] + (ix + 0.5) * cw[0], lo[1] + (iy + 0.5) * cw[1], lo[2] + (iz + 0.5) * cw[2]};
                double dmin = INFINITY;
                for (uint32_t p = 0; p < n; ++p) {
                    d[p] = sdf_host(s->prims_h.data() + 8 * p, c);
                    dmin = std::min(dmin, d[p]);
                }
                uint32_t word = 0, cnt = 0;
                for (uint32_t p = 0; p < n; ++p) {
                    if (d[p] - r > dmin + r + margin) continue;
                    if (cnt < kCandMax) word |= p << (2 + 4 * cnt);
                    ++cnt;
                }
                tab[cell] = (uint16_t)(cnt <= kCandMax ? (word | cnt) : 0u);
            }
    int rc = check_hip(hipMalloc(&s->d_cand, tab.size() * sizeof(uint16_t)), "hipMalloc(candidates)");
    if (!rc)
        rc = check_hip(hipMemcpy(s->d_cand, tab.data(), tab.size() * sizeof(uint16_t), hipMemcpyHostToDevice),
                       "hipMemcpy(candidates)");
    return rc;
}

void fill_dev(gpss_scene* s) {
    const gpss_scene_desc& D = s->desc;
    gpss::SceneDev& V = s->dev;
    V.mean_kind = D.mean_kind;
    V.mean_const = D.mean_const;
    V.n_prims = D.mean_kind == GPSS_MEAN_SDF ? (int)D.n_prims : 0;
    V.prims = reinterpret_cast<const float4*>(s->d_prims);
    V.offset = s->d_offset;
    V.var_grid = s->d_var;
    V.variance = D.variance;
    V.lengthscale = D.lengthscale;
    V.sigma0 = std::sqrt(D.variance);
    V.s0 = V.sigma0 / D.lengthscale;
    V.inv_l = 1.0f / D.lengthscale;
    set_policy(s);
    V.aniso_k = aniso_k(D);
    V.ggx = D.ndf_kind == GPSS_NDF_GGX;
    V.f_eta = D.fresnel_eta;
    V.f_k = D.fresnel_k;
    V.n_obs = (int)D.n_obs;
    V.obs = reinterpret_cast<const float4*>(s->d_obs);
    V.obs_tri = s->d_obs ? reinterpret_cast<const float4*>(s->d_obs + 4 * gpss::kMaxObs) : nullptr;
    V.albedo = D.albedo;
    V.albedo_per_prim = D.albedo_per_prim ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        const double lo = D.bounds[a], hi = D.bounds[3 + a], ext = hi - lo;
        V.lo[a] = D.bounds[a];
        V.hi[a] = D.bounds[3 + a];
        V.M[a] = (int)D.majorant_res[a];
        V.cw[a] = (float)(ext / D.majorant_res[a]);
        V.inv_cw[a] = (float)(D.majorant_res[a] / ext);
        V.lo_d[a] = lo;
        V.hi_d[a] = hi;
        V.cw_d[a] = ext / D.majorant_res[a];
        V.inv_cw_d[a] = D.majorant_res[a] / ext;
        V.off_res[a] = (int)D.off_res[a];
        V.off_scale[a] = D.mean_offset || s->d_offset ? (float)((D.off_res[a] - 1) / ext) : 0.0f;
        V.var_res[a] = (int)D.var_res[a];
        V.var_scale[a] = s->d_var ? (float)((D.var_res[a] - 1) / ext) : 0.0f;
        V.off_scale_d[a] = D.mean_offset || s->d_offset ? (D.off_res[a] - 1) / ext : 0.0;
        V.var_scale_d[a] = s->d_var ? (D.var_res[a] - 1) / ext : 0.0;
    }
    V.maj16 = s->d_maj16;
    V.prim_cand = s->d_cand;
    V.R = D.mix_R;
    for (int k = 0; k < 4; ++k) {
        V.dl[k] = D.dir_light[k];
        V.pl[k] = D.point_light[k];
    }
    V.env = D.env_radiance;
    V.cam_kind = D.cam_kind;
    // camera frame in double from the float inputs
    double eye[3], fwd[3], up[3], right[3], upc[3];
    for (int k = 0; k < 3; ++k) {
        eye[k] = D.cam_eye[k];
        fwd[k] = (double)D.cam_target[k] - (double)D.cam_eye[k];
        up[k] = D.cam_up[k];
    }
    auto nrm = [](double* v) {
        const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        v[0] /= n; v[1] /= n; v[2] /= n;
    };
    auto crs = [](const double* a, const double* b, double* r) {
        r[0] = a[1] * b[2] - a[2] * b[1];
        r[1] = a[2] * b[0] - a[0] * b[2];
        r[2] = a[0] * b[1] - a[1] * b[0];
    };
    nrm(fwd);
    crs(fwd, up, right);
    nrm(right);
    crs(right, fwd, upc);
    for (int k = 0; k < 3; ++k) {
        V.eye[k] = eye[k];
        V.fwd[k] = fwd[k];
        V.right[k] = right[k];
        V.upc[k] = upc[k];
    }
    V.tan_half = std::tan(0.5 * (double)D.cam_fov_deg * 3.14159265358979323846 / 180.0);
    V.aspect = (double)D.width / D.height;
    V.win[0] = D.cam_window[0];
    V.win[1] = D.cam_window[1];
    V.W = (int)D.width;
    V.H = (int)D.height;
    V.max_depth = (int)D.max_depth;
    V.key0 = (uint32_t)(D.seed & 0xFFFFFFFFull);
    V.key1 = (uint32_t)(D.seed >> 32) ^ D.scene_id;
}

// One call renders at most 2^31 - 1 paths (32-bit path slots in the kernels); checked before
// any allocation so that an oversized range fails fast with a clear message.
}  // namespace

namespace gpss {
int check_path_count(const gpss_scene* s, uint32_t s0, uint32_t s1) {
    if (s1 <= s0) return set_error(GPSS_ERR_INVALID_ARG, "empty sample range [%u, %u)", s0, s1);
    const uint64_t n = s->n_pixels() * (uint64_t)(s1 - s0);
    if (n > 0x7FFFFFFFull)
        return set_error(GPSS_ERR_INVALID_ARG, "%llu paths in one call: at most 2^31 - 1 (split [s0, s1))",
                         (unsigned long long)n);
    return GPSS_OK;
}
}  // namespace gpss

extern "C" {

const char* gpss_last_error(void) { return g_last_error.c_str(); }

int gpss_scene_create(const gpss_scene_desc* desc, gpss_scene_t* out) {
    gpss::Range range("gpss_scene_create");
    try {
        if (!out) return set_error(GPSS_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        int rc = validate_desc(desc);
        if (rc) return rc;
        gpss_scene* s = new (std::nothrow) gpss_scene();
        if (!s) return set_error(GPSS_ERR_OOM, "host allocation");
        s->desc = *desc;
        rc = check_hip(hipGetDevice(&s->device), "hipGetDevice");
        const gpss_scene_desc& D = *desc;
        if (!rc && D.mean_kind == GPSS_MEAN_SDF) {
            s->prims_h.assign(D.prims, D.prims + 8 * D.n_prims);
            rc = upload(s->prims_h.data(), s->prims_h.size(), &s->d_prims);
            if (!rc) rc = build_candidates(s);
        }
        if (!rc && D.mean_offset) {
            const size_t n = (size_t)D.off_res[0] * D.off_res[1] * D.off_res[2];
            s->offset_h.assign(D.mean_offset, D.mean_offset + n);
            rc = upload(s->offset_h.data(), n, &s->d_offset);
        }
        if (!rc && D.variance_grid) {
            const size_t n = (size_t)D.var_res[0] * D.var_res[1] * D.var_res[2];
            s->var_h.assign(D.variance_grid, D.variance_grid + n);
            rc = upload(s->var_h.data(), n, &s->d_var);
        }
        if (!rc && D.n_obs > 0) rc = prepare_observations(s, D);
        const size_t nmaj = (size_t)D.majorant_res[0] * D.majorant_res[1] * D.majorant_res[2];
        if (!rc) rc = check_hip(hipMalloc(&s->d_maj, nmaj * sizeof(float)), "hipMalloc(majorants)");
        if (!rc) rc = check_hip(hipMalloc(&s->d_maj16, nmaj * sizeof(uint16_t)), "hipMalloc(majorants16)");
        s->desc.prims = nullptr;
        s->desc.mean_offset = nullptr;
        s->desc.variance_grid = nullptr;
        s->desc.observations = nullptr;
        if (!rc) {
            fill_dev(s);
            rc = gpss::launch_majorants(s, nullptr);
        }
        if (!rc) {
            s->maj_h.resize(nmaj);
            rc = check_hip(hipMemcpy(s->maj_h.data(), s->d_maj, nmaj * sizeof(float), hipMemcpyDeviceToHost),
                           "hipMemcpy majorants");
        }
        // persistent-kernel state: path counter, device record (uploaded here) and its staging
        if (!rc) rc = check_hip(hipMalloc(&s->d_head, 64), "hipMalloc(path counter)");
        if (!rc) rc = check_hip(hipMalloc(&s->d_dev, sizeof(gpss::SceneDev)), "hipMalloc(scene record)");
        if (!rc) rc = check_hip(hipHostMalloc(reinterpret_cast<void**>(&s->h_rec), sizeof(gpss::SceneDev)),
                                "hipHostMalloc(scene record)");
        if (!rc) rc = check_hip(hipEventCreateWithFlags(&s->rec_event, hipEventDisableTiming), "hipEventCreate");
        if (!rc) rc = check_hip(hipMemcpy(s->d_dev, &s->dev, sizeof(gpss::SceneDev), hipMemcpyHostToDevice),
                                "hipMemcpy(scene record)");
        if (!rc) {
            s->dev_uploaded = s->dev_version;
            int cus = 0;
            rc = gpss::device_cus(s->device, &cus);
            s->sched_grid = (uint32_t)cus * (uint32_t)gpss::sched_waves_per_simd();
        }
        if (rc) {
            free_scene(s);
            return rc;
        }
        s->spp = D.spp;
        *out = s;
        return GPSS_OK;
    } catch (...) {
        return set_error(GPSS_ERR_OOM, "unexpected host exception in gpss_scene_create");
    }
}

int gpss_scene_destroy(gpss_scene_t scene) {
    if (!scene) return set_error(GPSS_ERR_INVALID_ARG, "scene is NULL");
    gpss::forget_scene_plans(scene);
    free_scene(scene);
    return GPSS_OK;
}

int gpss_scene_set_kernel(gpss_scene_t scene, int32_t kernel) {
    if (!scene) return set_error(GPSS_ERR_INVALID_ARG, "scene is NULL");
    if (kernel != GPSS_KERNEL_AUTO && kernel != GPSS_KERNEL_MEGA && kernel != GPSS_KERNEL_WAVEFRONT &&
        kernel != GPSS_KERNEL_PERSISTENT)
        return set_error(GPSS_ERR_INVALID_ARG, "unknown kernel %d", kernel);
    scene->kernel = kernel;
    return GPSS_OK;
}

int gpss_scene_get_majorants(gpss_scene_t scene, float* out, uint64_t n) {
    if (!scene || !out) return set_error(GPSS_ERR_INVALID_ARG, "NULL argument");
    if (scene->maj_h_stale) {
        int rc = check_hip(hipMemcpy(scene->maj_h.data(), scene->d_maj, scene->maj_h.size() * sizeof(float),
                                     hipMemcpyDeviceToHost),
                           "hipMemcpy majorants");
        if (rc) return rc;
        scene->maj_h_stale = false;
    }
    if (n < scene->maj_h.size()) return set_error(GPSS_ERR_INVALID_ARG, "output holds %llu < %zu floats",
                                                  (unsigned long long)n, scene->maj_h.size());
    std::memcpy(out, scene->maj_h.data(), scene->maj_h.size() * sizeof(float));
    return GPSS_OK;
}

int gpss_render_paths(gpss_scene_t scene, float* paths_dev, uint64_t* counters_dev, uint32_t s0, uint32_t s1,
                      gpss_stream_t stream) {
    gpss::Range range("gpss_render_paths");
    if (!scene || !paths_dev) return set_error(GPSS_ERR_INVALID_ARG, "NULL argument");
    if (int rc = gpss::check_path_count(scene, s0, s1)) return rc;
    return gpss::launch_render_paths(scene, paths_dev, counters_dev, s0, s1 - s0,
                                     reinterpret_cast<hipStream_t>(stream));
}

int gpss_render(gpss_scene_t scene, float* image_dev, uint32_t s0, uint32_t s1, gpss_stream_t stream) {
    gpss::Range range("gpss_render");
    if (!scene || !image_dev) return set_error(GPSS_ERR_INVALID_ARG, "NULL argument");
    if (int rc = gpss::check_path_count(scene, s0, s1)) return rc;
    const uint32_t ns = s1 - s0;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (scene->kernel == GPSS_KERNEL_MEGA || scene->kernel == GPSS_KERNEL_WAVEFRONT) {
        // these forms keep per-path radiances, reduced per pixel afterwards
        int rc = gpss::ensure_scratch(scene, (size_t)scene->n_pixels() * ns);
        if (!rc) rc = gpss::launch_render_paths(scene, scene->d_scratch, nullptr, s0, ns, st);
        if (!rc) rc = gpss::launch_reduce(scene, scene->d_scratch, image_dev, ns, st);
        return rc;
    }
    // persistent form: each path adds to its pixel's fixed-point sum (O(pixels) memory)
    int rc = gpss::ensure_acc(scene);
    if (!rc) rc = gpss::launch_acc_clear(scene->d_acc, scene->n_pixels(), st);
    if (!rc) rc = gpss::sched_render(scene, nullptr, scene->d_acc, nullptr, s0, ns, st);
    if (!rc) rc = gpss::launch_acc_finalize(scene->d_acc, image_dev, ns, scene->n_pixels(), st);
    return rc;
}

int gpss_scene_set_params(gpss_scene_t scene, const float* mean_offset_dev, float variance, float lengthscale,
                          float albedo, gpss_stream_t stream) {
    gpss::Range range("gpss_scene_set_params");
    if (!scene) return set_error(GPSS_ERR_INVALID_ARG, "scene is NULL");
    if (scene->dev.n_obs > 0)
        return set_error(GPSS_ERR_UNSUPPORTED, "parameters of a conditioned GP are fixed at creation");
    if (mean_offset_dev && !scene->d_offset)
        return set_error(GPSS_ERR_INVALID_ARG, "scene has no mean-offset grid");
    if (!(variance > 0.0f) || !std::isfinite(variance)) return set_error(GPSS_ERR_INVALID_ARG, "variance must be > 0");
    if (!(lengthscale > 0.0f) || !std::isfinite(lengthscale))
        return set_error(GPSS_ERR_INVALID_ARG, "lengthscale must be > 0");
    if (!(albedo >= 0.0f && albedo <= 1.0f)) return set_error(GPSS_ERR_INVALID_ARG, "albedo not in [0,1]");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (mean_offset_dev) {
        const size_t n = (size_t)scene->desc.off_res[0] * scene->desc.off_res[1] * scene->desc.off_res[2];
        int rc = check_hip(hipMemcpyAsync(scene->d_offset, mean_offset_dev, n * sizeof(float),
                                          hipMemcpyDeviceToDevice, st),
                           "hipMemcpyAsync(offset)");
        if (rc) return rc;
    }
    scene->desc.variance = variance;
    scene->desc.lengthscale = lengthscale;
    scene->desc.albedo = albedo;
    scene->dev.variance = variance;
    scene->dev.lengthscale = lengthscale;
    scene->dev.sigma0 = std::sqrt(variance);
    scene->dev.s0 = scene->dev.sigma0 / lengthscale;
    scene->dev.inv_l = 1.0f / lengthscale;
    set_policy(scene);
    scene->dev.aniso_k = aniso_k(scene->desc);
    scene->dev.albedo = albedo;
    scene->dev_version++;
    scene->maj_h_stale = true;
    return gpss::launch_majorants(scene, st);
}

int gpss_render_adjoint(gpss_scene_t scene, const float* dloss_dimage_dev, float* grad_offset_dev,
                        float* grad_scalars_dev, uint32_t s0, uint32_t s1, gpss_stream_t stream) {
    gpss::Range range("gpss_render_adjoint");
    if (!scene || !dloss_dimage_dev || !grad_scalars_dev) return set_error(GPSS_ERR_INVALID_ARG, "NULL argument");
    if (int rc = gpss::check_path_count(scene, s0, s1)) return rc;
    if (scene->d_offset && !grad_offset_dev)
        return set_error(GPSS_ERR_INVALID_ARG, "scene has a mean-offset grid: grad_offset_dev is required");
    if (scene->dev.aniso_k != 0.0f || scene->dev.ggx || scene->dev.n_obs > 0)
        return set_error(GPSS_ERR_UNSUPPORTED, "the adjoint supports the unconditioned generalized macrofacet "
                                               "with the isotropic kernel only");
    return gpss::launch_adjoint(scene, dloss_dimage_dev, grad_offset_dev, grad_scalars_dev, s0, s1 - s0,
                                reinterpret_cast<hipStream_t>(stream));
}

int gpss_render_batch(const gpss_scene_t* scenes, uint32_t n, float* const* images_dev, gpss_stream_t stream) {
    gpss::Range range("gpss_render_batch");
    try {
        return gpss::render_batch(scenes, n, images_dev, reinterpret_cast<hipStream_t>(stream));
    } catch (...) {
        return set_error(GPSS_ERR_OOM, "unexpected host exception in gpss_render_batch");
    }
}

int gpss_batch_autotune(const gpss_scene_t* scenes, uint32_t n, float* const* images_dev, gpss_stream_t stream,
                        uint32_t* tile, uint32_t* waves_per_cu, float* ms) {
    gpss::Range range("gpss_batch_autotune");
    try {
        return gpss::autotune_batch(scenes, n, images_dev, reinterpret_cast<hipStream_t>(stream), tile,
                                    waves_per_cu, ms);
    } catch (...) {
        return set_error(GPSS_ERR_OOM, "unexpected host exception in gpss_batch_autotune");
    }
}

int gpss_eval_medium(gpss_scene_t scene, const float* points_dev, const float* dirs_dev, float* out_dev,
                     uint64_t n, gpss_stream_t stream) {
    if (!scene || !points_dev || !dirs_dev || !out_dev) return set_error(GPSS_ERR_INVALID_ARG, "NULL argument");
    if (n == 0) return GPSS_OK;
    return gpss::launch_eval(scene, points_dev, dirs_dev, out_dev, n, reinterpret_cast<hipStream_t>(stream));
}

int gpss_debug_trace(gpss_scene_t scene, const uint32_t* ids_dev, uint32_t n, float* out_dev, uint32_t kmax,
                     gpss_stream_t stream) {
    if (!scene || !ids_dev || !out_dev) return set_error(GPSS_ERR_INVALID_ARG, "NULL argument");
    if (kmax < 1 || kmax > 65535) return set_error(GPSS_ERR_INVALID_ARG, "kmax must be 1..65535");
    if (n == 0) return GPSS_OK;
    return gpss::launch_debug_trace(scene, ids_dev, n, out_dev, (int)kmax, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
