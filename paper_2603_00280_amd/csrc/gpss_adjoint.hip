// Path-replay adjoint of the forward tracer.
//
// The estimator differentiated is the frozen-sampling form of the forward tracer: every
// sampling decision (tentative-collision positions, real/null choices, Russian roulette,
// phase samples) is taken at the current parameters theta0, and only the weights depend
// on theta.  At theta0 it equals the forward estimator.  A path's radiance is a sum of
// contributions C_k, each a product of factors:
//   null collision        (m - sigma_t) / (m - sigma_t0)
//   real collision        sigma_t / sigma_t0
//   phase weight          albedo <v, w_m> D(w_m) / (sigma(d) pdf0)
//   light connection      albedo D(w_h) / (4 sigma(d)) * prod (1 - sigma_t / m) * Le
// (sigma(d) of a real collision cancels against the phase weight and the light
// connection).  d C_k = C_k sum over its factors of d log(factor), so a factor contributes
// d log(factor) times the radiance of all contributions that contain it.  Each path is traced
// twice by the same thread (or lane): a primal pass, the forward tracer's own, gives its
// radiance L; a replay of the same random streams then carries the remaining radiance
// L_rem = L - (contributions already passed), and adds
//   nulls before vertex k:   -sigma_t / (m - sigma_t) d log sigma_t        x L_rem
//   vertex k:                d log rho + d log albedo                      x L_rem
//                            d log D(w_h, light)                           x C_k,light
//                            sum over the shadow ray -sigma_t/(m-sigma_t) d log sigma_t  x C_k,light
//                            d log D(w_m)                                  x (L_rem - C_k)
// to the gradient, weighted by dloss/dimage of the pixel over the number of samples.
// Nothing is stored per path outside the thread: memory is the gradient and the caller's
// d loss / d image (O(pixels)).
#include "gpss_internal.hpp"
#include "gpss_grad.hpp"
#include "gpss_sched.hpp"
#include "gpss_trace.hpp"

namespace gpss {

// Replay of one shadow ray: coefficient coef on d log of its transmittance estimate.
__device__ void ratio_track_grad(const SceneDev& S, D3 o, D3 d, float3 df, double t1, Rng& rng, float coef,
                                 float* grad_off, GradAcc& acc) {
    PathStats st;
    Segment sg;
    sg.begin<false>(S, o, d, 0.0, t1, rng, st);
    float Tr = 1.0f;
    for (;;) {
        const int ev = sg.step<false>(S, st);
        if (ev == kCell) continue;
        if (ev == kEnd) return;
        sg.advance();
        if (++sg.steps > kStepCap) return;
        const float3 x = sg.pos();
        const PointQ q = eval_point(S, x);
        const float sig = sigma_t_of(q, df);
        add_dlog_sigma_t(S, sg.o + sg.t * sg.d, q, df, -coef * sig / (sg.maj - sig), grad_off, acc);
        Tr *= null_ratio(sig, sg.maj);
        if (!roulette(Tr, rng)) return;
        sg.redraw(rng);
    }
}

template <int NLIGHT>
struct VertexNee {
    float E[NLIGHT];
    float3 wh[NLIGHT];
};

// Replay of path (pixel, sample) with radiance L_total (the sum of its contributions in
// double, so that the remaining radiance stays accurate after large contributions have been
// passed); wpix = dloss/dI_pixel / samples.
__device__ void replay_path(const SceneDev& S, uint32_t pixel, uint32_t sample, double L_total, float wpix,
                            float* grad_off, GradAcc& acc) {
    PathStats st;
    Rng rng;
    rng.init(S.key0, S.key1, pixel, sample, 0u, kStreamCam);
    const float ux = rng.uniform(), uy = rng.uniform();
    D3 o, d;
    camera_ray(S, pixel, ux, uy, o, d);
    float beta = 1.0f;
    double Lrem = L_total;
    int b = 0;
    for (;;) {
        double t0, t1;
        if (!clip_box(S, o, d, t0, t1)) break;
        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamTrack);
        const float3 df = to_f3(d);
        Segment sg;
        sg.begin<false>(S, o, d, t0, t1, rng, st);
        bool hit = false;
        for (;;) {
            const int ev = sg.step<false>(S, st);
            if (ev == kCell) continue;
            if (ev == kEnd) break;
            sg.advance();
            if (++sg.steps > kStepCap) break;
            const float u2 = rng.uniform();
            const float3 x = sg.pos();
            const PointQ q = eval_point(S, x);
            const float sig = sigma_t_of(q, df);
            if (u2 * sg.maj < sig) {
                hit = true;
                break;
            }
            if (Lrem != 0.0)
                add_dlog_sigma_t(S, sg.o + sg.t * sg.d, q, df, -wpix * (float)Lrem * sig / (sg.maj - sig), grad_off, acc);
            sg.redraw(rng);
        }
        if (!hit) break;
        ++b;
        if (b > S.max_depth) break;
        const D3 x = o + sg.t * d;
        const float3 xf = to_f3(x);
        const PointQ q = eval_point(S, xf);
        VertexNee<2> nv;
        double Etot = 0.0;
#pragma unroll 1
        for (int li = 0; li < 2; ++li) {
            nv.E[li] = 0.0f;
            D3 wl, inv;
            double tend;
            float Le;
            if (!light_sample(S, li, x, wl, tend, Le, inv)) continue;
            const float3 wlf = to_f3(wl);
            const float p = phase_eval(q, df, wlf);
            Rng rn;
            rn.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamNee0 + (uint32_t)li);
            const float Tr = ratio_track<false>(S, x, wl, inv, wlf, tend, rn, st);
            nv.E[li] = nee_contribution(mul_rn(beta, p), Tr, Le);
            Etot += (double)nv.E[li];
            if (nv.E[li] != 0.0f) {
                Rng rn2;
                rn2.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamNee0 + (uint32_t)li);
                ratio_track_grad(S, x, wl, wlf, tend, rn2, wpix * nv.E[li], grad_off, acc);
                const float3 h = wlf - df;
                const float hn = sqrtf(dot(h, h));
                float3 dG;
                float ds;
                if (hn >= 1e-7f && dlog_ndf(q.G, q.s, (1.0f / hn) * h, dG, ds)) {
                    const float c = wpix * nv.E[li];
                    scatter_grad(S, x, q, 0.0f, c * dG, 0.0f, c * ds, grad_off, acc, true);
                }
            }
        }
        // density and albedo: every contribution from this vertex on
        {
            float dmu, dsig;
            dlog_rho(q.mu, q.sigma, dmu, dsig);
            const float c = wpix * (float)Lrem;
            scatter_grad(S, x, q, c * dmu, f3(0.0f, 0.0f, 0.0f), c * dsig, 0.0f, grad_off, acc, true);
            if (!S.albedo_per_prim && S.albedo > 0.0f) acc.alb += c / S.albedo;
        }
        // phase sampling (same draws as the forward pass)
        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamPhase);
        D3 wi;
        float wgt, pdf;
        float3 wm;
        const bool ok = sample_scatter(S, q, scatter_frame(S, q, x, d), d, df, rng, wi, wgt, wm, pdf);
        const double Lafter = Lrem - Etot;
        if (ok && Lafter != 0.0) {
            float3 dG;
            float ds;
            if (dlog_ndf(q.G, q.s, wm, dG, ds)) {
                const float c = wpix * (float)Lafter;
                scatter_grad(S, x, q, 0.0f, c * dG, 0.0f, c * ds, grad_off, acc, true);
            }
        }
        if (!ok) break;
        Lrem = Lafter;
        beta = mul_rn(beta, wgt);
        o = x;
        d = wi;
    }
}

#ifndef GPSS_ADJ_MIN_WAVES
#define GPSS_ADJ_MIN_WAVES 4
#endif

// One thread per path (pixel p / ns, sample s0 + p % ns): its primal pass, then its replay.
static_assert(kSchedBlock == kGradCacheLanes, "the gradient cache has one column per thread of a block");

__global__ __launch_bounds__(256, GPSS_ADJ_MIN_WAVES) void adjoint_kernel(SceneDev S, const float* __restrict__ dloss,
                                                                         float* __restrict__ grad_off,
                                                                         float* __restrict__ grad_scalars, uint32_t s0,
                                                                         uint32_t ns, uint64_t npaths) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    GradAcc acc{0.0f, 0.0f, 0.0f};
    grad_table_init();
    if (p < npaths) {
        const uint32_t pixel = (uint32_t)(p / ns), sample = s0 + (uint32_t)(p % ns);
        const float wpix = dloss[pixel] / (float)ns;
        if (wpix != 0.0f) {
            PathStats st;
            st.clear();
            double Ld = 0.0;
            const float L = trace_path<false>(S, pixel, sample, st, nullptr, 0, &Ld);
            // L = 0 (or an invalid estimate) gives no gradient: every contribution is non-negative
            if (L > 0.0f && L < INFINITY) replay_path(S, pixel, sample, Ld, wpix, grad_off, acc);
        }
    }
    flush_grad_cell(S, grad_off, acc);
    grad_table_flush(grad_off);
    float v[3] = {acc.var, acc.len, acc.alb};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (v[0] != 0.0f) atomicAdd(&grad_scalars[0], v[0]);
        if (v[1] != 0.0f) atomicAdd(&grad_scalars[1], v[1]);
        if (v[2] != 0.0f) atomicAdd(&grad_scalars[2], v[2]);
    }
}

__global__ void adjoint_head_reset_kernel(uint32_t* head) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *head = 0u;
}

// Scheduled replay: persistent waves over the launch's paths (see run_scheduled).
__global__ __launch_bounds__(256, GPSS_SCHED_MIN_WAVES) void sched_adjoint_kernel(const SceneDev* __restrict__ Sp,
                                                                                 AdjointIo io,
                                                                                 uint32_t* head,
                                                                                 float* __restrict__ grad_scalars,
                                                                                 uint32_t s0, uint32_t ns,
                                                                                 uint32_t npaths) {
    const SceneDev& S = *Sp;
    PathStats st;
    st.clear();
    LaunchSource src;
    src.init(npaths);
    src.head = head;
    src.s0 = s0;
    src.ns = ns;
    GradAcc acc{0.0f, 0.0f, 0.0f};
    __shared__ SchedLds<true> lds;
    grad_table_init();
    const PathOut out{nullptr, nullptr};
    run_scheduled<false, true, kMedIso>(S, src, out, st, io, acc, lds);
    flush_grad_cell(S, io.grad_off, acc);
    grad_table_flush(io.grad_off);
    float v[3] = {acc.var, acc.len, acc.alb};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (v[0] != 0.0f) atomicAdd(&grad_scalars[0], v[0]);
        if (v[1] != 0.0f) atomicAdd(&grad_scalars[1], v[1]);
        if (v[2] != 0.0f) atomicAdd(&grad_scalars[2], v[2]);
    }
}

__global__ void zero_kernel(float* __restrict__ a, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0f;
}

int launch_adjoint(gpss_scene* s, const float* dloss, float* grad_off, float* grad_scalars, uint32_t s0,
                   uint32_t ns, hipStream_t stream) {
    const uint64_t noff = (uint64_t)s->desc.off_res[0] * s->desc.off_res[1] * s->desc.off_res[2];
    if (grad_off && s->d_offset)
        hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)((noff + 255) / 256)), dim3(256), 0, stream, grad_off, noff);
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, stream, grad_scalars, (uint64_t)3);
    const uint64_t npaths = s->n_pixels() * ns;
    const uint64_t blocks = (npaths + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return set_error(GPSS_ERR_INVALID_ARG, "too many paths in one launch");
    float* go = s->d_offset ? grad_off : nullptr;
    if (s->kernel == GPSS_KERNEL_MEGA) {   // one thread per path: primal pass and replay
        hipLaunchKernelGGL(adjoint_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, s->dev, dloss, go,
                           grad_scalars, s0, ns, npaths);
        return check_hip(hipGetLastError(), "adjoint_kernel launch");
    }
    // scheduled: each lane traces its path's primal pass, then replays it
    int rc = ensure_sched(s, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(adjoint_head_reset_kernel, dim3(1), dim3(64), 0, stream, s->d_head);
    AdjointIo io;
    io.dloss = dloss;
    io.grad_off = go;
    io.inv_ns = 1.0f / (float)ns;
    hipLaunchKernelGGL(sched_adjoint_kernel, dim3(s->sched_grid), dim3(kSchedBlock), 0, stream, s->d_dev, io,
                       s->d_head, grad_scalars, s0, ns, (uint32_t)npaths);
    return check_hip(hipGetLastError(), "sched_adjoint_kernel launch");
}

}  // namespace gpss
