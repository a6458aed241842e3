// Null-scattering path tracing of the macrofacet medium (per-path device routines):
// camera rays, delta tracking and ratio tracking through the majorant grid, next-event
// estimation to delta lights and mixture phase sampling.
#pragma once

#include "gpss_device.hpp"

namespace gpss {

enum TrackResult : int { kEscape = 0, kCollide = 1, kAbsorbed = 2 };

// Delta tracking over [t0, t1]: per tentative collision an optical depth tau = -ln(1 - u1)
// is consumed cell by cell through the majorant grid; the collision is real iff
// u2 * majorant < sigma_t.
template <bool STATS>
__device__ __forceinline__ int delta_track(const SceneDev& S, D3 o, D3 d, float3 df, double t0, double t1,
                                           Rng& rng, double& t_hit, PathStats& st) {
    Walker w;
    w.init(S, o, d, t0);
    double t = t0;
    double tau = -(double)logf(1.0f - rng.uniform());
    int steps = 0;
    if (STATS) st.cells++;
    for (;;) {
        int ax;
        const double tn = w.exit(ax);
        const double tc = fmin(tn, t1);
        const float maj = w.majorant(S);
        const double seg = fmax(0.0, tc - t);
        if (maj > 0.0f && tau < (double)maj * seg) {
            t += tau / (double)maj;
            const float3 x = to_f3(o + t * d);
            if (STATS) st.track_steps++;
            if (++steps > kStepCap) {
                if (STATS) st.capped++;
                return kAbsorbed;
            }
            const float u2 = rng.uniform();
            const PointQ q = eval_point(S, x);
            const float sig = sigma_t_of(q, df);
            if (STATS && sig > maj) st.violations++;
            if (u2 * maj < sig) {
                t_hit = t;
                return kCollide;
            }
            tau = -(double)logf(1.0f - rng.uniform());
            continue;
        }
        if (maj > 0.0f) tau -= (double)maj * seg;
        t = tc;
        if (tn >= t1) return kEscape;
        if (!w.step(S, ax)) return kEscape;
        if (STATS) st.cells++;
    }
}

// Ratio tracking transmittance over [0, t1]: product of (1 - sigma_t / majorant) at
// tentative collisions (one uniform each), 0 once below kTrCutoff.
template <bool STATS>
__device__ __forceinline__ float ratio_track(const SceneDev& S, D3 o, D3 d, float3 df, double t1, Rng& rng,
                                             PathStats& st) {
    Walker w;
    w.init(S, o, d, 0.0);
    double t = 0.0;
    float Tr = 1.0f;
    double tau = -(double)logf(1.0f - rng.uniform());
    int steps = 0;
    if (STATS) st.cells++;
    for (;;) {
        int ax;
        const double tn = w.exit(ax);
        const double tc = fmin(tn, t1);
        const float maj = w.majorant(S);
        const double seg = fmax(0.0, tc - t);
        if (maj > 0.0f && tau < (double)maj * seg) {
            t += tau / (double)maj;
            const float3 x = to_f3(o + t * d);
            if (STATS) st.nee_steps++;
            if (++steps > kStepCap) {
                if (STATS) st.capped++;
                return 0.0f;
            }
            const PointQ q = eval_point(S, x);
            const float sig = sigma_t_of(q, df);
            if (STATS && sig > maj) st.violations++;
            Tr *= 1.0f - sig / maj;
            if (Tr < kTrCutoff) return 0.0f;
            tau = -(double)logf(1.0f - rng.uniform());
            continue;
        }
        if (maj > 0.0f) tau -= (double)maj * seg;
        t = tc;
        if (tn >= t1) break;
        if (!w.step(S, ax)) break;
        if (STATS) st.cells++;
    }
    return Tr;
}

__device__ __forceinline__ void camera_ray(const SceneDev& S, uint32_t pixel, float ux, float uy, D3& o, D3& d) {
    const int i = (int)(pixel % (uint32_t)S.W), j = (int)(pixel / (uint32_t)S.W);
    const D3 fwd = d3(S.fwd[0], S.fwd[1], S.fwd[2]);
    const D3 rt = d3(S.right[0], S.right[1], S.right[2]);
    const D3 up = d3(S.upc[0], S.upc[1], S.upc[2]);
    const D3 eye = d3(S.eye[0], S.eye[1], S.eye[2]);
    if (S.cam_kind == 0) {
        const double px = (((double)i + ux) / (double)S.W - 0.5) * S.win[0];
        const double py = (0.5 - ((double)j + uy) / (double)S.H) * S.win[1];
        o = eye + px * rt + py * up;
        d = fwd;
    } else {
        const double px = (2.0 * ((double)i + ux) / (double)S.W - 1.0) * S.tan_half * S.aspect;
        const double py = (1.0 - 2.0 * ((double)j + uy) / (double)S.H) * S.tan_half;
        o = eye;
        d = normalize(fwd + px * rt + py * up);
    }
}

// Light direction, segment length inside the medium and arriving radiance for light li
// (0 directional, 1 point) seen from x; false if the light is absent.
__device__ __forceinline__ bool light_sample(const SceneDev& S, int li, D3 x, D3& wl, double& tend, float& Le) {
    double a0, a1;
    if (li == 0) {
        if (!(S.dl[3] > 0.0f)) return false;
        wl = d3(S.dl[0], S.dl[1], S.dl[2]);
        if (!clip_box(S, x, wl, a0, a1)) a1 = 0.0;
        tend = a1;
        Le = S.dl[3];
        return true;
    }
    if (!(S.pl[3] > 0.0f)) return false;
    const D3 dv = d3((double)S.pl[0] - x.x, (double)S.pl[1] - x.y, (double)S.pl[2] - x.z);
    const double r2 = dot(dv, dv);
    const double r = sqrt(r2);
    wl = (1.0 / r) * dv;
    if (!clip_box(S, x, wl, a0, a1)) a1 = 0.0;
    tend = fmin(a1, r);
    Le = (float)((double)S.pl[3] / r2);
    return true;
}

// Per-vertex record of a traced path (diagnostics): kRecFields floats per real collision.
constexpr int kRecFields = 16;

// One path (pixel, sample): returns its radiance estimate.  With REC, vertex k's record
// goes to rec[k * kRecFields ...] for k < kmax: x, t_hit, track steps, (phase, Tr) per
// light, w_m, pdf, weight, beta after the vertex, L after its next-event estimates.
template <bool STATS, bool REC = false>
__device__ float trace_path(const SceneDev& S, uint32_t pixel, uint32_t sample, PathStats& st,
                            float* rec = nullptr, int kmax = 0) {
    Rng rng;
    rng.init(S.key0, S.key1, pixel, sample, 0u, kStreamCam);
    const float ux = rng.uniform(), uy = rng.uniform();
    D3 o, d;
    camera_ray(S, pixel, ux, uy, o, d);
    float beta = 1.0f, L = 0.0f;
    int b = 0;
    for (;;) {
        double t0, t1;
        if (!clip_box(S, o, d, t0, t1)) {
            L += beta * S.env;
            if (STATS) st.escaped++;
            break;
        }
        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamTrack);
        double th = 0.0;
        const uint32_t steps_before = st.track_steps;
        const float3 df = to_f3(d);
        const int res = delta_track<STATS || REC>(S, o, d, df, t0, t1, rng, th, st);
        float* r = (REC && b < kmax) ? rec + b * kRecFields : nullptr;
        if (res == kAbsorbed) break;
        if (res == kEscape) {
            L += beta * S.env;
            if (STATS) st.escaped++;
            break;
        }
        if (STATS) st.real++;
        ++b;
        if (b > S.max_depth) {
            if (STATS) st.truncated++;
            break;
        }
        const D3 x = o + th * d;
        const PointQ q = eval_point(S, to_f3(x));
        if (REC && r) {
            r[0] = (float)x.x; r[1] = (float)x.y; r[2] = (float)x.z; r[3] = (float)th;
            r[4] = (float)(st.track_steps - steps_before);
        }
        // next-event estimation: directional light on stream kStreamNee0, point light on +1
#pragma unroll 1
        for (int li = 0; li < 2; ++li) {
            D3 wl;
            double tend;
            float Le;
            if (!light_sample(S, li, x, wl, tend, Le)) continue;
            if (STATS) st.nee++;
            const float3 wlf = to_f3(wl);
            const float p = phase_eval(q, df, wlf);
            Rng rn;
            rn.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamNee0 + (uint32_t)li);
            const float Tr = ratio_track<STATS>(S, x, wl, wlf, tend, rn, st);
            L += beta * p * Tr * Le;
            if (REC && r) { r[5 + 2 * li] = p; r[6 + 2 * li] = Tr; }
        }
        // phase sampling
        const float3 v = -df;
        const Proposal prop = make_proposal(q, S.R, v);
        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamPhase);
        const float usel = rng.uniform();
        const uint32_t ua = rng.next24(), ub = rng.next24();
        const float3 wm = sample_half_vector(prop, v, usel, ua, ub);
        const float pdf = mixture_pdf(prop, v, wm);
        const float vm = dot(v, wm);
        if (STATS) st.phase++;
        if (!(pdf > 0.0f) || !(vm > 0.0f)) break;  // degenerate sample: the path ends
        const D3 wmd = d3(wm);
        const D3 vd = -d;
        const D3 wi = normalize((2.0 * dot(vd, wmd)) * wmd - vd);
        const float wgt = q.albedo * vm * ndf(q.G, q.s, wm) / (sigma_proj(q.G, q.s, df) * pdf);
        beta *= wgt;
        if (REC && r) {
            r[9] = wm.x; r[10] = wm.y; r[11] = wm.z; r[12] = pdf; r[13] = wgt; r[14] = beta; r[15] = L;
        }
        o = x;
        d = wi;
    }
    return L;
}

}  // namespace gpss
