// Null-scattering path tracing of the macrofacet medium (per-path device routines):
// camera rays, delta tracking and ratio tracking through the majorant grid, next-event
// estimation to delta lights and mixture phase sampling.
#pragma once

#include "gpss_device.hpp"

namespace gpss {

enum TrackResult : int { kEscape = 0, kCollide = 1, kAbsorbed = 2 };
enum WalkEvent : int { kCell = 0, kTentative = 1, kEnd = 2 };

// Free-flight walk of one segment [t0, t1] of a ray through the majorant grid: tentative
// collisions of the null-scattering process with the piecewise-constant majorant, an
// optical depth tau = -ln(1 - u) being consumed cell by cell per tentative collision.
struct Segment {
    D3 o, d;
    double t, t1, tau;
    Walker w;
    float maj;      // majorant of the tentative collision (set when step() returns kTentative)
    uint32_t majb;  // the current cell's majorant as its top 16 bits (Walker::majorant_of)
    int steps;      // tentative collisions so far
    template <bool STATS>
    __device__ __forceinline__ void begin(const SceneDev& S, D3 o_, D3 d_, D3 inv, double t0, double t1_,
                                          Rng& rng, PathStats& st) {
        o = o_;
        d = d_;
        t = t0;
        t1 = t1_;
        w.init(S, o, d, inv, t0);
        majb = w.majorant_bits(S);
        tau = -(double)logf(1.0f - rng.uniform());
        steps = 0;
        if (STATS) st.cells++;
    }
    template <bool STATS>
    __device__ __forceinline__ void begin(const SceneDev& S, D3 o_, D3 d_, double t0, double t1_, Rng& rng,
                                          PathStats& st) {
        begin<STATS>(S, o_, d_, d3(1.0 / d_.x, 1.0 / d_.y, 1.0 / d_.z), t0, t1_, rng, st);
    }
    __device__ __forceinline__ void redraw(Rng& rng) { tau = -(double)logf(1.0f - rng.uniform()); }
    __device__ __forceinline__ float3 pos() const { return to_f3(o + t * d); }
    // One event of the walk: reach the next tentative collision in the current cell
    // (kTentative; maj set, t left at the start of the cell's remaining part until advance()
    // moves it to the collision), cross into the next cell (kCell), or reach the end of the
    // segment (kEnd).  Callers loop over events, so that lanes of a wave crossing cells and
    // lanes evaluating collisions progress in the same iterations.
    template <bool STATS>
    __device__ __forceinline__ int step(const SceneDev& S, PathStats& st) {
        int ax;
        const double tn = w.exit(ax);
        // the next cell's majorant is requested before this cell's work and kept as loaded
        // (converted at its use in the next step), so that the load can complete while the
        // walk finishes this cell and starts the next
        const uint32_t mn = w.next_majorant_bits(S, ax);
        const double tc = tn < t1 ? tn : t1;
        const float m = Walker::majorant_of(majb);
        const double seg = fmax(0.0, tc - t);
        if (m > 0.0f && tau < (double)m * seg) {
            maj = m;
            return kTentative;
        }
        if (m > 0.0f) tau -= (double)m * seg;
        t = tc;
        if (tn >= t1) return kEnd;
        if (!w.step(ax)) return kEnd;
        majb = mn;
        if (STATS) st.cells++;
        return kCell;
    }
    // Move t to the tentative collision found by step().
    __device__ __forceinline__ void advance() { t += tau / (double)maj; }
};

// Delta tracking over [t0, t1]: the tentative collision is real iff u2 * majorant < sigma_t.
template <bool STATS>
__device__ __forceinline__ int delta_track(const SceneDev& S, D3 o, D3 d, D3 inv, float3 df, double t0,
                                           double t1, Rng& rng, double& t_hit, PathStats& st) {
    Segment sg;
    sg.begin<STATS>(S, o, d, inv, t0, t1, rng, st);
    for (;;) {
        const int ev = sg.step<STATS>(S, st);
        if (ev == kCell) continue;
        if (ev == kEnd) return kEscape;
        sg.advance();
        if (STATS) st.track_steps++;
        if (++sg.steps > kStepCap) {
            if (STATS) st.capped++;
            return kAbsorbed;
        }
        const float u2 = rng.uniform();
        const PointQ q = eval_point(S, sg.pos());
        const float sig = sigma_t_of(q, df);
        if (STATS && sig > sg.maj) st.violations++;
        if (u2 * sg.maj < sig) {
            t_hit = sg.t;
            return kCollide;
        }
        sg.redraw(rng);
    }
}

// Russian roulette on a shadow ray's running transmittance: below kRRThreshold it survives
// with probability 1/2 (one uniform) and is doubled.  Returns false when terminated.
__device__ __forceinline__ bool roulette(float& Tr, Rng& rng) {
    if (Tr < kRRThreshold) {
        if (rng.uniform() < 0.5f) return false;
        Tr = Tr * 2.0f;
    }
    return true;
}

// Ratio tracking transmittance over [0, t1]: product of (1 - sigma_t / majorant) at
// tentative collisions (one uniform each for the free flight), with Russian roulette.
template <bool STATS>
__device__ __forceinline__ float ratio_track(const SceneDev& S, D3 o, D3 d, D3 inv, float3 df, double t1,
                                             Rng& rng, PathStats& st) {
    Segment sg;
    sg.begin<STATS>(S, o, d, inv, 0.0, t1, rng, st);
    float Tr = 1.0f;
    for (;;) {
        const int ev = sg.step<STATS>(S, st);
        if (ev == kCell) continue;
        if (ev == kEnd) return Tr;
        sg.advance();
        if (STATS) st.nee_steps++;
        if (++sg.steps > kStepCap) {
            if (STATS) st.capped++;
            return 0.0f;
        }
        const PointQ q = eval_point(S, sg.pos());
        const float sig = sigma_t_of(q, df);
        if (STATS && sig > sg.maj) st.violations++;
        Tr *= null_ratio(sig, sg.maj);
        if (!roulette(Tr, rng)) return 0.0f;
        sg.redraw(rng);
    }
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
// (0 directional, 1 point) seen from x; false if the light is absent.  inv receives the
// per-axis reciprocals of the direction.
__device__ __forceinline__ bool light_sample(const SceneDev& S, int li, D3 x, D3& wl, double& tend, float& Le,
                                             D3& inv) {
    double a0, a1;
    if (li == 0) {
        if (!(S.dl[3] > 0.0f)) return false;
        wl = d3(S.dl[0], S.dl[1], S.dl[2]);
        if (!clip_box(S, x, wl, a0, a1, inv)) a1 = 0.0;
        tend = a1;
        Le = S.dl[3];
        return true;
    }
    if (!(S.pl[3] > 0.0f)) return false;
    const D3 dv = d3((double)S.pl[0] - x.x, (double)S.pl[1] - x.y, (double)S.pl[2] - x.z);
    const double r2 = dot(dv, dv);
    const double r = sqrt(r2);
    wl = (1.0 / r) * dv;
    if (!clip_box(S, x, wl, a0, a1, inv)) a1 = 0.0;
    tend = fmin(a1, r);
    Le = (float)((double)S.pl[3] / r2);
    return true;
}
__device__ __forceinline__ bool light_sample(const SceneDev& S, int li, D3 x, D3& wl, double& tend, float& Le) {
    D3 inv;
    return light_sample(S, li, x, wl, tend, Le, inv);
}

// The proposal's frame at real collision x for travel direction d, in double, from the mean
// gradient and spread there.  Only N, alpha, cos(theta_v) and a are kept (sample_scatter forms
// the tangents).
__device__ __forceinline__ FrameD scatter_frame(const SceneDev& S, D3 x, D3 d) {
    FrameD fr = make_frame_d(eval_geom_d(S, x), -d);
    fr.T = fr.B = d3(0.0, 0.0, 0.0);
    return fr;
}
// The same from single-precision point statistics (a conditioned GP's posterior).
__device__ __forceinline__ FrameD scatter_frame(const PointQ& q, D3 d) {
    GeomD gd;
    gd.G = d3(q.G);
    gd.s = (double)q.s;
    FrameD fr = make_frame_d(gd, -d);
    fr.T = fr.B = d3(0.0, 0.0, 0.0);
    return fr;
}
// The frame for q at x: the conditioned GP's from q, every other medium's from the scene.
__device__ __forceinline__ FrameD scatter_frame(const SceneDev& S, const PointQ& q, D3 x, D3 d) {
    return q.cond ? scatter_frame(q, d) : scatter_frame(S, x, d);
}

// Phase-function sampling at a real collision (Sec. 4.2.2 proposal) with the frame fr of
// scatter_frame: draws (select, a, b) from the PHASE stream, returns the scattered direction
// and the throughput weight albedo <v, w_m> D(w_m) / (sigma(d) pdf(w_m)); false for a
// degenerate sample.  The half vector is formed in double, since the scattered direction
// starts the next segment; the inverse-CDF draws, the pdf and the weight are single precision.
__device__ __forceinline__ bool sample_scatter(const SceneDev& S, const PointQ& q, const FrameD& fr, D3 d, float3 df,
                                               Rng& rng, D3& wi, float& wgt, float3& wm, float& pdf) {
    const float3 v = -df;
    const D3 vd = -d;
    Proposal prop = proposal_of(fr, S.R, q.ggx);
    if (fr.beck) {   // the single-precision tangents of the frame
        const float3 vt = v - prop.cosv * prop.N;
        const float st = sqrtf(dot(vt, vt));
        if (st > 1e-7f) {
            prop.T = (1.0f / st) * vt;
        } else {
            float3 bb;
            onb(prop.N, prop.T, bb);
        }
        prop.B = cross(prop.N, prop.T);
    }
    const float usel = rng.uniform();
    const uint32_t ua = rng.next24(), ub = rng.next24();
    const HalfDraw hd = draw_half(prop, usel, ua, ub);
    const D3 wmd = combine_half_d(hd, fr, vd);
    wm = to_f3(wmd);
    pdf = mixture_pdf(prop, v, wm);
    const double vmd = dot(vd, wmd);
    if (!(pdf > 0.0f) || !(vmd > 0.0)) return false;
    const float vm = fmaxf(dot(v, wm), 0.0f);
    wi = normalize((2.0 * vmd) * wmd - vd);
    wgt = fresnel_F(q, vm) * vm * ndf_at(q, wm) / (sigma_proj_at(q, df) * pdf);
    return true;
}

// Radiance added by one light connection: ((beta * phase) * Tr) * Le.
__device__ __forceinline__ float nee_contribution(float beta_phase, float Tr, float Le) {
    return mul_rn(mul_rn(beta_phase, Tr), Le);
}

// Per-vertex record of a traced path (diagnostics): kRecFields floats per real collision.
constexpr int kRecFields = 16;

// One path (pixel, sample): returns its radiance estimate.  With REC, vertex k's record
// goes to rec[k * kRecFields ...] for k < kmax: x, t_hit, track steps, (phase, Tr) per
// light, w_m, pdf, weight, beta after the vertex, L after its next-event estimates.  Lsum
// (nullable) receives the sum of the same contributions in double.
template <bool STATS, bool REC = false>
__device__ float trace_path(const SceneDev& S, uint32_t pixel, uint32_t sample, PathStats& st,
                            float* rec = nullptr, int kmax = 0, double* Lsum = nullptr) {
    Rng rng;
    rng.init(S.key0, S.key1, pixel, sample, 0u, kStreamCam);
    const float ux = rng.uniform(), uy = rng.uniform();
    D3 o, d;
    camera_ray(S, pixel, ux, uy, o, d);
    float beta = 1.0f, L = 0.0f;
    int b = 0;
    for (;;) {
        double t0, t1;
        D3 inv;
        if (!clip_box(S, o, d, t0, t1, inv)) {
            if (Lsum) *Lsum += (double)mul_rn(beta, S.env);
            L = add_rn(L, mul_rn(beta, S.env));
            if (STATS) st.escaped++;
            break;
        }
        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamTrack);
        double th = 0.0;
        const uint32_t steps_before = st.track_steps;
        const float3 df = to_f3(d);
                const int res = delta_track<STATS || REC>(S, o, d, inv, df, t0, t1, rng, th, st);
        float* r = (REC && b < kmax) ? rec + b * kRecFields : nullptr;
        if (res == kAbsorbed) break;
        if (res == kEscape) {
            if (Lsum) *Lsum += (double)mul_rn(beta, S.env);
            L = add_rn(L, mul_rn(beta, S.env));
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
            D3 wl, inv;
            double tend;
            float Le;
            if (!light_sample(S, li, x, wl, tend, Le, inv)) continue;
            if (STATS) st.nee++;
            const float3 wlf = to_f3(wl);
            const float p = phase_eval(q, df, wlf);
            Rng rn;
            rn.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamNee0 + (uint32_t)li);
                        const float Tr = ratio_track<STATS>(S, x, wl, inv, wlf, tend, rn, st);
            const float E = nee_contribution(mul_rn(beta, p), Tr, Le);
            if (Lsum) *Lsum += (double)E;
            L = add_rn(L, E);
            if (REC && r) { r[5 + 2 * li] = p; r[6 + 2 * li] = Tr; }
        }
        // phase sampling
        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamPhase);
        D3 wi;
        float wgt, pdf;
        float3 wm;
        if (STATS) st.phase++;
        if (!sample_scatter(S, q, scatter_frame(S, q, x, d), d, df, rng, wi, wgt, wm, pdf)) break;  // degenerate: the path ends
        beta = mul_rn(beta, wgt);
        if (REC && r) {
            r[9] = wm.x; r[10] = wm.y; r[11] = wm.z; r[12] = pdf; r[13] = wgt; r[14] = beta; r[15] = L;
        }
        o = x;
        d = wi;
    }
    return L;
}

}  // namespace gpss
