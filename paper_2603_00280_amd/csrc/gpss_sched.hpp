// Scheduled path tracing loop of the persistent kernels (single render and batch).
//
// One lane carries one path at a time through a small state machine; idle lanes take new
// paths from a path source.  A path's work splits into operations of very different cost:
//   walk    - one majorant-cell step of the current segment (cheap, most frequent);
//   eval    - medium evaluation at a tentative collision (density, projected area) and its
//             outcome: accept/reject for delta tracking, the transmittance factor and
//             Russian roulette for ratio tracking;
//   scatter - at a real collision: light-connection set-up and phase-function sampling;
//   begin   - start of a segment (box clip, cell walker, first free-flight draw), either
//             the next track segment or a shadow ray toward one light.
// Each iteration the wave counts its lanes per pending operation (ballots) and runs ONE
// operation for all lanes waiting on it.  Expensive operations wait until enough lanes
// are ready, so that they run with most lanes active; while they wait, the other lanes
// keep walking.  Every decision is wave-uniform, so the only divergence left is inside an
// operation.
//
// Per path the operations run in the same order, with the same random-number streams and
// the same floating-point roundings as the one-thread-per-path routine trace_path; the
// path radiances are bit-identical to it.
#pragma once

#include "gpss_trace.hpp"
#include "gpss_waves.hpp"

namespace gpss {

enum LaneOp : int { kOpIdle = 0, kOpWalk = 1, kOpEval = 2, kOpScatter = 3, kOpBegin = 4 };

// Minimum number of waiting lanes (of 64) before an operation runs while other lanes could
// still walk, and the number of cell steps per walk operation.
#ifndef GPSS_SCHED_EVAL_MIN
#define GPSS_SCHED_EVAL_MIN 16
#endif
#ifndef GPSS_SCHED_SCATTER_MIN
#define GPSS_SCHED_SCATTER_MIN 16
#endif
#ifndef GPSS_SCHED_BEGIN_MIN
#define GPSS_SCHED_BEGIN_MIN 16
#endif
#ifndef GPSS_SCHED_REFILL_MIN
#define GPSS_SCHED_REFILL_MIN 8
#endif
#ifndef GPSS_SCHED_WALK_STEPS
#define GPSS_SCHED_WALK_STEPS 6
#endif
#ifndef GPSS_SCHED_MIN_WAVES
#define GPSS_SCHED_MIN_WAVES 3
#endif

// Trace every path of `src` (a wave-collective path source: take(idle, slot, pixel, sample)
// hands idle lanes new paths, exhausted() is wave-uniform) and write each path's radiance to
// paths[slot].  Must be called by whole waves; returns when the source is exhausted and
// every lane's path has ended.
// Threads per workgroup of the kernels that run the scheduled loop (per-lane LDS columns).
constexpr int kSchedBlock = 256;

template <bool STATS, class Source>
__device__ __forceinline__ void run_scheduled(const SceneDev& S, Source& src, float* __restrict__ paths,
                                              PathStats& st) {
    // Cold per-lane state (touched once per segment or vertex) lives in LDS, one column per
    // lane, so that registers hold what the cell walk and the medium evaluation use.
    __shared__ uint32_t cs_u[3][kSchedBlock];   // output slot, pixel, sample
    __shared__ float cs_f[6][kSchedBlock];      // beta, L, beta*phase and Le per light
    __shared__ double cs_d[3][kSchedBlock];     // direction of the next track segment
    const int lt = threadIdx.x;
    enum { kSlot = 0, kPixel = 1, kSample = 2 };
    enum { kBeta = 0, kL = 1, kBp0 = 2, kBp1 = 3, kLe0 = 4, kLe1 = 5 };
    enum { kHas0 = 1, kHas1 = 2, kDead = 4 };

    int op = kOpIdle;
    int b = 0;                 // real collisions so far
    int mode = 0;              // current segment: 0 track, 1 + li shadow ray toward light li
    int flags = 0;             // kHas0 | kHas1 (lights connected at this vertex) | kDead
    float Tr = 1.0f;
    Segment sg;
    sg.o = d3(0.0, 0.0, 0.0);
    Rng rng;
    auto finish = [&](float L) {   // the path's radiance to its output slot; the lane falls idle
        paths[cs_u[kSlot][lt]] = L;
        op = kOpIdle;
    };

    for (;;) {
        const uint64_t mIdle = __ballot(op == kOpIdle);
        const uint64_t mWalk = __ballot(op == kOpWalk);
        const uint64_t mEval = __ballot(op == kOpEval);
        const uint64_t mScat = __ballot(op == kOpScatter);
        const uint64_t mBegin = __ballot(op == kOpBegin);
        const int nIdle = __popcll(mIdle), nWalk = __popcll(mWalk), nEval = __popcll(mEval),
                  nScat = __popcll(mScat), nBegin = __popcll(mBegin);
        const int nBusy = nWalk + nEval + nScat + nBegin;

        // ---- refill idle lanes with new paths (camera rays) ----
        if (nIdle > 0 && !src.exhausted() && (nIdle >= GPSS_SCHED_REFILL_MIN || nBusy == 0)) {
            uint32_t slot = 0, pixel = 0, sample = 0;
            if (src.take(op == kOpIdle, slot, pixel, sample)) {
                Rng rc;
                rc.init(S.key0, S.key1, pixel, sample, 0u, kStreamCam);
                const float ux = rc.uniform(), uy = rc.uniform();
                D3 o, d;
                camera_ray(S, pixel, ux, uy, o, d);
                cs_u[kSlot][lt] = slot;
                cs_u[kPixel][lt] = pixel;
                cs_u[kSample][lt] = sample;
                cs_d[0][lt] = d.x;
                cs_d[1][lt] = d.y;
                cs_d[2][lt] = d.z;
                cs_f[kBeta][lt] = 1.0f;
                cs_f[kL][lt] = 0.0f;
                sg.o = o;
                b = 0;
                mode = 0;
                flags = 0;
                op = kOpBegin;
            }
            continue;
        }
        if (nBusy == 0) break;  // every lane idle and no paths left

        // ---- phase sampling and light-connection set-up at real collisions ----
        if (nScat > 0 && (nScat >= GPSS_SCHED_SCATTER_MIN || nWalk + nEval + nBegin == 0)) {
            if (op == kOpScatter) {
                ++b;
                const D3 x = sg.o + sg.t * sg.d;
                const D3 d = sg.d;
                const float3 df = to_f3(d);
                const PointQ q = eval_point(S, to_f3(x));
                float beta = cs_f[kBeta][lt];
                flags = 0;
#pragma unroll
                for (int li = 0; li < 2; ++li) {
                    D3 wl;
                    double tend;
                    float Le;
                    if (!light_sample(S, li, x, wl, tend, Le)) continue;
                    if (STATS) st.nee++;
                    const float ph = phase_eval(q, df, to_f3(wl));
                    flags |= li == 0 ? kHas0 : kHas1;
                    cs_f[kBp0 + li][lt] = mul_rn(beta, ph);
                    cs_f[kLe0 + li][lt] = Le;
                }
                rng.init(S.key0, S.key1, cs_u[kPixel][lt], cs_u[kSample][lt], (uint32_t)b, kStreamPhase);
                D3 wi;
                float wgt, pdf;
                float3 wm;
                if (STATS) st.phase++;
                if (sample_scatter(S, q, d, df, rng, wi, wgt, wm, pdf)) {
                    cs_f[kBeta][lt] = mul_rn(beta, wgt);
                    cs_d[0][lt] = wi.x;
                    cs_d[1][lt] = wi.y;
                    cs_d[2][lt] = wi.z;
                } else {
                    flags |= kDead;   // the path ends after this vertex's light connections
                }
                sg.o = x;
                mode = (flags & kHas0) ? 1 : ((flags & kHas1) ? 2 : 0);
                if (mode == 0 && (flags & kDead)) finish(cs_f[kL][lt]);
                else op = kOpBegin;
            }
            continue;
        }

        // ---- segment starts: next track segment or shadow ray ----
        if (nBegin > 0 && (nBegin >= GPSS_SCHED_BEGIN_MIN || nWalk + nEval == 0)) {
            if (op == kOpBegin) {
                const uint32_t pixel = cs_u[kPixel][lt], sample = cs_u[kSample][lt];
                if (mode == 0) {
                    const D3 o = sg.o, d = d3(cs_d[0][lt], cs_d[1][lt], cs_d[2][lt]);
                    double t0, t1;
                    D3 inv;
                    if (!clip_box(S, o, d, t0, t1, inv)) {
                        if (STATS) st.escaped++;
                        finish(add_rn(cs_f[kL][lt], mul_rn(cs_f[kBeta][lt], S.env)));
                    } else {
                        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamTrack);
                        sg.begin<STATS>(S, o, d, inv, t0, t1, rng, st);
                        op = kOpWalk;
                    }
                } else {
                    const int li = mode - 1;
                    const D3 x = sg.o;
                    D3 wl, inv;
                    double tend;
                    float Le;
                    light_sample(S, li, x, wl, tend, Le, inv);
                    rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamNee0 + (uint32_t)li);
                    sg.begin<STATS>(S, x, wl, inv, 0.0, tend, rng, st);
                    Tr = 1.0f;
                    op = kOpWalk;
                }
            }
            continue;
        }

        // ---- medium evaluation at tentative collisions ----
        bool nee_done = false;
        if (nEval > 0 && (nEval >= GPSS_SCHED_EVAL_MIN || nWalk == 0)) {
            if (op == kOpEval) {
                sg.advance();
                // the generator's key and address words are recomputed here rather than kept
                // live through the other operations: key, pixel, sample, bounce | stream
                rng.key = make_uint2(S.key0, S.key1);
                rng.ctr.x = cs_u[kPixel][lt];
                rng.ctr.y = cs_u[kSample][lt];
                const uint32_t stream = mode == 0 ? kStreamTrack : kStreamNee0 + (uint32_t)(mode - 1);
                rng.ctr.z = ((uint32_t)b & 0xFFFFu) | (stream << 16);
                rng.ensure2();   // this operation's draws (collision test or roulette, next flight)
                if (STATS) {
                    if (mode == 0) st.track_steps++;
                    else st.nee_steps++;
                }
                const bool capped = ++sg.steps > kStepCap;
                float u2 = 0.0f;
                if (!capped && mode == 0) u2 = rng.uniform();
                const PointQ q = eval_point(S, sg.pos());
                const float sig = sigma_t_of(q, to_f3(sg.d));   // single-precision travel direction
                if (capped) {
                    if (STATS) st.capped++;
                    if (mode == 0) {
                        finish(cs_f[kL][lt]);
                    } else {
                        Tr = 0.0f;
                        nee_done = true;
                    }
                } else {
                    if (STATS && sig > sg.maj) st.violations++;
                    if (mode == 0) {
                        if (u2 * sg.maj < sig) {
                            if (STATS) st.real++;
                            if (b + 1 > S.max_depth) {
                                if (STATS) st.truncated++;
                                finish(cs_f[kL][lt]);
                            } else {
                                op = kOpScatter;
                            }
                        } else {
                            sg.redraw(rng);
                            op = kOpWalk;
                        }
                    } else {
                        Tr *= 1.0f - sig / sg.maj;
                        if (!roulette(Tr, rng)) {
                            Tr = 0.0f;
                            nee_done = true;
                        } else {
                            sg.redraw(rng);
                            op = kOpWalk;
                        }
                    }
                }
            }
        } else if (op == kOpWalk) {
            // ---- cell walk: up to GPSS_SCHED_WALK_STEPS events per lane ----
#pragma unroll 1
            for (int k = 0; k < GPSS_SCHED_WALK_STEPS; ++k) {
                const int ev = sg.step<STATS>(S, st);
                if (ev == kCell) continue;
                if (ev == kTentative) {
                    op = kOpEval;
                } else if (mode == 0) {   // track segment left the medium
                    if (STATS) st.escaped++;
                    finish(add_rn(cs_f[kL][lt], mul_rn(cs_f[kBeta][lt], S.env)));
                } else {
                    nee_done = true;
                }
                break;
            }
        }
        if (nee_done) {
            // shadow ray finished: add its contribution, then the next light or the next
            // track segment (or the end of a path whose phase sample was degenerate)
            const int li = mode - 1;
            const float L = add_rn(cs_f[kL][lt], nee_contribution(cs_f[kBp0 + li][lt], Tr, cs_f[kLe0 + li][lt]));
            cs_f[kL][lt] = L;
            mode = (li == 0 && (flags & kHas1)) ? 2 : 0;
            if (mode == 0 && (flags & kDead)) finish(L);
            else op = kOpBegin;
        }
    }
}

}  // namespace gpss
