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
// operation.  Paths that ended in the previous iteration are first added to their pixels,
// one pixel at a time, through the wave's LDS pixel table (forward form with a pixel
// accumulator).
//
// Per path the operations run in the same order, with the same random-number streams and
// the same floating-point roundings as the one-thread-per-path routine trace_path; the
// path radiances are bit-identical to it.
#pragma once

#include "gpss_accum.hpp"
#include "gpss_grad.hpp"
#include "gpss_trace.hpp"
#include "gpss_waves.hpp"

namespace gpss {

// kOpOut: the path has ended and its radiance (column kL) waits to be added to its pixel
enum LaneOp : int { kOpIdle = 0, kOpWalk = 1, kOpEval = 2, kOpScatter = 3, kOpBegin = 4, kOpOut = 5 };

// Minimum number of waiting lanes (of 64) before an operation runs while other lanes could
// still walk, and the number of cell steps per walk operation.
#ifndef GPSS_SCHED_EVAL_MIN
#define GPSS_SCHED_EVAL_MIN 16
#endif
// the conditioned GP's evaluation costs about thirty times the others': it waits for fuller waves
#ifndef GPSS_SCHED_EVAL_MIN_COND
#define GPSS_SCHED_EVAL_MIN_COND 32
#endif
#ifndef GPSS_SCHED_BEGIN_MIN
#define GPSS_SCHED_BEGIN_MIN 16
#endif
#ifndef GPSS_SCHED_REFILL_MIN
#define GPSS_SCHED_REFILL_MIN 8
#endif
// Drain (adjoint form): once the path source is exhausted and at most this many lanes are
// busy, the wave runs every pending operation as soon as one lane needs it, for the latency
// of its last paths rather than for full operations.  The adjoint traces each path twice in
// one lane, so on its million-path launches the last paths' latency is much of the call.
// The forward form keeps the throughput policy throughout: the same drain in it shortened
// small launches but changed the headline kernel's register allocation, which then either
// spilled in the scatter operation or ran 1.3 % slower.
#ifndef GPSS_SCHED_DRAIN
#define GPSS_SCHED_DRAIN 32
#endif
// The scatter threshold and the cell steps per walk come from the scene record (walk_steps,
// scatter_min): see sched_policy in gpss_device.hpp.
#ifndef GPSS_SCHED_MIN_WAVES
#define GPSS_SCHED_MIN_WAVES 3
#endif

// Threads per workgroup of the kernels that run the scheduled loop (per-lane LDS columns).
constexpr int kSchedBlock = 256;

// Paths p in [0, npaths) of one launch: pixel p / ns, sample s0 + p % ns, slot p.  Large
// launches are claimed 256 consecutive paths at a time (at 256 samples per pixel one pixel,
// whose sum then leaves the wave's pixel table, below, about once); launches with fewer than
// kLaunchChunkMinClaims such claims per resident wave take 64, so that no wave runs out of
// paths early.
constexpr uint32_t kLaunchChunkBig = 256;
constexpr uint32_t kLaunchChunkMinClaims = 32;
struct LaunchSource {
    ChunkReader rd;
    __device__ __forceinline__ void init(uint32_t npaths) {
        const uint32_t waves = gridDim.x * (blockDim.x / 64u);
        const bool big = npaths / waves >= kLaunchChunkMinClaims * kLaunchChunkBig;
        rd.init(npaths, big ? kLaunchChunkBig : kChunk);
    }
    uint32_t* head;
    uint32_t s0, ns;
    __device__ __forceinline__ bool exhausted() const { return rd.exhausted; }
    __device__ __forceinline__ bool take(bool idle, uint32_t& slot, uint32_t& pixel, uint32_t& sample) {
        uint32_t qi = 0;
        if (!rd.take(idle, head, qi)) return false;
        slot = qi;
        pixel = qi / ns;
        sample = s0 + qi % ns;
        return true;
    }
};

// Where the forward form puts each path's radiance: paths[slot] when `paths` is set (per-path
// output), else its pixel's fixed-point accumulator `acc` (two words per pixel, gpss_accum.hpp).
struct PathOut {
    float* paths;
    unsigned long long* acc;
};

// Inputs and outputs of the path-replay adjoint form of the loop.
struct AdjointIo {
    const float* dloss;        // d loss / d pixel
    float* grad_off;           // offset-grid gradient (nullable), accumulated atomically per cell
    float inv_ns;              // 1 / samples per pixel of the launch
};

// Light connections per path whose contribution the adjoint's primal pass keeps for the
// replay (one LDS column each); later connections are walked twice in the replay.
constexpr int kAdjConn = 4;

// Trace every path of `src` (a wave-collective path source: take(idle, slot, pixel, sample)
// hands idle lanes new paths, exhausted() is wave-uniform).  Forward form (ADJ false): each
// path's radiance goes to `out`.  Adjoint form: each path with dloss[pixel] != 0 is traced
// twice by its lane: a primal pass, the forward tracer's own, gives its radiance L and keeps
// the contributions of its first kAdjConn light connections; a replay of the same random
// streams then carries L_rem (L less the contributions already passed) and accumulates the
// parameter gradient with weight dloss[pixel] / ns (frozen-sampling estimator; the terms are
// those of the one-thread replay in gpss_adjoint.hip) into io.grad_off and acc.  A shadow ray
// whose contribution was kept is walked once in the replay, for its gradient, and not at all
// when the contribution is 0.  Nothing is stored per path outside the lane.  The caller
// empties the workgroup's gradient table before (grad_table_init) and adds the lane's cached
// cells and the table to the grid after (flush_grad_cell, grad_table_flush).  Must be called
// by whole waves; returns when the source is exhausted and every lane's path has ended.
// MED: the scene's medium when the kernel is specialized for it (kMedIso generalized with the
// isotropic kernel, kMedGgx, kMedAniso generalized with the anisotropic kernel), so that
// the other media's code is not compiled in; kMedAny takes everything from the scene record.
enum { kMedAny = -1, kMedIso = 0, kMedGgx = 1, kMedAniso = 2, kMedCond = 3 };

__host__ __device__ inline int medium_of(const SceneDev& S) {
    return S.n_obs > 0 ? kMedCond : (S.ggx ? kMedGgx : (S.aniso_k != 0.0f ? kMedAniso : kMedIso));
}

// Cold per-lane state (touched once per segment or vertex) lives in LDS, one column per
// lane, so that registers hold what the cell walk and the medium evaluation use.  The
// kernel declares it (__shared__) and hands it to run_scheduled.
// Per-wave table of pixel sums (direct-mapped by pixel): a wave takes consecutive paths, which
// share pixels, so ended paths add to their pixel's entry here and an entry goes to the global
// accumulator (two integer atomics) only when it changes pixel and at the end.  The device-
// scope atomics of one add per path reach past the per-XCD L2 and wrote about 100 bytes of
// memory traffic per path.
constexpr int kAccTable = 16;
constexpr int kSchedWaves = kSchedBlock / 64;
struct AccTable {
    unsigned long long lo[kSchedWaves][kAccTable], hi[kSchedWaves][kAccTable];
    uint32_t px[kSchedWaves][kAccTable];   // pixel + 1 of the entry, 0 = empty
};

struct NoAccTable {};
template <bool ADJ>
struct SchedLds {
    uint32_t u[3][kSchedBlock];                     // output slot, pixel, sample
    float f[ADJ ? 15 + kAdjConn : 6][kSchedBlock];  // beta, L, beta*phase and Le per light (+ adjoint terms)
    double d[3][kSchedBlock];                       // direction of the next track segment
    double o[3][kSchedBlock];                       // origin of the current segment
    double sd[3][kSchedBlock];                      // direction of the current segment
    typename std::conditional<ADJ, NoAccTable, AccTable>::type acc;   // forward form's pixel table
};

template <bool STATS, bool ADJ, int MED, class Source>
__device__ __forceinline__ void run_scheduled(const SceneDev& S, Source& src, const PathOut& out,
                                              PathStats& st, const AdjointIo& io, GradAcc& acc,
                                              SchedLds<ADJ>& lds) {
    auto& cs_u = lds.u;
    auto& cs_f = lds.f;
    auto& cs_d = lds.d;
    auto& cs_o = lds.o;
    auto& cs_sd = lds.sd;
    const int lt = threadIdx.x;
    const int lane = lt & 63, wv = lt >> 6;
    const bool accumulate = !ADJ && !out.paths;   // wave-uniform
    AccTable* tab = nullptr;   // the forward form's pixel table (the adjoint's LDS has none)
    if constexpr (!ADJ) tab = &lds.acc;
    if (accumulate && lane < kAccTable) tab->px[wv][lane] = 0u;
    enum { kSlot = 0, kPixel = 1, kSample = 2 };
    // forward: kL = radiance so far.  Adjoint: kL + kLlo = radiance so far (primal pass), then
    // the remaining radiance L_rem (replay), kept as a two-float sum (ff_add) so that L_rem
    // stays accurate after large contributions have been passed.  kE0 + c: contribution of the
    // path's light connection c < kAdjConn.
    enum { kBeta = 0, kL = 1, kBp0 = 2, kBp1 = 3, kLe0 = 4, kLe1 = 5,
           kWpix = 6, kLlo = 7, kE = 8, kWm = 9, kDin = 12, kE0 = 15 };   // kWm, kDin: 3 columns each
    enum { kHas0 = 1, kHas1 = 2, kDead = 4, kGradPass = 8, kVertex = 16, kReplay = 32 };

    int op = kOpIdle;
    int b = 0;                 // real collisions so far
    int mode = 0;              // current segment: 0 track, 1 + li shadow ray toward light li
    int flags = 0;             // kHas0 | kHas1 (lights connected at this vertex) | kDead | ...
    int conn = 0;              // adjoint: light connections of the path completed so far
    float Tr = 1.0f;
    float coef = 0.0f;         // adjoint: weight of the shadow ray being replayed for its gradient
    // The segment's origin and direction are read at tentative collisions, vertices and
    // segment starts only, not by the cell walk: they live in LDS (columns cs_o, cs_sd) rather
    // than in registers, and sg.o, sg.d are not read.
    Segment sg;
    auto origin = [&]() { return d3(cs_o[0][lt], cs_o[1][lt], cs_o[2][lt]); };
    auto set_origin = [&](D3 o) {
        cs_o[0][lt] = o.x;
        cs_o[1][lt] = o.y;
        cs_o[2][lt] = o.z;
    };
    auto seg_dir = [&]() { return d3(cs_sd[0][lt], cs_sd[1][lt], cs_sd[2][lt]); };
    auto set_seg_dir = [&](D3 d) {
        cs_sd[0][lt] = d.x;
        cs_sd[1][lt] = d.y;
        cs_sd[2][lt] = d.z;
    };
    Rng rng;
    auto point = [&](float3 x) {   // medium statistics at x, with the specialized NDF kind
        PointQ q = eval_point(S, x);
        if (MED != kMedAny) {
            q.ggx = MED == kMedGgx;
            if (MED != kMedAniso) q.ak = 0.0f;
        }
        if (MED == kMedCond) condition_point(S, x, q);
        return q;
    };
    auto start = [&]() {   // camera ray of the lane's path (pixel, sample in its columns)
        const uint32_t pixel = cs_u[kPixel][lt], sample = cs_u[kSample][lt];
        Rng rc;
        rc.init(S.key0, S.key1, pixel, sample, 0u, kStreamCam);
        const float ux = rc.uniform(), uy = rc.uniform();
        D3 o, d;
        camera_ray(S, pixel, ux, uy, o, d);
        cs_d[0][lt] = d.x;
        cs_d[1][lt] = d.y;
        cs_d[2][lt] = d.z;
        cs_f[kBeta][lt] = 1.0f;
        set_origin(o);
        b = 0;
        mode = 0;
        conn = 0;
        op = kOpBegin;
    };
    auto finish = [&](float L) {   // end of the path (or of the adjoint's primal pass)
        if (ADJ && !(flags & kReplay)) {
            // primal pass done (its radiance is kL + kLlo): replay the path against it.  L = 0
            // makes every gradient term 0 (all contributions are non-negative), so such paths
            // end here.
            if (L > 0.0f && L < INFINITY) {
                flags = kReplay;
                start();
                return;
            }
        }
        if (!ADJ) {
            if (STATS) {
                const int c = acc_class(L);
                st.nonfinite += c == kAccNonFinite;
                st.saturated += c == kAccSaturated;
            }
            if (out.paths) {
                out.paths[cs_u[kSlot][lt]] = L;
            } else {   // added to the pixel's sum at the top of the next iteration
                cs_f[kL][lt] = L;
                op = kOpOut;
                return;
            }
        }
        op = kOpIdle;
    };
    // add one entry of the pixel table to the global accumulator and empty it (lane-local)
    auto flush_entry = [&](int e) {
        const uint32_t p1 = tab->px[wv][e];
        if (p1 == 0u) return;
        unsigned long long* w = out.acc + 2ull * (p1 - 1u);
        const unsigned long long lo = tab->lo[wv][e], hi = tab->hi[wv][e];
        if (lo) atomicAdd(w, lo);
        if (hi) atomicAdd(w + 1, hi);
        tab->px[wv][e] = 0u;
    };
    // a track segment left the medium: the environment it sees ends the path
    auto escape = [&]() {
        const float c = mul_rn(cs_f[kBeta][lt], S.env);
        if (ADJ && !(flags & kReplay)) {
            ff_add(cs_f[kL][lt], cs_f[kLlo][lt], c);
            finish(cs_f[kL][lt]);
        } else {
            finish(add_rn(cs_f[kL][lt], c));
        }
    };
    // after light li's connection: the next light, the next track segment, or the end of a
    // path whose phase sample was degenerate
    auto next_connection = [&](int li) {
        mode = (li == 0 && (flags & kHas1)) ? 2 : 0;
        if (mode == 0 && (flags & kDead)) finish(cs_f[kL][lt]);
        else op = kOpBegin;
    };

    for (;;) {
        if (accumulate) {
            // ended paths: one pixel at a time (wave-uniform), its entry taken over by that pixel
            // if it held another, then every lane of the pixel adds its fixed-point radiance
            for (uint64_t mOut = __ballot(op == kOpOut); mOut;) {
                const int leader = __builtin_ctzll(mOut);
                const uint32_t P = __shfl(cs_u[kPixel][lt], leader, 64);
                const int e = (int)(P % (uint32_t)kAccTable);
                if (lane == leader && tab->px[wv][e] != P + 1u) {
                    flush_entry(e);
                    tab->lo[wv][e] = 0ull;
                    tab->hi[wv][e] = 0ull;
                    tab->px[wv][e] = P + 1u;
                }
                const bool mine = op == kOpOut && cs_u[kPixel][lt] == P;
                if (mine) {
                    const uint64_t v = acc_fixed(cs_f[kL][lt]);
                    if (v & 0xFFFFFFFFull) atomicAdd(&tab->lo[wv][e], (unsigned long long)(v & 0xFFFFFFFFull));
                    if (v >> 32) atomicAdd(&tab->hi[wv][e], (unsigned long long)(v >> 32));
                    op = kOpIdle;
                }
                mOut &= ~__ballot(mine);
            }
        }
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
            bool got = src.take(op == kOpIdle, slot, pixel, sample);
            float wpix = 0.0f;
            if (ADJ && got) {
                wpix = io.dloss[pixel] * io.inv_ns;
                got = wpix != 0.0f;   // paths of pixels without loss gradient are skipped
            }
            if (got) {
                cs_u[kSlot][lt] = slot;
                cs_u[kPixel][lt] = pixel;
                cs_u[kSample][lt] = sample;
                cs_f[kL][lt] = 0.0f;
                if (ADJ) {
                    cs_f[kLlo][lt] = 0.0f;
                    cs_f[kWpix][lt] = wpix;
                }
                flags = 0;
                start();
            }
            continue;
        }
        if (nBusy == 0) {   // every lane idle and no paths left
            if (accumulate && lane < kAccTable) flush_entry(lane);
            break;
        }
        // wave-uniform, and read through a scalar register so that the compiler knows it: a
        // condition it takes for divergent turns the operations' branches into masked code
        const bool drain =
            ADJ && __builtin_amdgcn_readfirstlane((int)(src.exhausted() && nBusy <= GPSS_SCHED_DRAIN)) != 0;

        // ---- phase sampling and light-connection set-up at real collisions ----
        if (nScat > 0 && (drain || nScat >= S.scatter_min || nWalk + nEval + nBegin == 0)) {
            if (op == kOpScatter) {
                ++b;
                const D3 d = seg_dir();
                const D3 x = origin() + sg.t * d;
                const float3 df = to_f3(d);
                const float3 xf = to_f3(x);
                // the double frame before the point statistics: fewer values are live
                FrameD fr;
                if (MED != kMedCond) fr = scatter_frame(S, x, d);
                const PointQ q = point(xf);
                if (MED == kMedCond) fr = scatter_frame(q, d);
                const float beta = cs_f[kBeta][lt];
                const bool replay = ADJ && (flags & kReplay);
                flags &= kReplay;
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
                if (replay) {
                    // density and albedo: every contribution from this vertex on (L_rem)
                    float dmu, dsig;
                    dlog_rho(q.mu, q.sigma, dmu, dsig);
                    const float c = cs_f[kWpix][lt] * (cs_f[kL][lt] + cs_f[kLlo][lt]);
                    scatter_grad(S, x, q, c * dmu, f3(0.0f, 0.0f, 0.0f), c * dsig, 0.0f, io.grad_off, acc, true);
                    if (!S.albedo_per_prim && S.albedo > 0.0f) acc.alb += c / S.albedo;
                    cs_f[kDin + 0][lt] = df.x;
                    cs_f[kDin + 1][lt] = df.y;
                    cs_f[kDin + 2][lt] = df.z;
                }
                rng.init(S.key0, S.key1, cs_u[kPixel][lt], cs_u[kSample][lt], (uint32_t)b, kStreamPhase);
                D3 wi;
                float wgt, pdf;
                float3 wm;
                if (STATS) st.phase++;
                if (sample_scatter(S, q, fr, d, df, rng, wi, wgt, wm, pdf)) {
                    cs_f[kBeta][lt] = mul_rn(beta, wgt);
                    cs_d[0][lt] = wi.x;
                    cs_d[1][lt] = wi.y;
                    cs_d[2][lt] = wi.z;
                    if (replay) {
                        cs_f[kWm + 0][lt] = wm.x;
                        cs_f[kWm + 1][lt] = wm.y;
                        cs_f[kWm + 2][lt] = wm.z;
                        flags |= kVertex;   // phase-sample gradient once the connections are done
                    }
                } else {
                    flags |= kDead;   // the path ends after this vertex's light connections
                }
                set_origin(x);
                mode = (flags & kHas0) ? 1 : ((flags & kHas1) ? 2 : 0);
                if (mode == 0 && (flags & kDead)) finish(cs_f[kL][lt]);
                else op = kOpBegin;
            }
            continue;
        }

        // ---- segment starts: next track segment or shadow ray ----
        if (nBegin > 0 && (drain || nBegin >= GPSS_SCHED_BEGIN_MIN || nWalk + nEval == 0)) {
            if (op == kOpBegin) {
                const uint32_t pixel = cs_u[kPixel][lt], sample = cs_u[kSample][lt];
                if (mode == 0) {
                    if (ADJ && (flags & kVertex)) {
                        // phase sample of the vertex just left: contributions after its lights
                        // (their contributions have been taken off L_rem)
                        flags &= ~kVertex;
                        const float Lafter = cs_f[kL][lt] + cs_f[kLlo][lt];
                        if (Lafter != 0.0f) {
                            const D3 o = origin();
                            const PointQ q = point(to_f3(o));
                            const float3 wm = f3(cs_f[kWm][lt], cs_f[kWm + 1][lt], cs_f[kWm + 2][lt]);
                            float3 dG;
                            float ds;
                            if (dlog_ndf(q.G, q.s, wm, dG, ds)) {
                                const float c = cs_f[kWpix][lt] * Lafter;
                                scatter_grad(S, o, q, 0.0f, c * dG, 0.0f, c * ds, io.grad_off, acc, true);
                            }
                        }
                    }
                    const D3 o = origin(), d = d3(cs_d[0][lt], cs_d[1][lt], cs_d[2][lt]);
                    double t0, t1;
                    D3 inv;
                    if (!clip_box(S, o, d, t0, t1, inv)) {
                        if (STATS) st.escaped++;
                        escape();
                    } else {
                        rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamTrack);
                        sg.begin<STATS>(S, o, d, inv, t0, t1, rng, st);
                        set_seg_dir(d);
                        op = kOpWalk;
                    }
                } else {
                    const int li = mode - 1;
                    if (ADJ && (flags & kReplay) && !(flags & kGradPass) && conn < kAdjConn) {
                        // replay of a connection whose contribution E the primal pass kept:
                        // no walk when E = 0, else the gradient pass only
                        const float E = cs_f[kE0 + conn][lt];
                        ff_add(cs_f[kL][lt], cs_f[kLlo][lt], -E);
                        if (E == 0.0f) {
                            ++conn;
                            next_connection(li);
                            continue;
                        }
                        cs_f[kE][lt] = E;
                        coef = cs_f[kWpix][lt] * E;
                        flags |= kGradPass;
                    }
                    const D3 x = origin();
                    D3 wl, inv;
                    double tend;
                    float Le;
                    light_sample(S, li, x, wl, tend, Le, inv);
                    rng.init(S.key0, S.key1, pixel, sample, (uint32_t)b, kStreamNee0 + (uint32_t)li);
                    sg.begin<STATS>(S, x, wl, inv, 0.0, tend, rng, st);
                    set_seg_dir(wl);
                    Tr = 1.0f;
                    op = kOpWalk;
                }
            }
            continue;
        }

        // ---- medium evaluation at tentative collisions ----
        bool nee_done = false;
        constexpr int kEvalMin = MED == kMedCond ? GPSS_SCHED_EVAL_MIN_COND : GPSS_SCHED_EVAL_MIN;
        // with fewer than 8 lanes walking, waiting for fuller evaluations gains little
        const bool run_eval = nEval > 0 && (drain || nEval >= kEvalMin || nWalk < 8);
        if (run_eval) {
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
                const D3 dd = seg_dir();
                const D3 xd = origin() + sg.t * dd;
                const float3 xf = to_f3(xd);
                const float3 df = to_f3(dd);   // single-precision travel direction
                const PointQ q = point(xf);
                const float sig = sigma_t_of(q, df);
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
                            if (ADJ && (flags & kReplay)) {   // null collision: every remaining contribution
                                const float Lrem = cs_f[kL][lt] + cs_f[kLlo][lt];
                                if (Lrem != 0.0f)
                                    add_dlog_sigma_t(S, xd, q, df, -cs_f[kWpix][lt] * Lrem * sig / (sg.maj - sig),
                                                     io.grad_off, acc);
                            }
                            sg.redraw(rng);
                            op = kOpWalk;
                        }
                    } else {
                        if (ADJ && (flags & kGradPass))   // shadow-ray factor of this connection
                            add_dlog_sigma_t(S, xd, q, df, -coef * sig / (sg.maj - sig), io.grad_off, acc);
                        Tr *= null_ratio(sig, sg.maj);
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
            // ---- cell walk: up to S.walk_steps events per lane ----
#pragma unroll 1
            for (int k = 0; k < S.walk_steps; ++k) {
                const int ev = sg.step<STATS>(S, st);
                if (ev == kCell) continue;
                if (ev == kTentative) {
                    op = kOpEval;
                } else if (mode == 0) {   // track segment left the medium
                    if (STATS) st.escaped++;
                    escape();
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
            bool next = true;
            if (!ADJ) {
                cs_f[kL][lt] = add_rn(cs_f[kL][lt], nee_contribution(cs_f[kBp0 + li][lt], Tr, cs_f[kLe0 + li][lt]));
            } else if (!(flags & kReplay)) {
                // primal pass: add the contribution and keep it for the replay
                const float E = nee_contribution(cs_f[kBp0 + li][lt], Tr, cs_f[kLe0 + li][lt]);
                ff_add(cs_f[kL][lt], cs_f[kLlo][lt], E);
                if (conn < kAdjConn) cs_f[kE0 + conn][lt] = E;
                ++conn;
            } else if (!(flags & kGradPass)) {
                // replay of a connection beyond the kept ones: this walk gives its contribution
                // E; a second pass over the same random stream differentiates it when E != 0
                const float E = nee_contribution(cs_f[kBp0 + li][lt], Tr, cs_f[kLe0 + li][lt]);
                ff_add(cs_f[kL][lt], cs_f[kLlo][lt], -E);
                if (E != 0.0f) {
                    cs_f[kE][lt] = E;
                    coef = cs_f[kWpix][lt] * E;
                    flags |= kGradPass;
                    next = false;
                    op = kOpBegin;
                } else {
                    ++conn;
                }
            } else {
                // gradient pass done: the NDF at the connection's half vector
                flags &= ~kGradPass;
                ++conn;
                const float3 din = f3(cs_f[kDin][lt], cs_f[kDin + 1][lt], cs_f[kDin + 2][lt]);
                const float3 h = to_f3(seg_dir()) - din;
                const float hn = sqrtf(dot(h, h));
                float3 dG;
                float ds;
                if (hn >= 1e-7f) {
                    const D3 o = origin();
                    const PointQ q = point(to_f3(o));
                    if (dlog_ndf(q.G, q.s, (1.0f / hn) * h, dG, ds)) {
                        const float c = cs_f[kWpix][lt] * cs_f[kE][lt];
                        scatter_grad(S, o, q, 0.0f, c * dG, 0.0f, c * ds, io.grad_off, acc, true);
                    }
                }
            }
            if (next) next_connection(li);
        }
    }
}

}  // namespace gpss
