// Wavefront form of the forward tracer.
//
// Path state lives in structure-of-arrays buffers in HBM (one slot per path of the launch,
// slot = pixel * ns + sample offset).  Each bounce runs three kernels over queues of slots:
//   track   - free-flight sampling of the current segment (delta tracking) until a real
//             collision, an escape or the depth limit; also folds in the radiance of the
//             previous vertex's light connections;
//   scatter - at each real collision: light-connection set-up (phase value, arriving
//             radiance) and phase-function sampling of the next direction;
//   nee     - ratio tracking toward each light for the connections set up by scatter.
// track and nee run persistent waves: a wave takes 64-slot chunks of its input queue with
// one atomic, refills lanes whose segment has finished from the chunk (ballot + popcount
// ranks), and appends outputs to the next queue with one atomic per wave (ballot +
// prefix ranks).  The arithmetic per path is the same, operation for operation, as the
// one-thread-per-path kernel, so both give bit-identical path radiances.
#include "gpss_accum.hpp"
#include "gpss_internal.hpp"
#include "gpss_trace.hpp"
#include "gpss_waves.hpp"

namespace gpss {

constexpr uint32_t kDead = 0x80000000u;   // path ended at its last vertex (degenerate phase sample)

__device__ __forceinline__ void pixel_sample(const WfState& W, uint32_t p, uint32_t& pixel, uint32_t& sample) {
    pixel = p / W.ns;
    sample = W.s0 + p % W.ns;
}

// ---------------------------------------------------------------------------
// Camera rays for every slot; the first track queue is the identity.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wf_init_kernel(SceneDev S, WfState W) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        W.cnt[kQInCount] = (uint32_t)W.npaths;
        W.cnt[kQInHead] = 0;
        W.cnt[kQOutCount] = 0;
        W.cnt[kQScatterCount] = 0;
        W.cnt[kQScatterHead] = 0;
        W.cnt[kQNeeCount] = 0;
        W.cnt[kQNeeHead] = 0;
    }
    if (p >= W.npaths) return;
    uint32_t pixel, sample;
    pixel_sample(W, (uint32_t)p, pixel, sample);
    Rng rng;
    rng.init(S.key0, S.key1, pixel, sample, 0u, kStreamCam);
    const float ux = rng.uniform(), uy = rng.uniform();
    D3 o, d;
    camera_ray(S, pixel, ux, uy, o, d);
    W.ox[p] = o.x; W.oy[p] = o.y; W.oz[p] = o.z;
    W.dx[p] = d.x; W.dy[p] = d.y; W.dz[p] = d.z;
    W.beta[p] = 1.0f;
    W.L[p] = 0.0f;
    W.bounce[p] = 0u;
    W.nee_c[2 * p] = 0.0f;
    W.nee_c[2 * p + 1] = 0.0f;
    W.q_a[p] = (uint32_t)p;
}

// Next bounce: the output track queue becomes the input queue.
__global__ void wf_next_kernel(WfState W) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        W.cnt[kQInCount] = W.cnt[kQOutCount];
        W.cnt[kQInHead] = 0;
        W.cnt[kQOutCount] = 0;
        W.cnt[kQScatterCount] = 0;
        W.cnt[kQScatterHead] = 0;
        W.cnt[kQNeeCount] = 0;
        W.cnt[kQNeeHead] = 0;
    }
}

template <bool STATS>
__device__ __forceinline__ void flush_stats_wf(const PathStats& st, unsigned long long* counters) {
    if (!STATS) return;
    const uint32_t vals[12] = {st.track_steps, st.real, st.nee_steps, st.violations, st.capped,
                               st.escaped, st.truncated, st.cells, st.phase, st.nee, st.nonfinite, st.saturated};
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        uint32_t v = vals[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(&counters[i], (unsigned long long)v);
    }
}

// Final radiance of path p (counted when it is not a valid estimate, see gpss_accum.hpp).
template <bool STATS>
__device__ __forceinline__ void wf_emit(const WfState& W, uint32_t p, float L, PathStats& st) {
    if (STATS) {
        const int c = acc_class(L);
        st.nonfinite += c == kAccNonFinite;
        st.saturated += c == kAccSaturated;
    }
    W.out[p] = L;
}

#ifndef GPSS_WF_TRACK_MIN_WAVES
#define GPSS_WF_TRACK_MIN_WAVES 4
#endif
#ifndef GPSS_WF_NEE_MIN_WAVES
#define GPSS_WF_NEE_MIN_WAVES 4
#endif

// ---------------------------------------------------------------------------
// track: delta tracking of the segment of every queued path.
// ---------------------------------------------------------------------------
template <bool STATS>
__global__ __launch_bounds__(256, GPSS_WF_TRACK_MIN_WAVES) void wf_track_kernel(SceneDev S, WfState W,
                                                                               const uint32_t* __restrict__ qin,
                                                                               unsigned long long* counters) {
    PathStats st;
    st.clear();
    ChunkReader rd;
    rd.init(W.cnt[kQInCount]);
    bool active = false;
    uint32_t p = 0, b = 0;
    float beta = 0.0f, L = 0.0f;
    float3 df = f3(0.0f, 0.0f, 0.0f);
    Segment sg;
    Rng rng;
    for (;;) {
        // refill lanes without a segment
        uint32_t qi;
        bool loaded = rd.take(!active, &W.cnt[kQInHead], qi);
        if (loaded) {
            p = qin[qi];
            const uint32_t bf = W.bounce[p];
            L = W.L[p];
            L = add_rn(L, W.nee_c[2 * p]);
            L = add_rn(L, W.nee_c[2 * p + 1]);
            if (bf & kDead) {
                wf_emit<STATS>(W, p, L, st);
            } else {
                b = bf;
                beta = W.beta[p];
                const D3 o = d3(W.ox[p], W.oy[p], W.oz[p]);
                const D3 d = d3(W.dx[p], W.dy[p], W.dz[p]);
                double t0, t1;
                D3 inv;
                if (!clip_box(S, o, d, t0, t1, inv)) {
                    L = add_rn(L, mul_rn(beta, S.env));
                    if (STATS) st.escaped++;
                    wf_emit<STATS>(W, p, L, st);
                } else {
                    uint32_t pixel, sample;
                    pixel_sample(W, p, pixel, sample);
                    rng.init(S.key0, S.key1, pixel, sample, b, kStreamTrack);
                    df = to_f3(d);
                    sg.begin<STATS>(S, o, d, inv, t0, t1, rng, st);
                    active = true;
                }
            }
        }
        if (!__any(active)) {
            if (rd.exhausted) break;
            continue;
        }
        bool push = false;
        if (active) {
            int res = -1;
            // walk cells to the next tentative collision (or the end of the segment) so that
            // the wave evaluates the medium for all its lanes together
            int ev;
            do {
                ev = sg.step<STATS>(S, st);
            } while (ev == kCell);
            if (ev == kEnd) {
                res = kEscape;
            } else {
                sg.advance();
                if (STATS) st.track_steps++;
                if (++sg.steps > kStepCap) {
                    if (STATS) st.capped++;
                    res = kAbsorbed;
                } else {
                    const float u2 = rng.uniform();
                    const PointQ q = eval_point(S, sg.pos());
                    const float sig = sigma_t_of(q, df);
                    if (STATS && sig > sg.maj) st.violations++;
                    if (u2 * sg.maj < sig) res = kCollide;
                    else sg.redraw(rng);
                }
            }
            if (res >= 0) {
                active = false;
                if (res == kEscape) {
                    L = add_rn(L, mul_rn(beta, S.env));
                    if (STATS) st.escaped++;
                    wf_emit<STATS>(W, p, L, st);
                } else if (res == kAbsorbed) {
                    wf_emit<STATS>(W, p, L, st);
                } else {
                    if (STATS) st.real++;
                    if ((int)b + 1 > S.max_depth) {
                        if (STATS) st.truncated++;
                        wf_emit<STATS>(W, p, L, st);
                    } else {
                        const D3 x = sg.o + sg.t * sg.d;
                        W.ox[p] = x.x; W.oy[p] = x.y; W.oz[p] = x.z;
                        W.L[p] = L;
                        W.bounce[p] = b + 1;
                        push = true;
                    }
                }
            }
        }
        wave_push(push, p, W.q_scatter, &W.cnt[kQScatterCount]);
    }
    flush_stats_wf<STATS>(st, counters);
}

// ---------------------------------------------------------------------------
// scatter: light-connection set-up and phase sampling at every real collision.
// ---------------------------------------------------------------------------
template <bool STATS>
__global__ __launch_bounds__(256) void wf_scatter_kernel(SceneDev S, WfState W, uint32_t* __restrict__ qout,
                                                         unsigned long long* counters) {
    PathStats st;
    st.clear();
    const uint32_t n = W.cnt[kQScatterCount];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < n;
        uint32_t p = 0;
        bool nee_push[2] = {false, false};
        if (valid) {
            p = W.q_scatter[i];
            const uint32_t b = W.bounce[p];
            uint32_t pixel, sample;
            pixel_sample(W, p, pixel, sample);
            const D3 x = d3(W.ox[p], W.oy[p], W.oz[p]);
            const D3 d = d3(W.dx[p], W.dy[p], W.dz[p]);
            const float3 df = to_f3(d);
            const float beta = W.beta[p];
            const PointQ q = eval_point(S, to_f3(x));
#pragma unroll
            for (int li = 0; li < 2; ++li) {
                D3 wl;
                double tend;
                float Le;
                if (light_sample(S, li, x, wl, tend, Le)) {
                    if (STATS) st.nee++;
                    const float ph = phase_eval(q, df, to_f3(wl));
                    W.nee_bp[2 * p + li] = mul_rn(beta, ph);
                    W.nee_le[2 * p + li] = Le;
                    nee_push[li] = true;
                } else {
                    W.nee_c[2 * p + li] = 0.0f;
                }
            }
            Rng rng;
            rng.init(S.key0, S.key1, pixel, sample, b, kStreamPhase);
            D3 wi;
            float wgt, pdf;
            float3 wm;
            if (STATS) st.phase++;
            if (sample_scatter(S, q, scatter_frame(S, q, x, d), d, df, rng, wi, wgt, wm, pdf)) {
                W.dx[p] = wi.x; W.dy[p] = wi.y; W.dz[p] = wi.z;
                W.beta[p] = mul_rn(beta, wgt);
            } else {
                W.bounce[p] = b | kDead;
            }
        }
        wave_push(nee_push[0], 2 * p, W.q_nee, &W.cnt[kQNeeCount]);
        wave_push(nee_push[1], 2 * p + 1, W.q_nee, &W.cnt[kQNeeCount]);
        wave_push(valid, p, qout, &W.cnt[kQOutCount]);
    }
    flush_stats_wf<STATS>(st, counters);
}

// ---------------------------------------------------------------------------
// nee: ratio tracking toward the light of every queued connection.
// ---------------------------------------------------------------------------
template <bool STATS>
__global__ __launch_bounds__(256, GPSS_WF_NEE_MIN_WAVES) void wf_nee_kernel(SceneDev S, WfState W,
                                                                           unsigned long long* counters) {
    PathStats st;
    st.clear();
    ChunkReader rd;
    rd.init(W.cnt[kQNeeCount]);
    bool active = false;
    uint32_t k = 0;
    float Tr = 1.0f;
    float3 wf = f3(0.0f, 0.0f, 0.0f);
    Segment sg;
    Rng rng;
    for (;;) {
        uint32_t qi;
        if (rd.take(!active, &W.cnt[kQNeeHead], qi)) {
            k = W.q_nee[qi];
            const uint32_t p = k >> 1, li = k & 1u;
            const uint32_t b = W.bounce[p] & ~kDead;
            uint32_t pixel, sample;
            pixel_sample(W, p, pixel, sample);
            const D3 x = d3(W.ox[p], W.oy[p], W.oz[p]);
            D3 wl, inv;
            double tend;
            float Le;
            light_sample(S, (int)li, x, wl, tend, Le, inv);
            wf = to_f3(wl);
            rng.init(S.key0, S.key1, pixel, sample, b, kStreamNee0 + li);
            sg.begin<STATS>(S, x, wl, inv, 0.0, tend, rng, st);
            Tr = 1.0f;
            active = true;
        }
        if (!__any(active)) {
            if (rd.exhausted) break;
            continue;
        }
        if (active) {
            bool done = false;
            int ev;
            do {
                ev = sg.step<STATS>(S, st);
            } while (ev == kCell);
            if (ev == kEnd) {
                done = true;
            } else {
                sg.advance();
                if (STATS) st.nee_steps++;
                if (++sg.steps > kStepCap) {
                    if (STATS) st.capped++;
                    Tr = 0.0f;
                    done = true;
                } else {
                    const PointQ q = eval_point(S, sg.pos());
                    const float sig = sigma_t_of(q, wf);
                    if (STATS && sig > sg.maj) st.violations++;
                    Tr *= null_ratio(sig, sg.maj);
                    if (!roulette(Tr, rng)) {
                        Tr = 0.0f;
                        done = true;
                    } else {
                        sg.redraw(rng);
                    }
                }
            }
            if (done) {
                W.nee_c[k] = nee_contribution(W.nee_bp[k], Tr, W.nee_le[k]);
                active = false;
            }
        }
    }
    flush_stats_wf<STATS>(st, counters);
}

// ---------------------------------------------------------------------------
// Host driver.
// ---------------------------------------------------------------------------
int wf_render(gpss_scene* s, float* paths, uint64_t* counters, uint32_t s0, uint32_t ns, hipStream_t stream) {
    const uint64_t npaths = s->n_pixels() * ns;
    if (npaths > 0x7FFFFFFFull) return set_error(GPSS_ERR_INVALID_ARG, "wavefront launch limited to 2^31 paths");
    int rc = ensure_wavefront(s, npaths);
    if (rc) return rc;
    WfState W = s->wf;
    W.out = paths;
    W.s0 = s0;
    W.ns = ns;
    W.npaths = npaths;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counters);
    const dim3 blk(256);
    hipLaunchKernelGGL(wf_init_kernel, dim3((uint32_t)((npaths + 255) / 256)), blk, 0, stream, s->dev, W);
    const uint32_t grid = s->wf_grid;
    uint32_t* qa = W.q_a;
    uint32_t* qb = W.q_b;
    for (int it = 0; it <= s->dev.max_depth; ++it) {
        if (counters) hipLaunchKernelGGL(wf_track_kernel<true>, dim3(grid), blk, 0, stream, s->dev, W, qa, cnt);
        else hipLaunchKernelGGL(wf_track_kernel<false>, dim3(grid), blk, 0, stream, s->dev, W, qa, cnt);
        if (it == s->dev.max_depth) break;
        if (counters) {
            hipLaunchKernelGGL(wf_scatter_kernel<true>, dim3(grid), blk, 0, stream, s->dev, W, qb, cnt);
            hipLaunchKernelGGL(wf_nee_kernel<true>, dim3(grid), blk, 0, stream, s->dev, W, cnt);
        } else {
            hipLaunchKernelGGL(wf_scatter_kernel<false>, dim3(grid), blk, 0, stream, s->dev, W, qb, cnt);
            hipLaunchKernelGGL(wf_nee_kernel<false>, dim3(grid), blk, 0, stream, s->dev, W, cnt);
        }
        hipLaunchKernelGGL(wf_next_kernel, dim3(1), dim3(64), 0, stream, W);
        uint32_t* t = qa;
        qa = qb;
        qb = t;
    }
    return check_hip(hipGetLastError(), "wavefront launch");
}

}  // namespace gpss
