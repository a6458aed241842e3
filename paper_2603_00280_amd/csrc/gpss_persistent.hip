// Persistent scheduled form of the forward tracer for one scene: a grid sized to the
// resident waves, each wave taking its paths in chunks of 64 or 256 (one atomic per chunk) and
// tracing them with the scheduled loop of gpss_sched.hpp.  Each path's radiance goes to the
// per-path output or to its pixel's fixed-point accumulator.
#include "gpss_internal.hpp"
#include "gpss_sched.hpp"

namespace gpss {

int sched_waves_per_simd() { return GPSS_SCHED_MIN_WAVES; }

template <bool STATS>
__device__ __forceinline__ void flush_stats_sched(const PathStats& st, unsigned long long* counters) {
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

__global__ void sched_reset_kernel(uint32_t* head) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *head = 0u;
}

template <bool STATS, int MED>
__global__ __launch_bounds__(256, GPSS_SCHED_MIN_WAVES) void sched_render_kernel(
    const SceneDev* __restrict__ Sp, PathOut out, uint32_t* head, unsigned long long* counters,
    uint32_t s0, uint32_t ns, uint32_t npaths) {
    const SceneDev& S = *Sp;
    PathStats st;
    st.clear();
    LaunchSource src;
    src.init(npaths);
    src.head = head;
    src.s0 = s0;
    src.ns = ns;
    const AdjointIo io{};
    GradAcc acc{0.0f, 0.0f, 0.0f};
    __shared__ SchedLds<false> lds;
    run_scheduled<STATS, false, MED>(S, src, out, st, io, acc, lds);
    flush_stats_sched<STATS>(st, counters);
}


int sched_render(gpss_scene* s, float* paths, unsigned long long* acc, uint64_t* counters, uint32_t s0,
                 uint32_t ns, hipStream_t stream, uint32_t* head) {
    const PathOut out{paths, acc};
    const uint64_t npaths = s->n_pixels() * ns;
    if (npaths > 0x7FFFFFFFull) return set_error(GPSS_ERR_INVALID_ARG, "persistent launch limited to 2^31 paths");
    int rc = ensure_sched(s, stream);
    if (rc) return rc;
    if (!head) head = s->d_head;
    hipLaunchKernelGGL(sched_reset_kernel, dim3(1), dim3(64), 0, stream, head);
    const dim3 blk(256);
    const dim3 grid(s->sched_grid);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counters);
    const int med = medium_of(s->dev);
#define GPSS_SCHED_LAUNCH(ST, M)                                                                                    \
    hipLaunchKernelGGL((sched_render_kernel<ST, M>), grid, blk, 0, stream, s->d_dev, out, head,                    \
                       ST ? cnt : nullptr, s0, ns, (uint32_t)npaths)
    if (counters) {
        if (med == kMedGgx) GPSS_SCHED_LAUNCH(true, kMedGgx);
        else if (med == kMedAniso) GPSS_SCHED_LAUNCH(true, kMedAniso);
        else if (med == kMedCond) GPSS_SCHED_LAUNCH(true, kMedCond);
        else GPSS_SCHED_LAUNCH(true, kMedIso);
    } else {
        if (med == kMedGgx) GPSS_SCHED_LAUNCH(false, kMedGgx);
        else if (med == kMedAniso) GPSS_SCHED_LAUNCH(false, kMedAniso);
        else if (med == kMedCond) GPSS_SCHED_LAUNCH(false, kMedCond);
        else GPSS_SCHED_LAUNCH(false, kMedIso);
    }
#undef GPSS_SCHED_LAUNCH
    return check_hip(hipGetLastError(), "sched_render_kernel launch");
}

}  // namespace gpss
