// Host-side scene object and helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/gpss.h"
#include "gpss_device.hpp"

namespace gpss {

// A roctx range over the host side of an entry point (argument checks and enqueue, not the
// device's execution): rocprofv3 --marker-trace shows it on the calling thread's timeline.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
// Structure-of-arrays path state and queues of the wavefront tracer (device pointers).
struct WfState {
    double *ox, *oy, *oz, *dx, *dy, *dz;   // ray origin (collision point after track) and direction
    float *beta, *L, *out;                 // throughput, radiance so far, final radiance per slot
    uint32_t* bounce;                      // real collisions so far (high bit: path ended)
    float *nee_c, *nee_bp, *nee_le;        // per slot and light: contribution, beta*phase, Le
    uint32_t *q_a, *q_b, *q_scatter, *q_nee;
    uint32_t* cnt;                         // queue counters, indexed by kQ*
    uint32_t s0, ns;
    uint64_t npaths;
};
enum { kQInCount = 0, kQInHead, kQOutCount, kQScatterCount, kQScatterHead, kQNeeCount, kQNeeHead, kQNum };
}  // namespace gpss

struct gpss_scene {
    gpss_scene_desc desc{};            // host pointers cleared after create
    gpss::SceneDev dev{};              // device view (pointers into the buffers below)
    std::vector<float> prims_h, offset_h, var_h, maj_h;
    bool maj_h_stale = false;          // device majorants rebuilt since maj_h was copied
    float* d_prims = nullptr;
    float* d_offset = nullptr;
    float* d_var = nullptr;
    float* d_maj = nullptr;
    uint16_t* d_maj16 = nullptr;       // the walk's copy of the majorants (SceneDev::maj16)
    uint16_t* d_cand = nullptr;        // per majorant cell: the union's candidate primitives (or null)
    float* d_obs = nullptr;            // conditioned GP: kMaxObs float4 (position, alpha) + packed L^-1 rows
    double* d_obs_d = nullptr;         // the same in double for the majorant: 3n positions, n alpha, n x n L^-1
    float* d_scratch = nullptr;        // per-path radiances of the wavefront and one-thread forms
    size_t scratch_floats = 0;
    unsigned long long* d_acc = nullptr;  // per-pixel fixed-point radiance sums (two words per pixel)
    int device = 0;
    uint32_t spp = 0;
    int kernel = 0;                    // GPSS_KERNEL_*
    gpss::WfState wf{};                // wavefront buffers (allocated on first use)
    void* wf_mem = nullptr;
    uint64_t wf_cap = 0;               // paths the wavefront buffers hold
    uint32_t wf_grid = 0;              // persistent workgroups per wavefront launch
    uint32_t* d_head = nullptr;        // path counter of the persistent scheduled kernel
    gpss::SceneDev* d_dev = nullptr;   // device copy of `dev` read by the persistent kernels
    gpss::SceneDev* h_rec = nullptr;   // pinned staging of the record's asynchronous uploads
    hipEvent_t rec_event = nullptr;    // completion of the last upload from h_rec
    uint64_t dev_version = 1;          // bumped whenever `dev` changes
    uint64_t dev_uploaded = 0;         // version held by d_dev
    uint32_t sched_grid = 0;           // workgroups of the persistent scheduled kernel
    uint64_t n_pixels() const { return (uint64_t)desc.width * desc.height; }
};

namespace gpss {

int set_error(int code, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);
int ensure_scratch(gpss_scene* s, size_t floats);
int ensure_acc(gpss_scene* s);

// kernel launchers (gpss_forward.hip)
int launch_majorants(gpss_scene* s, hipStream_t stream);
int launch_render_paths(gpss_scene* s, float* paths, uint64_t* counters, uint32_t s0, uint32_t ns,
                        hipStream_t stream);
int launch_reduce(gpss_scene* s, const float* paths, float* image, uint32_t ns, hipStream_t stream);
int ensure_wavefront(gpss_scene* s, uint64_t npaths);
int wf_render(gpss_scene* s, float* paths, uint64_t* counters, uint32_t s0, uint32_t ns, hipStream_t stream);
int mega_render(gpss_scene* s, float* paths, uint64_t* counters, uint32_t s0, uint32_t ns, hipStream_t stream);
int ensure_sched(gpss_scene* s, hipStream_t stream);
int sched_waves_per_simd();
// paths (per-path output) or acc (per-pixel accumulator) receives the radiances; head: the
// launch's path counter (nullptr: the scene's)
int sched_render(gpss_scene* s, float* paths, unsigned long long* acc, uint64_t* counters, uint32_t s0,
                 uint32_t ns, hipStream_t stream, uint32_t* head = nullptr);
int check_path_count(const gpss_scene* s, uint32_t s0, uint32_t s1);
int launch_acc_clear(unsigned long long* acc, uint64_t npix, hipStream_t stream);
int launch_acc_finalize(const unsigned long long* acc, float* image, uint32_t ns, uint64_t npix,
                        hipStream_t stream);
int device_cus(int device, int* cus);
int launch_debug_trace(gpss_scene* s, const uint32_t* ids, uint32_t n, float* out, int kmax,
                       hipStream_t stream);
int launch_adjoint(gpss_scene* s, const float* dloss, float* grad_off, float* grad_scalars, uint32_t s0,
                   uint32_t ns, hipStream_t stream);
int render_batch(gpss_scene* const* scenes, uint32_t n, float* const* images, hipStream_t stream);
int autotune_batch(gpss_scene* const* scenes, uint32_t n, float* const* images, hipStream_t stream,
                   uint32_t* best_tile, uint32_t* best_wpc, float* best_ms);
void forget_scene_plans(gpss_scene* s);
int launch_eval(gpss_scene* s, const float* pts, const float* dirs, float* out, uint64_t n,
                hipStream_t stream);

}  // namespace gpss
