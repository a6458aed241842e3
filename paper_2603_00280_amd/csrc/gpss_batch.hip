// Batched rendering of many scenes in one persistent launch.
//
// A batch plan holds, in device memory, one record per scene (a copy of the scene's record
// and the offset of its pixels in the batch's pixel numbering) and a table of tiles,
// each a contiguous range of one scene's paths (path p = pixel * spp + sample).  A persistent
// kernel's waves take tiles from a global cursor (one atomic per tile) and trace each tile's
// paths with the scheduled loop of the persistent tracer, adding each path's radiance to its
// pixel's fixed-point accumulator (gpss_accum.hpp); a second kernel turns every scene's sums
// into its image.  [cursor reset, accumulator clear, persistent kernel, image kernel] is
// captured once into a hipGraph per plan and replayed on every call.  Images equal
// gpss_render's (same per-path routine, random numbers and accumulation).
#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "gpss_internal.hpp"
#include "gpss_sched.hpp"

namespace gpss {

struct BatchScene {
    SceneDev S;            // copy of the scene's record (read through the kernel's const array,
                           // so that its fields become scalar loads)
    uint64_t pix_base;     // first pixel of this scene in the batch's pixel numbering
    uint32_t spp;
    uint32_t npix;
};

struct Tile {
    uint32_t scene;
    uint32_t count;        // paths in the tile
    uint64_t p0;           // first path (within the scene)
};

__global__ void batch_reset_kernel(uint32_t* cursor) {
    if (threadIdx.x == 0) *cursor = 0u;
}

// Paths [p0, p0 + count) of one scene's tile, handed to idle lanes in order (the wave owns
// the tile, so no atomics): pixel p / spp, sample p % spp.
struct TileSource {
    uint64_t next, end;
    uint32_t spp;
    __device__ __forceinline__ bool exhausted() const { return next >= end; }
    __device__ __forceinline__ bool take(bool idle, uint32_t& slot, uint32_t& pixel, uint32_t& sample) {
        const uint64_t m = __ballot(idle);
        const uint64_t avail = end - next;
        const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt());
        const bool got = idle && rank < avail;
        const uint64_t p = next + rank;
        next += min((uint64_t)__popcll(m), avail);
        if (!got) return false;
        slot = (uint32_t)p;
        pixel = (uint32_t)(p / spp);
        sample = (uint32_t)(p % spp);
        return true;
    }
};

// Persistent waves take tiles from a global cursor (one atomic per tile) and trace each
// tile's paths with the scheduled loop; the scene record is wave-uniform.  MED: the medium
// kind every scene of the batch shares (that loop only), or kMedAny (the loop specialized for
// each tile's scene, all three compiled in, which costs registers).
template <int MED>
__global__ __launch_bounds__(256, GPSS_SCHED_MIN_WAVES) void batch_kernel(const BatchScene* __restrict__ scenes,
                                                                         const Tile* __restrict__ tiles, uint32_t ntiles,
                                                                         uint32_t* cursor,
                                                                         unsigned long long* __restrict__ acc) {
    const uint32_t lane = threadIdx.x & 63;
    PathStats st;
    st.clear();
    __shared__ SchedLds<false> lds;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(cursor, 1u);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
        if (t >= ntiles) break;
        const Tile tl = tiles[t];
        const BatchScene& B = scenes[tl.scene];
        const SceneDev& S = B.S;
        TileSource src;
        src.next = tl.p0;
        src.end = tl.p0 + tl.count;
        src.spp = B.spp;
        const PathOut out{nullptr, acc + 2 * B.pix_base};
        const AdjointIo io{};
        GradAcc gacc{0.0f, 0.0f, 0.0f};
        // the same specialization per medium as the single-scene kernel (identical images)
        if constexpr (MED != kMedAny) {
            run_scheduled<false, false, MED>(S, src, out, st, io, gacc, lds);
        } else {
            const int med = medium_of(S);
            if (med == kMedGgx) run_scheduled<false, false, kMedGgx>(S, src, out, st, io, gacc, lds);
            else if (med == kMedAniso) run_scheduled<false, false, kMedAniso>(S, src, out, st, io, gacc, lds);
            else run_scheduled<false, false, kMedIso>(S, src, out, st, io, gacc, lds);
        }
    }
}

// One thread per pixel of the batch: the scene's image from its fixed-point sums.
__global__ __launch_bounds__(256) void batch_image_kernel(const BatchScene* __restrict__ scenes, uint32_t nscenes,
                                                          float* const* __restrict__ images,
                                                          const unsigned long long* __restrict__ acc,
                                                          uint64_t total_pix) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_pix) return;
    uint32_t lo = 0, hi = nscenes - 1;   // last scene whose pix_base <= g
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (scenes[mid].pix_base <= g) lo = mid;
        else hi = mid - 1;
    }
    const BatchScene& B = scenes[lo];
    images[lo][g - B.pix_base] = acc_mean(acc[2 * g], acc[2 * g + 1], B.spp);
}

__global__ __launch_bounds__(256) void batch_clear_kernel(unsigned long long* __restrict__ acc, uint64_t nwords) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) acc[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Plans, graphs and tuning.
// ---------------------------------------------------------------------------
// Uploads of scene records and image pointers in flight per plan: each from its own pinned
// staging slot, reused once that slot's previous copy has completed.
constexpr int kImageRing = 4;

struct BatchPlan {
    std::vector<gpss_scene*> scenes;
    uint32_t tile = 0, grid = 0;
    BatchScene* d_scenes = nullptr;
    std::vector<uint64_t> versions;     // record version of each scene that d_scenes holds
    BatchScene* h_scenes[kImageRing] = {};   // pinned staging slots of the record uploads
    hipEvent_t ev_scenes[kImageRing] = {};
    int ring_scenes = 0;
    Tile* d_tiles = nullptr;
    uint32_t ntiles = 0;
    uint32_t* d_cursor = nullptr;
    float** d_images = nullptr;         // image pointers read by the graph
    std::vector<float*> images_set;     // the pointers d_images holds once the queued copies run
    float** h_images[kImageRing] = {};  // pinned staging slots of those copies
    hipEvent_t ev_images[kImageRing] = {};
    int ring = 0;
    unsigned long long* d_acc = nullptr;   // fixed-point sums, two words per pixel of the batch
    uint64_t total_paths = 0, total_pix = 0;
    int med = kMedAny;                  // batch_kernel instance in the captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
std::mutex g_mu;
std::vector<BatchPlan*> g_plans;

void free_plan(BatchPlan* P) {
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    (void)hipFree(P->d_scenes);
    (void)hipFree(P->d_tiles);
    (void)hipFree(P->d_cursor);
    (void)hipFree(P->d_images);
    for (int i = 0; i < kImageRing; ++i) {
        if (P->ev_images[i]) {
            (void)hipEventSynchronize(P->ev_images[i]);
            (void)hipEventDestroy(P->ev_images[i]);
        }
        if (P->h_images[i]) (void)hipHostFree(P->h_images[i]);
        if (P->ev_scenes[i]) {
            (void)hipEventSynchronize(P->ev_scenes[i]);
            (void)hipEventDestroy(P->ev_scenes[i]);
        }
        if (P->h_scenes[i]) (void)hipHostFree(P->h_scenes[i]);
    }
    (void)hipFree(P->d_acc);
    delete P;
}

// Batch signature for the tuning cache: device and the work of every scene.
std::string signature(gpss_scene* const* scenes, uint32_t n, int cus) {
    std::ostringstream o;
    o << "sched;cus" << cus;
    for (uint32_t i = 0; i < n; ++i) {
        const gpss_scene_desc& D = scenes[i]->desc;
        o << ";" << D.mean_kind << "," << D.n_prims << "," << D.width << "x" << D.height << "," << D.spp << ","
          << D.max_depth << "," << D.lengthscale << "," << D.variance << "," << D.majorant_res[0];
    }
    return o.str();
}

std::string cache_path() {
    if (const char* p = std::getenv("GPSS_TUNE_CACHE")) return p;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/gpss_batch_tuning.txt";
}

bool cache_lookup(const std::string& sig, uint32_t& tile, uint32_t& wpc) {
    std::ifstream f(cache_path());
    std::string line;
    size_t h = std::hash<std::string>{}(sig);
    while (std::getline(f, line)) {
        std::istringstream l(line);
        size_t key;
        uint32_t t, w;
        if (l >> key >> t >> w && key == h) {
            tile = t;
            wpc = w;
        }
    }
    return tile != 0;
}

void cache_store(const std::string& sig, uint32_t tile, uint32_t wpc) {
    const std::string path = cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) {
        const std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)   // create the directory, parents first
            if (i == dir.size() || dir[i] == '/') (void)::mkdir(dir.substr(0, i).c_str(), 0755);
    }
    std::ofstream f(path, std::ios::app);
    f << std::hash<std::string>{}(sig) << " " << tile << " " << wpc << "\n";
}
}  // namespace

int get_cus(int device, int& cus) {
    return check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device),
                     "hipDeviceGetAttribute");
}

static int build_plan(gpss_scene* const* scenes, uint32_t n, uint32_t tile, uint32_t waves_per_cu, BatchPlan** out) {
    BatchPlan* P = new (std::nothrow) BatchPlan();
    if (!P) return set_error(GPSS_ERR_OOM, "host allocation");
    P->scenes.assign(scenes, scenes + n);
    int cus = 0;
    int rc = get_cus(scenes[0]->device, cus);
    P->tile = tile;
    P->grid = std::max(1u, (uint32_t)std::max(1, cus) * waves_per_cu / 4u);
    std::vector<Tile> tiles;
    std::vector<BatchScene> recs(n);
    uint64_t pbase = 0, xbase = 0;
    for (uint32_t i = 0; i < n && !rc; ++i) {
        const gpss_scene* s = scenes[i];
        BatchScene& B = recs[i];
        B.S = s->dev;
        B.spp = s->desc.spp;
        B.npix = (uint32_t)s->n_pixels();
        B.pix_base = xbase;
        const uint64_t np = s->n_pixels() * s->desc.spp;
        for (uint64_t p0 = 0; p0 < np; p0 += tile)
            tiles.push_back(Tile{i, (uint32_t)std::min<uint64_t>(tile, np - p0), p0});
        pbase += np;
        xbase += s->n_pixels();
    }
    P->versions.resize(n);
    for (uint32_t i = 0; i < n; ++i) P->versions[i] = scenes[i]->dev_version;
    P->total_paths = pbase;
    P->total_pix = xbase;
    P->ntiles = (uint32_t)tiles.size();
    if (!rc) rc = check_hip(hipMalloc(&P->d_scenes, n * sizeof(BatchScene)), "hipMalloc");
    if (!rc)
        rc = check_hip(hipMemcpy(P->d_scenes, recs.data(), n * sizeof(BatchScene), hipMemcpyHostToDevice),
                       "hipMemcpy batch scenes");
    if (!rc) rc = check_hip(hipMalloc(&P->d_tiles, tiles.size() * sizeof(Tile)), "hipMalloc");
    if (!rc)
        rc = check_hip(hipMemcpy(P->d_tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice),
                       "hipMemcpy tiles");
    if (!rc) rc = check_hip(hipMalloc(&P->d_cursor, 64), "hipMalloc");
    if (!rc) rc = check_hip(hipMalloc(&P->d_images, n * sizeof(float*)), "hipMalloc");
    for (int i = 0; i < kImageRing && !rc; ++i) {
        rc = check_hip(hipHostMalloc(reinterpret_cast<void**>(&P->h_images[i]), n * sizeof(float*)), "hipHostMalloc");
        if (!rc) rc = check_hip(hipEventCreateWithFlags(&P->ev_images[i], hipEventDisableTiming), "hipEventCreate");
        if (!rc)
            rc = check_hip(hipHostMalloc(reinterpret_cast<void**>(&P->h_scenes[i]), n * sizeof(BatchScene)),
                           "hipHostMalloc");
        if (!rc) rc = check_hip(hipEventCreateWithFlags(&P->ev_scenes[i], hipEventDisableTiming), "hipEventCreate");
        if (!rc) std::copy(recs.begin(), recs.end(), P->h_scenes[i]);
    }
    if (!rc)
        rc = check_hip(hipMalloc(&P->d_acc, 2 * std::max<uint64_t>(1, xbase) * sizeof(unsigned long long)),
                       "hipMalloc(batch accumulator)");
    if (rc) {
        free_plan(P);
        return rc;
    }
    *out = P;
    return GPSS_OK;
}

static int capture_graph(BatchPlan* P) {
    hipStream_t cs;
    int rc = check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    if (rc) return rc;
    rc = check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (!rc) {
        const uint64_t nw = 2 * P->total_pix;
        hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, cs, P->d_cursor);
        hipLaunchKernelGGL(batch_clear_kernel, dim3((uint32_t)((nw + 255) / 256)), dim3(256), 0, cs, P->d_acc, nw);
        auto kernel = P->med == kMedIso     ? batch_kernel<kMedIso>
                      : P->med == kMedGgx   ? batch_kernel<kMedGgx>
                      : P->med == kMedAniso ? batch_kernel<kMedAniso>
                                            : batch_kernel<kMedAny>;
        hipLaunchKernelGGL(kernel, dim3(P->grid), dim3(256), 0, cs, P->d_scenes, P->d_tiles, P->ntiles, P->d_cursor,
                           P->d_acc);
        hipLaunchKernelGGL(batch_image_kernel, dim3((uint32_t)((P->total_pix + 255) / 256)), dim3(256), 0, cs,
                           P->d_scenes, (uint32_t)P->scenes.size(), P->d_images, P->d_acc, P->total_pix);
        hipGraph_t g = nullptr;
        rc = check_hip(hipStreamEndCapture(cs, &g), "hipStreamEndCapture");
        if (!rc) {
            P->graph = g;
            rc = check_hip(hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
    }
    (void)hipStreamDestroy(cs);
    return rc;
}

// Upload changed scene records and image pointers, then launch the plan's graph on `stream`.
// Everything is ordered on `stream`; the call does not wait for the batch.
static int run_plan(BatchPlan* P, float* const* images, hipStream_t stream) {
    const uint32_t n = (uint32_t)P->scenes.size();
    int rc = GPSS_OK;
    bool stale = false;   // a scene's parameters changed since its record was copied
    for (uint32_t i = 0; i < n; ++i) stale |= P->versions[i] != P->scenes[i]->dev_version;
    if (stale) {
        const int slot = P->ring_scenes;
        P->ring_scenes = (P->ring_scenes + 1) % kImageRing;
        rc = check_hip(hipEventSynchronize(P->ev_scenes[slot]), "hipEventSynchronize(scene records)");
        if (rc) return rc;
        for (uint32_t i = 0; i < n; ++i) {
            P->h_scenes[slot][i].S = P->scenes[i]->dev;
            P->versions[i] = P->scenes[i]->dev_version;
        }
        rc = check_hip(hipMemcpyAsync(P->d_scenes, P->h_scenes[slot], n * sizeof(BatchScene), hipMemcpyHostToDevice,
                                      stream),
                       "hipMemcpyAsync(batch scenes)");
        if (!rc) rc = check_hip(hipEventRecord(P->ev_scenes[slot], stream), "hipEventRecord");
        if (rc) return rc;
    }
    if (P->images_set.size() != n || !std::equal(P->images_set.begin(), P->images_set.end(), images)) {
        const int slot = P->ring;
        P->ring = (P->ring + 1) % kImageRing;
        rc = check_hip(hipEventSynchronize(P->ev_images[slot]), "hipEventSynchronize(image pointers)");
        if (rc) return rc;
        std::copy(images, images + n, P->h_images[slot]);
        rc = check_hip(hipMemcpyAsync(P->d_images, P->h_images[slot], n * sizeof(float*), hipMemcpyHostToDevice,
                                      stream),
                       "hipMemcpyAsync(batch images)");
        if (!rc) rc = check_hip(hipEventRecord(P->ev_images[slot], stream), "hipEventRecord");
        if (rc) return rc;
        P->images_set.assign(images, images + n);
    }
    // the medium kind the scenes share now (parameter changes can change it): the graph is
    // captured again when it launches another batch_kernel instance
    int med = medium_of(P->scenes[0]->dev);
    for (uint32_t i = 1; i < n && med != kMedAny; ++i)
        if (medium_of(P->scenes[i]->dev) != med) med = kMedAny;
    if (P->exec && med != P->med) {
        rc = check_hip(hipGraphExecDestroy(P->exec), "hipGraphExecDestroy");
        if (!rc) rc = check_hip(hipGraphDestroy(P->graph), "hipGraphDestroy");
        P->exec = nullptr;
        P->graph = nullptr;
        if (rc) return rc;
    }
    P->med = med;
    if (!P->exec) rc = capture_graph(P);
    if (!rc) rc = check_hip(hipGraphLaunch(P->exec, stream), "hipGraphLaunch");
    return rc;
}

static BatchPlan* find_plan(gpss_scene* const* scenes, uint32_t n) {
    for (BatchPlan* P : g_plans)
        if (P->scenes.size() == n && std::equal(P->scenes.begin(), P->scenes.end(), scenes)) return P;
    return nullptr;
}

void forget_scene_plans(gpss_scene* s) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::find((*it)->scenes.begin(), (*it)->scenes.end(), s) != (*it)->scenes.end()) {
            free_plan(*it);
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
}

static int validate_batch(gpss_scene* const* scenes, uint32_t n, float* const* images) {
    if (!scenes || !images || n == 0) return set_error(GPSS_ERR_INVALID_ARG, "empty or NULL batch");
    for (uint32_t i = 0; i < n; ++i) {
        if (!scenes[i] || !images[i]) return set_error(GPSS_ERR_INVALID_ARG, "NULL scene or image %u", i);
        if (scenes[i]->device != scenes[0]->device)
            return set_error(GPSS_ERR_INVALID_ARG, "scenes of one batch must share a device");
        if (scenes[i]->dev.n_obs > 0)
            return set_error(GPSS_ERR_UNSUPPORTED, "scene %u is a conditioned GP: render it with gpss_render", i);
    }
    return GPSS_OK;
}

int render_batch(gpss_scene* const* scenes, uint32_t n, float* const* images, hipStream_t stream) {
    int rc = validate_batch(scenes, n, images);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    BatchPlan* P = find_plan(scenes, n);
    if (!P) {
        int cus = 0;
        rc = get_cus(scenes[0]->device, cus);
        if (rc) return rc;
        uint32_t tile = 0, wpc = 4u * GPSS_SCHED_MIN_WAVES;
        if (!cache_lookup(signature(scenes, n, cus), tile, wpc)) {
            tile = 4096;
            wpc = 4u * GPSS_SCHED_MIN_WAVES;
        }
        rc = build_plan(scenes, n, tile, wpc, &P);
        if (rc) return rc;
        g_plans.push_back(P);
    }
    return run_plan(P, images, stream);
}

// Time every candidate (tile size x persistent waves per CU) on the batch itself, keep the
// fastest as the batch's plan and append it to the on-disk cache.
int autotune_batch(gpss_scene* const* scenes, uint32_t n, float* const* images, hipStream_t stream,
                   uint32_t* best_tile, uint32_t* best_wpc, float* best_ms) {
    int rc = validate_batch(scenes, n, images);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    int cus = 0;
    rc = get_cus(scenes[0]->device, cus);
    if (rc) return rc;
    const uint32_t tiles[] = {1024, 4096, 16384};
    const uint32_t wpcs[] = {4u * (GPSS_SCHED_MIN_WAVES - 1), 4u * GPSS_SCHED_MIN_WAVES};
    float bms = 1e30f;
    BatchPlan* best = nullptr;
    hipEvent_t e0, e1;
    rc = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (!rc) rc = check_hip(hipEventCreate(&e1), "hipEventCreate");
    for (uint32_t t : tiles) {
        for (uint32_t w : wpcs) {
            if (rc) break;
            BatchPlan* P = nullptr;
            rc = build_plan(scenes, n, t, w, &P);
            if (rc) break;
            rc = run_plan(P, images, stream);   // capture + warm-up
            if (!rc) rc = check_hip(hipEventRecord(e0, stream), "hipEventRecord");
            if (!rc) rc = run_plan(P, images, stream);
            if (!rc) rc = check_hip(hipEventRecord(e1, stream), "hipEventRecord");
            if (!rc) rc = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.0f;
            if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (!rc && ms < bms) {
                bms = ms;
                std::swap(best, P);
            }
            free_plan(P);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        free_plan(best);
        return rc;
    }
    BatchPlan* old = find_plan(scenes, n);
    if (old) {
        g_plans.erase(std::find(g_plans.begin(), g_plans.end(), old));
        free_plan(old);
    }
    g_plans.push_back(best);
    cache_store(signature(scenes, n, cus), best->tile, best->grid * 4u / (uint32_t)std::max(1, cus));
    if (best_tile) *best_tile = best->tile;
    if (best_wpc) *best_wpc = best->grid * 4u / (uint32_t)std::max(1, cus);
    if (best_ms) *best_ms = bms;
    return GPSS_OK;
}

}  // namespace gpss
