// gpss_render_noalloc: the persistent forward render with its scratch memory in a fixed
// device array of this library instead of memory the scene allocates, for callers that
// cannot allocate (code under stream capture, serving loops, harnesses that forbid it).
//
// The scratch of a render is the per-pixel fixed-point sum (two 64-bit words per pixel,
// gpss_accum.hpp) and the path counter of the persistent kernel.  Here they live in
// `scratch`, a file-scope __device__ array of kNoAllocWords words: every device the library
// runs on holds its own copy until the process ends.  Its device address is taken once per
// device with hipGetSymbolAddress (the array's name in host code is not a device address);
// every later use goes through that pointer.  All calls on one device share the array, so
// calls that overlap on one device (different streams, threads) race; each call clears what
// must start at zero (sums and counter) on its stream before rendering.
#include <mutex>

#include "gpss_internal.hpp"

namespace gpss {

// 1024 x 1024 pixels (two words each) and one 256-byte block for the path counter.
constexpr uint64_t kNoAllocMaxPixels = 1ull << 20;
constexpr uint64_t kNoAllocCounterWords = 32;
constexpr uint64_t kNoAllocWords = 2 * kNoAllocMaxPixels + kNoAllocCounterWords;

static __device__ __align__(256) unsigned long long scratch[kNoAllocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (taken on the first call there).
int scratch_on_device(int device, unsigned long long** out) {
    if (device < 0 || device >= kMaxDevices)
        return set_error(GPSS_ERR_UNSUPPORTED, "device %d: at most %d devices", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (rc) return rc;
        g_scratch_ptr[device] = static_cast<unsigned long long*>(p);
    }
    *out = g_scratch_ptr[device];
    return GPSS_OK;
}
}  // namespace

int render_noalloc(gpss_scene* s, float* image, uint32_t s0, uint32_t s1, hipStream_t stream) {
    const uint64_t npix = s->n_pixels();
    if (npix > kNoAllocMaxPixels)
        return set_error(GPSS_ERR_INVALID_ARG,
                         "%llu pixels: gpss_render_noalloc holds at most %llu (its fixed scratch array); "
                         "use gpss_render",
                         (unsigned long long)npix, (unsigned long long)kNoAllocMaxPixels);
    int device = 0;
    int rc = check_hip(hipGetDevice(&device), "hipGetDevice");
    if (rc) return rc;
    if (device != s->device)
        return set_error(GPSS_ERR_INVALID_ARG, "the scene lives on device %d, the current device is %d", s->device,
                         device);
    unsigned long long* base = nullptr;
    rc = scratch_on_device(device, &base);
    if (rc) return rc;
    unsigned long long* acc = base;
    uint32_t* head = reinterpret_cast<uint32_t*>(base + 2 * kNoAllocMaxPixels);
    const uint32_t ns = s1 - s0;
    rc = launch_acc_clear(acc, npix, stream);
    if (!rc) rc = sched_render(s, nullptr, acc, nullptr, s0, ns, stream, head);
    if (!rc) rc = launch_acc_finalize(acc, image, ns, npix, stream);
    return rc;
}

}  // namespace gpss

extern "C" int gpss_render_noalloc(gpss_scene_t scene, float* image_dev, uint32_t s0, uint32_t s1,
                                   gpss_stream_t stream) {
    gpss::Range range("gpss_render_noalloc");
    if (!scene || !image_dev) return gpss::set_error(GPSS_ERR_INVALID_ARG, "NULL argument");
    if (int rc = gpss::check_path_count(scene, s0, s1)) return rc;
    return gpss::render_noalloc(scene, image_dev, s0, s1, reinterpret_cast<hipStream_t>(stream));
}
