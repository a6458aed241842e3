// Wave-level helpers shared by the persistent kernels: lane masks, queue appends with one
// atomic per wave and a chunked reader of a work queue.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gpss {

constexpr uint32_t kChunk = 64;   // queue items taken per atomic (default)

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// Append `item` for lanes with `want` to queue q (counter *cnt): one atomic per wave.
__device__ __forceinline__ void wave_push(bool want, uint32_t item, uint32_t* __restrict__ q, uint32_t* cnt) {
    const uint64_t m = __ballot(want);
    if (m == 0) return;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (want) q[base + (uint32_t)__popcll(m & lanemask_lt())] = item;
}

// ---------------------------------------------------------------------------
// Persistent-wave chunked queue reader.
// ---------------------------------------------------------------------------
struct ChunkReader {
    uint32_t pos, end, n, step;   // step: items per claim (wave-uniform)
    bool exhausted;
    __device__ __forceinline__ void init(uint32_t n_items, uint32_t items_per_claim = kChunk) {
        pos = end = 0;
        n = n_items;
        step = items_per_claim;
        exhausted = false;
    }
    // Give each lane with `idle` the index of a queue item (true) while items remain.
    __device__ __forceinline__ bool take(bool idle, uint32_t* head, uint32_t& idx) {
        uint64_t m = __ballot(idle);
        bool got = false;
        while (m && !exhausted) {
            if (pos >= end) {
                uint32_t base = 0;
                if ((threadIdx.x & 63) == 0) base = atomicAdd(head, step);
                base = __shfl(base, 0, 64);
                if (base >= n) { exhausted = true; break; }
                pos = base;
                end = min(base + step, n);
            }
            const uint32_t avail = end - pos;
            const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt());
            const bool mine = idle && !got && ((m >> (threadIdx.x & 63)) & 1ull) && rank < avail;
            if (mine) {
                idx = pos + rank;
                got = true;
            }
            const uint32_t used = min((uint32_t)__popcll(m), avail);
            pos += used;
            m = __ballot(idle && !got);
        }
        return got;
    }
};

}  // namespace gpss
