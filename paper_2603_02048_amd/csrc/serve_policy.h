// serve_policy.h -- batching policy of the serving loop (pure host logic, no
// HIP), shared by serve.hip and the CPU tests of the policy.
#pragma once

#include <cstdint>
#include <cstring>
#include <vector>

namespace haze {

// What decides whether two requests can share one launch: the tracer's
// launch-uniform data (grid geometry, storage type and scale, step control,
// scene boards: each as origin, edge_u, edge_v; the triangle mesh, by
// identity).
constexpr int kKeyQuads = 8;
struct BatchKey {
    double lo[3], hi[3];
    int32_t res[3];
    int32_t dtype;
    float store_scale;
    int32_t uniform;
    float theta_max, ds_min, ds_max, eps, ds_uniform;
    int32_t max_steps;
    float tau_term;
    int32_t nquads;
    uint64_t mesh;   // the mesh scene's handle, 0 for none
    float quads[kKeyQuads][9];
};

inline bool same_key(const BatchKey &a, const BatchKey &b)
{
    return std::memcmp(&a, &b, sizeof(BatchKey)) == 0;
}

inline BatchKey zero_key()
{
    BatchKey k;
    std::memset(&k, 0, sizeof k);
    return k;
}

struct PendingInfo {
    BatchKey key;
    int64_t slots;       // queue slots (8x8-tile padded rays) the request needs
    int64_t out_bytes;   // device bytes of its outputs
};

// Choose the requests of the next launch, in arrival order: the oldest
// pending request starts the batch; later requests with the same key join
// while the batch's queue slots stay within `slot_capacity` and their output
// memory within `mem_avail`.  A request that does not fit is skipped (it
// keeps its place), so a large request never blocks smaller compatible ones
// behind it from joining this batch, but the oldest request always goes
// first.  Returns indices into `pending`; empty when even the oldest request
// does not fit `mem_avail` (admission waits for memory).
inline std::vector<size_t> plan_batch(const std::vector<PendingInfo> &pending, int64_t slot_capacity,
                                      int64_t mem_avail, size_t max_requests)
{
    std::vector<size_t> pick;
    if (pending.empty()) return pick;
    const PendingInfo &head = pending[0];
    if (head.slots > slot_capacity || head.out_bytes > mem_avail) return pick;
    int64_t slots = head.slots, mem = head.out_bytes;
    pick.push_back(0);
    for (size_t i = 1; i < pending.size() && pick.size() < max_requests; ++i) {
        const PendingInfo &p = pending[i];
        if (!same_key(p.key, head.key)) continue;
        if (slots + p.slots > slot_capacity || mem + p.out_bytes > mem_avail) continue;
        slots += p.slots;
        mem += p.out_bytes;
        pick.push_back(i);
    }
    return pick;
}

// Queue slots of a view: 8x8 pixel tiles, 64 slots each.
inline int64_t view_slots(int32_t width, int32_t height)
{
    return (int64_t)((width + 7) / 8) * ((height + 7) / 8) * 64;
}

// Device bytes of one ray's outputs: disp (2 f32), exit_pos (3 f32),
// exit_dir (3 f32), steps (u32), status (u8), surface (u8).
constexpr int64_t kOutBytesPerRay = 8 + 12 + 12 + 4 + 1 + 1;

// Request outputs come in size classes, four per octave from 64 KiB, so that
// a released block serves later requests of similar size: the class of a
// request of b bytes is the smallest p (1 + k/4), k = 0..4, p a power of two
// from 64 KiB with p <= b (64 KiB for smaller b), that holds b; at most 1.25 b
// above 64 KiB.
inline size_t out_class(int64_t bytes)
{
    size_t p = (size_t)64 << 10;
    while (p * 2 <= (size_t)bytes) p <<= 1;
    for (size_t k = 0; k <= 4; ++k)
        if ((size_t)bytes <= p + k * (p / 4)) return p + k * (p / 4);
    return 2 * p;
}

// A device block (pointer and bytes) the serving loop holds.
struct PoolBlock {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Released request outputs kept for reuse, keyed by size class.  Host
// bookkeeping only: the serving loop puts a block back once the request's
// batch has completed and its outputs have been released, so a block taken
// out is free on the device.
struct OutputPool {
    std::vector<PoolBlock> blocks;
    uint64_t bytes = 0;   // total held

    void put(void *ptr, size_t cls)
    {
        blocks.push_back({ptr, cls});
        bytes += cls;
    }
    // A held block of class `cls`, or nullptr.
    void *take(size_t cls)
    {
        for (size_t i = 0; i < blocks.size(); ++i)
            if (blocks[i].bytes == cls) {
                void *p = blocks[i].ptr;
                bytes -= cls;
                blocks[i] = blocks.back();
                blocks.pop_back();
                return p;
            }
        return nullptr;
    }
    // Everything held (to be freed), leaving the pool empty.
    std::vector<PoolBlock> drain()
    {
        std::vector<PoolBlock> all;
        all.swap(blocks);
        bytes = 0;
        return all;
    }
};

}  // namespace haze
