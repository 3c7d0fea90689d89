// ray_geom.h -- queue slots, pinhole rays and the slab test against the grid
// box, shared by the tracer and the gather microbenchmark that replays its
// rays (internal).
#pragma once

#include "haze_device.h"

namespace haze {

// Unit direction of pixel (p, q) of a view (q = 0 at the top), through the
// pixel centre.
__device__ __forceinline__ float3 pixel_dir(const TraceJob &J, int32_t p, int32_t q)
{
    const float sx = (float)p + 0.5f - J.half_w;
    const float sy = (float)q + 0.5f - J.half_h;
    float dx = J.fpx * J.f[0] + sx * J.r[0] - sy * J.u[0];
    float dy = J.fpx * J.f[1] + sx * J.r[1] - sy * J.u[1];
    float dz = J.fpx * J.f[2] + sx * J.r[2] - sy * J.u[2];
    const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    return make_float3(dx * inv, dy * inv, dz * inv);
}

// Slab test; on a hit returns the entry parameter clamped at 0 (and the exit
// parameter in t1 when asked).
__device__ __forceinline__ bool enter_volume(const TraceGrid &G, const float o[3], const float d[3], float &t0,
                                             float *t1 = nullptr)
{
    float a = -INFINITY, b = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0f) {
            if (o[k] < G.lo[k] || o[k] > G.hi[k]) return false;
            continue;
        }
        const float inv = 1.0f / d[k];
        float t1 = (G.lo[k] - o[k]) * inv, t2 = (G.hi[k] - o[k]) * inv;
        a = fmaxf(a, fminf(t1, t2));
        b = fminf(b, fmaxf(t1, t2));
    }
    if (a > b || b <= 0.0f) return false;
    t0 = fmaxf(a, 0.0f);
    if (t1) *t1 = b;
    return true;
}

// A queue slot's ray: its view (job), pixel and output index.
struct Ray {
    int32_t job;
    int32_t p, q;
    int64_t out;      // output index (flat index in subset mode, q * W + p otherwise)
};

// The view (job) whose tiles hold queue slot `slot` (not in subset mode).
// With a wave-uniform slot (the first of a wave's 64, one 8x8 tile of one
// view) the search runs on wave-uniform loads.
__device__ __forceinline__ int job_of_slot(const TraceJob *jobs, int njobs, int64_t slot)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].slot_begin <= slot)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// A queue slot of view J = jobs[job] (not in subset mode) to its pixel and
// output index; false for the padding slots of partial 8x8 tiles.
__device__ __forceinline__ bool decode_tile_slot(const TraceJob &J, int job, int64_t slot, Ray &r)
{
    const int32_t local = (int32_t)(slot - J.slot_begin);
    const int32_t tile = local >> 6;
    const int32_t within = local & 63;
    const int32_t ty = tile / J.tiles_x;
    r.job = job;
    // column-major inside the tile: consecutive slots (lanes) are vertically
    // adjacent pixels, whose rays sit at nearly the same height; with z the
    // field's fastest axis their gathers fall in the same cache lines, which
    // the texture-address unit serves together
    r.p = (tile - ty * J.tiles_x) * 8 + (within >> 3);
    r.q = ty * 8 + (within & 7);
    r.out = r.q * J.width + r.p;
    return r.p < J.width && r.q < J.height;
}

// Map a queue slot to its view (job), pixel and output index; false for the
// padding slots of partial 8x8 tiles.
__device__ __forceinline__ bool decode_slot(const TraceLaunch &L, int64_t slot, Ray &r)
{
    // all slot and ray counts are below 2^31 (checked on the host): 32-bit
    // division from here on
    if (L.subset) {
        const int64_t id = L.ray_ids[slot];
        int lo = 0, hi = L.njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.jobs[mid].ray_begin <= id)
                lo = mid;
            else
                hi = mid - 1;
        }
        const TraceJob &J = L.jobs[lo];
        const int64_t local64 = id - J.ray_begin;
        if (local64 < 0 || local64 >= (int64_t)J.width * J.height) return false;
        const int32_t local = (int32_t)local64;
        r.job = lo;
        r.q = local / J.width;
        r.p = local - r.q * J.width;
        r.out = slot;
        return true;
    }
    const int job = job_of_slot(L.jobs, L.njobs, slot);
    return decode_tile_slot(L.jobs[job], job, slot, r);
}

}  // namespace haze
