// ray_geom.h -- pinhole rays and the slab test against the grid box, shared
// by the tracer and the gather microbenchmark that replays its rays
// (internal).
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

}  // namespace haze
