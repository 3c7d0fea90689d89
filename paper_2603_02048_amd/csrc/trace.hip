// trace.hip -- curved-ray marching through the refractive-index field on gfx950.
//
// Paper Sec. 3.3.2-3.3.3.  Inside the volume every ray follows the explicit
// update of Eq. 16,
//     omega_{k+1} = normalize(omega_k + ds_k / n_k (I - omega_k omega_k^T) g_k)
//     C_{k+1}     = C_k + ds_k omega_{k+1},
// with n_k and g_k trilinearly sampled from the gridded (delta_n, grad n)
// (Sec. 3.3.1) and the step of Eq. 18,
//     ds_k = clamp(n_k theta_max / (|(I - omega omega^T) g_k| + eps), ds_min, ds_max),
// or the fixed step of Sec. 4.1.  Outside the volume rays are straight (Fig. 1
// caption); the image is formed only by bending (Sec. 3.3.2): the exit ray is
// intersected with a backdrop plane and re-projected through the same pinhole.
//
// Two launches per trace:
//   k_raygen  one thread per queue slot: pinhole ray, slab test against the
//             volume; rays that miss are finished at once, rays that enter
//             are appended to a compact hit list (wave ballot + mbcnt + one
//             atomic per wave)
//   k_march   persistent waves pull hit rays from the list; when enough lanes
//             have finished, the idle lanes are refilled together (ballot of
//             idle lanes, one atomic per wave, mbcnt rank), which keeps the
//             wave busy despite the spread of step counts adaptive stepping
//             causes.  Each ray's arithmetic is independent of which lane or
//             wave runs it, so results are bitwise repeatable.
//
// Positions are float32 metres with a compensated (Kahan) sum of the steps.
// The direction is carried as an unnormalised vector p = wr + dw (entry
// direction plus accumulated turns); since normalize() ignores scale, adding
// |p| ds/n P g to p reproduces Eq. 16 exactly while dw keeps the low-order bits
// of many small turns that a unit vector would round away.
#include "haze_device.h"

#include <hip/hip_fp16.h>

namespace haze {

struct Ray {
    int32_t job;
    int32_t p, q;
    int64_t out;      // output index (flat index in subset mode, q * W + p otherwise)
};

// Map a queue slot to its view (job), pixel and output index; false for the
// padding slots of partial 8x8 tiles.
__device__ __forceinline__ bool decode_slot(const TraceLaunch &L, int64_t slot, Ray &r)
{
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
        const int64_t local = id - J.ray_begin;
        r.job = lo;
        r.p = (int32_t)(local % J.width);
        r.q = (int32_t)(local / J.width);
        r.out = slot;
        return local >= 0 && r.q < J.height;
    }
    int lo = 0, hi = L.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.jobs[mid].slot_begin <= slot)
            lo = mid;
        else
            hi = mid - 1;
    }
    const TraceJob &J = L.jobs[lo];
    const int64_t local = slot - J.slot_begin;
    const int64_t tile = local >> 6;
    const int32_t within = (int32_t)(local & 63);
    r.job = lo;
    r.p = (int32_t)(tile % J.tiles_x) * 8 + (within & 7);
    r.q = (int32_t)(tile / J.tiles_x) * 8 + (within >> 3);
    r.out = (int64_t)r.q * J.width + r.p;
    return r.p < J.width && r.q < J.height;
}

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

// Slab test; on a hit returns the entry parameter clamped at 0.
__device__ __forceinline__ bool enter_volume(const TraceGrid &G, const float o[3], const float d[3], float &t0)
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
    return true;
}

// Exit distance along w from a point in the volume (clamped at 0).
__device__ __forceinline__ float exit_distance(const TraceGrid &G, const float c[3], const float w[3])
{
    float t = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (w[k] > 0.0f)
            t = fminf(t, (G.hi[k] - c[k]) / w[k]);
        else if (w[k] < 0.0f)
            t = fminf(t, (G.lo[k] - c[k]) / w[k]);
    }
    return fmaxf(t, 0.0f);
}

// Exit ray -> backdrop plane -> re-projection -> displacement; writes outputs.
__device__ __forceinline__ void finish_ray(const TraceLaunch &L, const Ray &r, const float x[3], const float w[3],
                                           uint32_t steps, int status)
{
    const TraceJob &J = L.jobs[r.job];
    float disp0 = __builtin_nanf(""), disp1 = __builtin_nanf("");
    if (status != 3) {
        const float denom = w[0] * J.plane_n[0] + w[1] * J.plane_n[1] + w[2] * J.plane_n[2];
        bool hit = denom < 0.0f;
        float t = 0.0f;
        if (hit) {
            t = ((J.plane_p[0] - x[0]) * J.plane_n[0] + (J.plane_p[1] - x[1]) * J.plane_n[1] +
                 (J.plane_p[2] - x[2]) * J.plane_n[2]) / denom;
            hit = t >= 0.0f;
        }
        float zc = 0.0f, xc = 0.0f, yc = 0.0f;
        if (hit) {
            const float hx = x[0] + t * w[0] - J.eye[0];
            const float hy = x[1] + t * w[1] - J.eye[1];
            const float hz = x[2] + t * w[2] - J.eye[2];
            xc = hx * J.r[0] + hy * J.r[1] + hz * J.r[2];
            yc = hx * J.u[0] + hy * J.u[1] + hz * J.u[2];
            zc = hx * J.f[0] + hy * J.f[1] + hz * J.f[2];
            hit = zc > 0.0f;
        }
        if (hit) {
            disp0 = (J.half_w + J.fpx * xc / zc) - ((float)r.p + 0.5f);
            disp1 = (J.half_h - J.fpx * yc / zc) - ((float)r.q + 0.5f);
        } else if (status == 0) {
            status = 2;
        }
    }
    float *disp, *ep, *ed;
    uint32_t *st;
    uint8_t *stat;
    if (L.subset) {
        disp = L.flat.disp; ep = L.flat.exit_pos; ed = L.flat.exit_dir; st = L.flat.steps; stat = L.flat.status;
    } else {
        disp = J.disp; ep = J.exit_pos; ed = J.exit_dir; st = J.steps; stat = J.status;
    }
    const int64_t o = r.out;
    if (disp) {
        disp[2 * o] = disp0;
        disp[2 * o + 1] = disp1;
    }
    if (ep) {
        ep[3 * o] = x[0];
        ep[3 * o + 1] = x[1];
        ep[3 * o + 2] = x[2];
    }
    if (ed) {
        ed[3 * o] = w[0];
        ed[3 * o + 1] = w[1];
        ed[3 * o + 2] = w[2];
    }
    if (st) st[o] = steps;
    if (stat) stat[o] = (uint8_t)status;
}

__global__ void k_trace_init(uint32_t *counters)
{
    if (threadIdx.x < 2) counters[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_raygen(TraceLaunch L)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool enters = false;
    if (slot < L.nslots) {
        Ray r;
        if (decode_slot(L, slot, r)) {
            const TraceJob &J = L.jobs[r.job];
            const float3 d3 = pixel_dir(J, r.p, r.q);
            const float d[3] = {d3.x, d3.y, d3.z};
            float t0;
            enters = enter_volume(L.grid, J.eye, d, t0);
            if (!enters) finish_ray(L, r, J.eye, d, 0u, 0);
        } else if (L.subset) {
            // ray id outside the views: flag it, leave no stale values behind
            const float nan = __builtin_nanf("");
            if (L.flat.disp) L.flat.disp[2 * slot] = L.flat.disp[2 * slot + 1] = nan;
            if (L.flat.exit_pos)
                L.flat.exit_pos[3 * slot] = L.flat.exit_pos[3 * slot + 1] = L.flat.exit_pos[3 * slot + 2] = nan;
            if (L.flat.exit_dir)
                L.flat.exit_dir[3 * slot] = L.flat.exit_dir[3 * slot + 1] = L.flat.exit_dir[3 * slot + 2] = nan;
            if (L.flat.steps) L.flat.steps[slot] = 0u;
            if (L.flat.status) L.flat.status[slot] = 4u;
        }
    }
    // wave-aggregated append of the entering slots
    const uint64_t mask = __ballot(enters);
    if (mask == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&L.counters[0], (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (enters) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        L.hits[base + rank] = (uint32_t)slot;
    }
}

template <int DT>
__device__ __forceinline__ float4 load_voxel(const void *__restrict__ f, int64_t i, float inv_scale)
{
    if (DT == DT_F32) {
        return reinterpret_cast<const float4 *>(f)[i];
    } else {
        const ushort4 h = reinterpret_cast<const ushort4 *>(f)[i];
        float4 v;
        if (DT == DT_F16) {
            v = make_float4(__half2float(__ushort_as_half(h.x)), __half2float(__ushort_as_half(h.y)),
                            __half2float(__ushort_as_half(h.z)), __half2float(__ushort_as_half(h.w)));
        } else {
            v = make_float4(__uint_as_float((uint32_t)h.x << 16), __uint_as_float((uint32_t)h.y << 16),
                            __uint_as_float((uint32_t)h.z << 16), __uint_as_float((uint32_t)h.w << 16));
        }
        v.x *= inv_scale;
        v.y *= inv_scale;
        v.z *= inv_scale;
        v.w *= inv_scale;
        return v;
    }
}

__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float t)
{
    return make_float4(fmaf(t, b.x - a.x, a.x), fmaf(t, b.y - a.y, a.y), fmaf(t, b.z - a.z, a.z),
                       fmaf(t, b.w - a.w, a.w));
}

// Trilinear (delta_n, g) at x: cell index clamped to [0, R-2], so the outer
// half-voxel extrapolates linearly.
template <int DT>
__device__ __forceinline__ float4 sample_field(const TraceGrid &G, const void *__restrict__ f, const float x[3])
{
    int32_t i[3];
    float t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = fmaf(x[a], G.inv_sp[a], G.off[a]);
        const float fl = fminf(fmaxf(floorf(u), 0.0f), G.maxi[a]);
        i[a] = (int32_t)fl;
        t[a] = u - fl;
    }
    const int64_t sy = G.res[0], sz = (int64_t)G.res[0] * G.res[1];
    const int64_t b = ((int64_t)i[2] * G.res[1] + i[1]) * G.res[0] + i[0];
    const float4 c000 = load_voxel<DT>(f, b, G.inv_scale);
    const float4 c100 = load_voxel<DT>(f, b + 1, G.inv_scale);
    const float4 c010 = load_voxel<DT>(f, b + sy, G.inv_scale);
    const float4 c110 = load_voxel<DT>(f, b + sy + 1, G.inv_scale);
    const float4 c001 = load_voxel<DT>(f, b + sz, G.inv_scale);
    const float4 c101 = load_voxel<DT>(f, b + sz + 1, G.inv_scale);
    const float4 c011 = load_voxel<DT>(f, b + sz + sy, G.inv_scale);
    const float4 c111 = load_voxel<DT>(f, b + sz + sy + 1, G.inv_scale);
    const float4 x00 = lerp4(c000, c100, t[0]);
    const float4 x10 = lerp4(c010, c110, t[0]);
    const float4 x01 = lerp4(c001, c101, t[0]);
    const float4 x11 = lerp4(c011, c111, t[0]);
    const float4 y0 = lerp4(x00, x10, t[1]);
    const float4 y1 = lerp4(x01, x11, t[1]);
    return lerp4(y0, y1, t[2]);
}

template <int DT>
__global__ __launch_bounds__(256) void k_march(TraceLaunch L)
{
    const TraceGrid &G = L.grid;
    const TraceStep &S = L.step;
    const uint32_t nh = L.counters[0];
    const uint32_t refill_min = (uint32_t)max(1, min(64, L.refill_min));
    const int lane = threadIdx.x & 63;

    bool active = false;
    bool drained = false;
    Ray r{0, 0, 0, 0};
    const void *field = nullptr;
    // direction omega = p / |p| with p = wr + dw: wr is the entry direction and
    // dw accumulates the turns, so small turns keep their low-order bits
    float c[3] = {0, 0, 0}, cc[3] = {0, 0, 0}, w[3] = {0, 0, 1}, wr[3] = {0, 0, 1}, dw[3] = {0, 0, 0};
    float pnorm = 1.0f;
    uint32_t steps = 0;

    for (;;) {
        uint64_t idle = __ballot(!active);
        if ((!drained && (uint32_t)__popcll(idle) >= refill_min) || idle == ~0ull) {
            if (drained) break;
            const uint32_t nidle = (uint32_t)__popcll(idle);
            const int leader = __ffsll((unsigned long long)idle) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&L.counters[1], nidle);
            base = __shfl(base, leader);
            if (base + nidle >= nh) drained = true;
            if (!active) {
                const uint32_t k = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (k < nh) {
                    const int64_t slot = L.hits[k];
                    decode_slot(L, slot, r);
                    const TraceJob &J = L.jobs[r.job];
                    field = J.field;
                    const float3 d3 = pixel_dir(J, r.p, r.q);
                    w[0] = d3.x; w[1] = d3.y; w[2] = d3.z;
                    wr[0] = d3.x; wr[1] = d3.y; wr[2] = d3.z;
                    dw[0] = dw[1] = dw[2] = 0.0f;
                    pnorm = sqrtf(d3.x * d3.x + d3.y * d3.y + d3.z * d3.z);
                    float t0 = 0.0f;
                    enter_volume(G, J.eye, w, t0);
                    c[0] = J.eye[0] + t0 * w[0];
                    c[1] = J.eye[1] + t0 * w[1];
                    c[2] = J.eye[2] + t0 * w[2];
                    cc[0] = cc[1] = cc[2] = 0.0f;
                    steps = 0;
                    active = true;
                }
            }
            continue;
        }
        if (!active) continue;

        // ---- one step of Eq. 16 with the step of Eq. 18 ----
        const float dmin = fminf(fminf(fminf(c[0] - G.lo[0], G.hi[0] - c[0]), fminf(c[1] - G.lo[1], G.hi[1] - c[1])),
                                 fminf(c[2] - G.lo[2], G.hi[2] - c[2]));
        const bool near = dmin <= S.near_cap;
        float te = INFINITY;
        int status = -1;
        if (near) {
            te = exit_distance(G, c, w);
            if (te <= S.tau) status = 0;
        }
        if (status < 0) {
            const float4 s = sample_field<DT>(G, field, c);
            const float n = 1.0f + s.x;
            const float wg = w[0] * s.y + w[1] * s.z + w[2] * s.w;
            const float pg0 = s.y - wg * w[0], pg1 = s.z - wg * w[1], pg2 = s.w - wg * w[2];
            float ds;
            if (S.uniform) {
                ds = S.ds_uniform;
            } else {
                const float pgn = sqrtf(pg0 * pg0 + pg1 * pg1 + pg2 * pg2);
                ds = fminf(fmaxf(n * S.theta_max / (pgn + S.eps), S.ds_min), S.ds_max);
            }
            ds = fminf(ds, te);
            // omega_{k+1} = normalize(omega_k + ds/n P g) = normalize(p + |p| ds/n P g)
            const float a = ds / n * pnorm;
            dw[0] = fmaf(a, pg0, dw[0]);
            dw[1] = fmaf(a, pg1, dw[1]);
            dw[2] = fmaf(a, pg2, dw[2]);
            const float p0 = wr[0] + dw[0], p1 = wr[1] + dw[1], p2 = wr[2] + dw[2];
            pnorm = sqrtf(p0 * p0 + p1 * p1 + p2 * p2);
            const float inv = 1.0f / pnorm;
            w[0] = p0 * inv;
            w[1] = p1 * inv;
            w[2] = p2 * inv;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                // compensated C += ds * w
                const float y = fmaf(ds, w[k], -cc[k]);
                const float t = c[k] + y;
                cc[k] = (t - c[k]) - y;
                c[k] = t;
            }
            ++steps;
            const bool fin = isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]) && isfinite(w[0]) &&
                             isfinite(w[1]) && isfinite(w[2]) && isfinite(n);
            if (!fin)
                status = 3;
            else if (c[0] < G.lo[0] || c[0] > G.hi[0] || c[1] < G.lo[1] || c[1] > G.hi[1] || c[2] < G.lo[2] ||
                     c[2] > G.hi[2])
                status = 0;
            else if ((int32_t)steps >= S.max_steps)
                status = 1;
        }
        if (status >= 0) {
            finish_ray(L, r, c, w, steps, status);
            active = false;
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

hipError_t launch_raygen(const TraceLaunch &L, hipStream_t s)
{
    hipLaunchKernelGGL(k_trace_init, dim3(1), dim3(64), 0, s, L.counters);
    if (L.nslots > 0)
        hipLaunchKernelGGL(k_raygen, dim3((unsigned)((L.nslots + 255) / 256)), dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_march(int dtype, const TraceLaunch &L, int march_blocks, hipStream_t s)
{
    if (dtype == DT_F32)
        hipLaunchKernelGGL(k_march<DT_F32>, dim3(march_blocks), dim3(256), 0, s, L);
    else if (dtype == DT_F16)
        hipLaunchKernelGGL(k_march<DT_F16>, dim3(march_blocks), dim3(256), 0, s, L);
    else
        hipLaunchKernelGGL(k_march<DT_BF16>, dim3(march_blocks), dim3(256), 0, s, L);
    return hipGetLastError();
}

int march_blocks_per_cu(int dtype)
{
    int nb = 0;
    hipError_t e;
    if (dtype == DT_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_march<DT_F32>, 256, 0);
    else if (dtype == DT_F16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_march<DT_F16>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_march<DT_BF16>, 256, 0);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace haze
