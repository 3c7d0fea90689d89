// membench.hip -- achievable read bandwidth of the memory level a buffer of a
// given size lives in (HBM for buffers far above the 256 MB MALL, L2/MALL for
// field-sized buffers read repeatedly), and of the tracer's own access pattern
// (8-corner gathers along the benchmarked views' own pinhole rays, walked
// straight through a field-sized grid) with no arithmetic around it.  Used to
// put the tracer's gather rate next to what the memory system delivers.
#include "haze.h"
#include "ray_geom.h"
#include "serve.h"
#include "serve_policy.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

namespace haze {
hz_status make_job(const hz_view *v, const void *field, int64_t slot_begin, int64_t ray_begin, TraceJob *J,
                   const char *fn, int index);
void make_trace_grid(const hz_grid &g, float store_scale, TraceGrid *G);
float length_bin_scale(const hz_grid &g);
hipError_t launch_raygen(const TraceLaunch &, bool, hipStream_t, const KTimer &);

// Grid-stride read of n float4; each block writes one partial sum so the
// loads cannot be optimised away.
__global__ __launch_bounds__(256) void k_read(const float4 *__restrict__ a, int64_t n, float *__restrict__ sink)
{
    float acc = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float4 v = a[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    __shared__ float part[256];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = part[0];
}

__global__ void k_init(float4 *a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = make_float4(1.0f, 2.0f, 3.0f, 4.0f);
}

typedef uint32_t gb_u32x4 __attribute__((ext_vector_type(4), aligned(8)));
typedef const gb_u32x4 __attribute__((address_space(1))) *gb_ptr;

// One thread per entering ray, in the order of the tracer's length-sorted
// hit list (the order the march hands rays to its waves: 64 consecutive hits
// per wave, longest rays first): the thread casts its pixel's pinhole ray
// and walks straight through the grid box in steps of `step` metres from the
// entry point, reading at every sample the 8 corners of its cell as the
// marcher does (cell index clamped to [0, R-2]; the two z-neighbours of each
// of the 4 rows in one 16 or 32 byte stretch).  The words are folded into
// one value per thread so no load can be dropped; the samples are counted
// (one atomic per wave).
template <int EB>
__global__ __launch_bounds__(256) void k_gather_hits(const char *__restrict__ f, TraceLaunch L, uint32_t nh,
                                                     float step, uint32_t *__restrict__ sink,
                                                     unsigned long long *__restrict__ nsamples)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0u, n = 0u;
    if (k < nh) {
        Ray r;
        decode_slot(L, L.hits[k], r);
        const TraceJob &J = L.jobs[r.job];
        const float3 d3 = pixel_dir(J, r.p, r.q);
        const float d[3] = {d3.x, d3.y, d3.z};
        float t0 = 0.0f, t1 = 0.0f;
        const bool in = enter_volume(L.grid, J.eye, d, t0, &t1);
        const TraceGrid &G = L.grid;
        // the packed field's layout: z fastest, then x, then y
        const uint32_t row = (uint32_t)G.res[2], slab = (uint32_t)G.res[0] * (uint32_t)G.res[2];
        for (uint32_t s = 0; in; ++s) {
            const float t = fmaf((float)s, step, t0);
            if (!(t < t1)) break;
            uint32_t i[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float u = fmaf(fmaf(t, d[a], J.eye[a]), G.inv_sp[a], G.off[a]);
                i[a] = (uint32_t)__builtin_amdgcn_fmed3f(floorf(u), 0.0f, G.maxi[a]);
            }
            const uint32_t b = (i[1] * slab + i[0] * row) + i[2];
            const uint32_t c[4] = {b, b + row, b + slab, b + slab + row};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const gb_ptr pp = (gb_ptr)(f + (size_t)c[j] * EB);
                const gb_u32x4 a = pp[0];
                acc ^= (a.x ^ a.y) ^ (a.z ^ a.w);
                if (EB == 16) {
                    const gb_u32x4 b2 = pp[1];
                    acc ^= (b2.x ^ b2.y) ^ (b2.z ^ b2.w);
                }
            }
            ++n;
        }
        sink[k] = acc;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n += (uint32_t)__shfl_xor((int)n, off);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(nsamples, (unsigned long long)n);
}

}  // namespace haze

using namespace haze;

extern "C" hz_status hz_membench(hz_ctx *c, uint64_t bytes, int32_t reps, double *read_gbps, void *hip_stream)
{
    if (!c || !read_gbps) return set_error(HZ_E_INVALID, "hz_membench: NULL argument");
    if (bytes < 4096 || reps < 1 || reps > 10000) return set_error(HZ_E_INVALID, "hz_membench: bad size or reps");
    if (hipSetDevice(ctx_device(c)) != hipSuccess) return set_error(HZ_E_DEVICE, "hz_membench: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = (int64_t)(bytes / 16);
    const int blocks = ctx_num_cus(c) * 8;
    void *buf = nullptr, *sink = nullptr;
    hz_status st = ctx_alloc(c, &buf, (size_t)n * 16);
    if (st != HZ_OK) return st;
    st = ctx_alloc(c, &sink, sizeof(float) * (size_t)blocks);
    if (st != HZ_OK) {
        ctx_free(c, buf, (size_t)n * 16);
        return st;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (float4 *)buf, n);
        hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, s, (const float4 *)buf, n, (float *)sink);  // warm
        ok = hipEventRecord(e0, s) == hipSuccess;
        for (int r = 0; ok && r < reps; ++r)
            hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, s, (const float4 *)buf, n, (float *)sink);
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess && hipGetLastError() == hipSuccess;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx_free(c, buf, (size_t)n * 16);
    ctx_free(c, sink, sizeof(float) * (size_t)blocks);
    if (!ok || ms <= 0.0f) return set_error(HZ_E_DEVICE, "hz_membench: timing failed");
    *read_gbps = (double)n * 16.0 * reps / (ms * 1e-3) / 1e9;
    return HZ_OK;
}

extern "C" hz_status hz_membench_gather(hz_ctx *c, const hz_grid *grid, int32_t voxel_bytes, const hz_view *views,
                                        int32_t nviews, float step_len, int32_t reps, double *gather_gbps,
                                        int64_t *samples, void *hip_stream)
{
    if (!c || !grid || !views || !gather_gbps) return set_error(HZ_E_INVALID, "hz_membench_gather: NULL argument");
    if (voxel_bytes != 8 && voxel_bytes != 16)
        return set_error(HZ_E_INVALID, "hz_membench_gather: voxel_bytes not 8 or 16");
    int64_t nvox = 1;
    for (int a = 0; a < 3; ++a) {
        if (grid->res[a] < 2 || grid->res[a] > 65535 || !(grid->hi[a] > grid->lo[a]))
            return set_error(HZ_E_INVALID, "hz_membench_gather: grid res outside [2, 65535] or hi <= lo");
        nvox *= grid->res[a];
    }
    if (nvox >= (1ll << 31)) return set_error(HZ_E_INVALID, "hz_membench_gather: grid of 2^31 voxels or more");
    if (nviews < 1 || nviews > 4096 || reps < 1 || reps > 10000)
        return set_error(HZ_E_INVALID, "hz_membench_gather: nviews or reps out of range");
    double vox = 1e300;
    for (int a = 0; a < 3; ++a) vox = std::min(vox, (grid->hi[a] - grid->lo[a]) / grid->res[a]);
    if (!(step_len >= 1e-3 * vox && step_len <= 1e3 * vox))
        return set_error(HZ_E_INVALID, "hz_membench_gather: step_len outside [1e-3, 1e3] voxels");
    const size_t fbytes = (size_t)nvox * (size_t)voxel_bytes;
    if (hipSetDevice(ctx_device(c)) != hipSuccess) return set_error(HZ_E_DEVICE, "hz_membench_gather: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    void *buf = nullptr;
    hz_status st = ctx_alloc(c, &buf, fbytes);
    if (st != HZ_OK) return st;
    std::vector<TraceJob> jobs((size_t)nviews);
    int64_t nslots = 0;
    for (int i = 0; i < nviews; ++i) {
        st = make_job(&views[i], buf, nslots, 0, &jobs[(size_t)i], "hz_membench_gather", i);
        if (st != HZ_OK) {
            ctx_free(c, buf, fbytes);
            return st;
        }
        nslots += view_slots(views[i].width, views[i].height);
    }
    if (nslots > INT32_MAX) {
        ctx_free(c, buf, fbytes);
        return set_error(HZ_E_INVALID, "hz_membench_gather: more than 2^31 - 1 rays");
    }
    // the tracer's ray generation builds the length-sorted hit list (no
    // outputs: its rays that miss write nothing)
    const size_t jbytes = (sizeof(TraceJob) * jobs.size() + 255) & ~(size_t)255;
    const size_t aux_bytes = 256 + jbytes + kCounterBytes + 4 * (size_t)nslots + (size_t)nslots + 4 * (size_t)nslots;
    void *aux = nullptr;
    st = ctx_alloc(c, &aux, aux_bytes);
    if (st != HZ_OK) {
        ctx_free(c, buf, fbytes);
        return st;
    }
    char *p = (char *)aux;
    unsigned long long *count = (unsigned long long *)p;
    TraceJob *djobs = (TraceJob *)(p + 256);
    uint32_t *counters = (uint32_t *)(p + 256 + jbytes);
    uint32_t *hits = (uint32_t *)((char *)counters + kCounterBytes);
    uint8_t *bins = (uint8_t *)(hits + nslots);
    uint32_t *sink = (uint32_t *)(bins + nslots);
    TraceLaunch L{};
    L.jobs = djobs;
    L.njobs = nviews;
    L.nslots = nslots;
    L.hits = hits;
    L.slot_bin = bins;
    L.counters = counters;
    L.counters_next = counters + kCounterSetWords;
    make_trace_grid(*grid, 1.0f, &L.grid);
    L.inv_len_bin = length_bin_scale(*grid);
    const int64_t n4 = (int64_t)(fbytes / 16);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    unsigned long long total = 0;
    std::vector<uint32_t> bin_tot((size_t)kCounterSetWords);
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
              hipMemcpyAsync(djobs, jobs.data(), sizeof(TraceJob) * jobs.size(), hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemsetAsync(count, 0, 16, s) == hipSuccess && launch_raygen(L, true, s, KTimer{}) == hipSuccess &&
              hipMemcpyAsync(bin_tot.data(), counters, 4 * bin_tot.size(), hipMemcpyDeviceToHost, s) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess;
    uint32_t nh = 0;
    for (int k = 0; ok && k < kRayBins; ++k) nh += bin_tot[(size_t)k * kCounterStride];
    if (ok && nh > 0) {
        const dim3 g((nh + 255) / 256), b(256);
        hipLaunchKernelGGL(k_init, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, (float4 *)buf, n4);
        for (int r = 0; r <= reps; ++r) {   // launch 0 warms the caches and counts the samples
            if (r == 1) ok = hipEventRecord(e0, s) == hipSuccess;
            unsigned long long *cnt = r == 0 ? count : count + 1;
            if (voxel_bytes == 16)
                hipLaunchKernelGGL(k_gather_hits<16>, g, b, 0, s, (const char *)buf, L, nh, step_len, sink, cnt);
            else
                hipLaunchKernelGGL(k_gather_hits<8>, g, b, 0, s, (const char *)buf, L, nh, step_len, sink, cnt);
        }
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess && hipGetLastError() == hipSuccess &&
             hipMemcpy(&total, count, 8, hipMemcpyDeviceToHost) == hipSuccess;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx_free(c, buf, fbytes);
    ctx_free(c, aux, aux_bytes);
    if (ok && nh == 0) return set_error(HZ_E_INVALID, "hz_membench_gather: no ray of the views enters the grid");
    if (!ok || ms <= 0.0f) return set_error(HZ_E_DEVICE, "hz_membench_gather: timing failed");
    if (total == 0) return set_error(HZ_E_INVALID, "hz_membench_gather: no ray of the views enters the grid");
    if (samples) *samples = (int64_t)total;
    *gather_gbps = (double)total * 8.0 * voxel_bytes * reps / (ms * 1e-3) / 1e9;
    return HZ_OK;
}
