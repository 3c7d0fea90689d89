// membench.hip -- achievable read bandwidth of the memory level a buffer of a
// given size lives in (HBM for buffers far above the 256 MB MALL, L2/MALL for
// field-sized buffers read repeatedly), and of the tracer's own access pattern
// (coherent 8-corner gathers along straight rays through a field-sized grid)
// with no arithmetic around it.  Used to put the tracer's gather rate next to
// what the memory system actually delivers.
#include "haze.h"
#include "serve.h"

#include <hip/hip_runtime.h>

namespace haze {

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

// One 8 x 8 pixel tile per wave, like the tracer's ray generation: walker
// (tile, lane) starts on the z = 0 face of an rx x ry x rz grid of EB-byte
// voxels at its pixel and walks a straight line one voxel per step, its
// direction tilted with its pixel's offset from the image centre (up to 1/4
// voxel per step sideways, a 28 degree field of view).  Each step reads the 8
// corners of its cell as the tracer does (the two x-neighbours of each of the
// 4 rows in one 16 or 32 byte stretch); indices are clamped into the grid.
// The words are folded into one value per walker so no load can be dropped.
template <int EB>
__global__ __launch_bounds__(256) void k_gather(const char *__restrict__ f, int32_t rx, int32_t ry, int32_t rz,
                                                int32_t walkers, int32_t tiles_x, int32_t steps,
                                                uint32_t *__restrict__ sink)
{
    const int32_t w = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (w >= walkers) return;
    const int32_t tile = w >> 6, lane = w & 63;
    const int32_t tiles_y = (walkers + 64 * tiles_x - 1) / (64 * tiles_x);
    const float iw = 1.0f / (float)(8 * tiles_x), ih = 1.0f / (float)(8 * tiles_y);
    const float u = ((float)((tile % tiles_x) * 8 + (lane & 7)) + 0.5f) * iw;   // (0, 1)
    const float v = ((float)((tile / tiles_x) * 8 + (lane >> 3)) + 0.5f) * ih;
    float x = u * (float)(rx - 1), y = v * (float)(ry - 1), z = 0.0f;
    const float dx = 0.5f * (u - 0.5f), dy = 0.5f * (v - 0.5f);
    const float inv = __builtin_amdgcn_rsqf(1.0f + dx * dx + dy * dy);
    const float sx = dx * inv, sy = dy * inv, sz = inv;
    const uint32_t row = (uint32_t)rx, slab = (uint32_t)rx * (uint32_t)ry;
    uint32_t acc = 0u;
    for (int32_t k = 0; k < steps; ++k) {
        const uint32_t ix = (uint32_t)__builtin_amdgcn_fmed3f(floorf(x), 0.0f, (float)(rx - 2));
        const uint32_t iy = (uint32_t)__builtin_amdgcn_fmed3f(floorf(y), 0.0f, (float)(ry - 2));
        const uint32_t iz = (uint32_t)__builtin_amdgcn_fmed3f(floorf(z), 0.0f, (float)(rz - 2));
        const uint32_t b = iz * slab + iy * row + ix;
        const uint32_t c[4] = {b, b + row, b + slab, b + slab + row};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const gb_ptr p = (gb_ptr)(f + (size_t)c[j] * EB);
            const gb_u32x4 a = p[0];
            acc ^= (a.x ^ a.y) ^ (a.z ^ a.w);
            if (EB == 16) {
                const gb_u32x4 b2 = p[1];
                acc ^= (b2.x ^ b2.y) ^ (b2.z ^ b2.w);
            }
        }
        x += sx;
        y += sy;
        z += sz;
    }
    sink[w] = acc;
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

extern "C" hz_status hz_membench_gather(hz_ctx *c, const int32_t res[3], int32_t voxel_bytes, int32_t walkers,
                                        int32_t steps, int32_t reps, double *gather_gbps, void *hip_stream)
{
    if (!c || !res || !gather_gbps) return set_error(HZ_E_INVALID, "hz_membench_gather: NULL argument");
    if (voxel_bytes != 8 && voxel_bytes != 16) return set_error(HZ_E_INVALID, "hz_membench_gather: voxel_bytes not 8 or 16");
    for (int a = 0; a < 3; ++a)
        if (res[a] < 2 || res[a] > 65535) return set_error(HZ_E_INVALID, "hz_membench_gather: res outside [2, 65535]");
    const int64_t nvox = (int64_t)res[0] * res[1] * res[2];
    if (nvox >= (1ll << 31)) return set_error(HZ_E_INVALID, "hz_membench_gather: grid of 2^31 voxels or more");
    if (walkers < 1 || walkers > (1 << 26) || steps < 1 || steps > 65536 || reps < 1 || reps > 10000)
        return set_error(HZ_E_INVALID, "hz_membench_gather: walkers, steps or reps out of range");
    if (hipSetDevice(ctx_device(c)) != hipSuccess) return set_error(HZ_E_DEVICE, "hz_membench_gather: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    // a pixel image about as wide as the grid is high in voxels, 8 x 8 tiles
    const int32_t tiles = (walkers + 63) / 64;
    int32_t tiles_x = 1;
    while ((int64_t)tiles_x * tiles_x * 9 < (int64_t)tiles * 16) ++tiles_x;   // ~16:9 image
    const size_t fbytes = (size_t)nvox * (size_t)voxel_bytes;
    void *buf = nullptr, *sink = nullptr;
    hz_status st = ctx_alloc(c, &buf, fbytes);
    if (st != HZ_OK) return st;
    st = ctx_alloc(c, &sink, sizeof(uint32_t) * (size_t)walkers);
    if (st != HZ_OK) {
        ctx_free(c, buf, fbytes);
        return st;
    }
    const int64_t n4 = (int64_t)(fbytes / 16);
    const dim3 g((unsigned)((walkers + 255) / 256)), b(256);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.0f;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_init, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, (float4 *)buf, n4);
        for (int r = 0; r <= reps; ++r) {   // launch 0 warms the caches
            if (r == 1) ok = hipEventRecord(e0, s) == hipSuccess;
            if (voxel_bytes == 16)
                hipLaunchKernelGGL(k_gather<16>, g, b, 0, s, (const char *)buf, res[0], res[1], res[2], walkers,
                                   tiles_x, steps, (uint32_t *)sink);
            else
                hipLaunchKernelGGL(k_gather<8>, g, b, 0, s, (const char *)buf, res[0], res[1], res[2], walkers,
                                   tiles_x, steps, (uint32_t *)sink);
        }
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess && hipGetLastError() == hipSuccess;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx_free(c, buf, fbytes);
    ctx_free(c, sink, sizeof(uint32_t) * (size_t)walkers);
    if (!ok || ms <= 0.0f) return set_error(HZ_E_DEVICE, "hz_membench_gather: timing failed");
    *gather_gbps = (double)walkers * steps * 8.0 * voxel_bytes * reps / (ms * 1e-3) / 1e9;
    return HZ_OK;
}
