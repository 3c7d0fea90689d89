// membench.hip -- achievable read bandwidth of the memory level a buffer of a
// given size lives in (HBM for buffers far above the 256 MB MALL, L2/MALL for
// field-sized buffers read repeatedly).  Used to put the tracer's gather rate
// next to what the memory system actually delivers.
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
