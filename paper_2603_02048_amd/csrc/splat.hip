// splat.hip -- particles -> refractive-index field on gfx950.
//
// Paper Sec. 3.3.1: density is rasterised to a regular grid by SPH kernel
// splatting at voxel centres, mapped to n = 1 + K_GD rho (Eq. 12), and its
// gradient grad n = K_GD grad rho is taken by finite differences on the grid
// (Eq. 13).  The field stores delta_n = n - 1 and grad n per voxel.
//
// Pipeline (all integer work exact, so the result is bitwise repeatable):
//   k_cell_count   particle -> cell id (cells of edge h over the grid box grown
//                  by 2h), integer histogram with atomics; one more workgroup
//                  buckets the gather's bricks by weight (order_bricks_count)
//   k_scan_onepass exclusive prefix sum of the histogram in one launch
//                  (tile sums published with tickets, lower tiles added);
//                  k_scan_* in three passes for very large cell counts
//   k_cell_scatter particle index -> its slot (cell start + arrival rank from
//                  the histogram atomics: an arbitrary order inside the cell)
//   k_cell_order   per particle, its rank by index among its cell's members
//                  (stable order); (x, y, z, m) into cell-sorted float4 records;
//                  one more workgroup lists the bricks heaviest first
//                  (order_bricks_place)
//   k_splat        one workgroup per 8x8x4 or 8x8x8 voxel brick (records the
//                  brick's candidate count for the next call's order), its cell-list
//                  rows dealt to four waves: every lane owns a column of
//                  voxels; each candidate particle is culled to the planes
//                  it reaches (64 candidates at a time, one per lane), then
//                  the wave's lanes walk the remaining candidates together
//                  (wave-uniform scalar loads), summing m_j W in a fixed order
//   k_splat_scatter  alternative: voxel tiles with 64-bit fixed-point LDS
//                  accumulators, particles walking their footprints (more
//                  accurate, bitwise repeatable, but about 2x slower than the
//                  gather on gfx950: 64-bit LDS atomics and divergent loops)
//   k_grad_pack    central differences (one-sided on faces) and packing of
//                  (delta_n, grad) into F32 / F16 / BF16 voxels
#include "haze_device.h"

#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

namespace haze {

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ int cell_coord(float x, float clo, float inv_cell, int nc)
{
    float c = floorf((x - clo) * inv_cell);
    if (!(c >= 0.0f) || c >= (float)nc) return -1;
    return (int)c;
}

// Dispatch order of the gather's bricks, heaviest first, in two phases that
// each run in one extra 256-thread workgroup of a cell-list kernel, beside
// that kernel's own work.  bwork[b] is the number of candidate particles
// brick b had in the previous gather over the same bricks and bwork[2 nb]
// their largest.  The bricks are bucketed by that count into kOrderBuckets
// buckets of equal width below the largest; border[] (= bwork + nb) lists them
// bucket by bucket, heaviest bucket first (in any order inside a bucket).
// Every brick sums in its own fixed order, so the field does not depend on
// the order; handing the heavy bricks out first shortens the launch's tail.
// Both phases bucket the same counts with the same scale, so the placement is
// a permutation of [0, nb).
constexpr int kOrderBuckets = 64;   // one per lane of the scan below
constexpr int kOrderUnroll = 16;
struct BrickOrder {
    uint32_t *work;    // [nb] counts, [nb] order, largest, scale (float bits), kOrderBuckets bucket sizes
    int32_t nb;
    int32_t order;     // 0: only clear the largest count for the gather that follows
    __device__ uint32_t *border() const { return work + nb; }
    __device__ uint32_t *bmax() const { return work + 2 * (size_t)nb; }
    __device__ uint32_t *scale() const { return work + 2 * (size_t)nb + 1; }
    __device__ uint32_t *hist() const { return work + 2 * (size_t)nb + 2; }
};

__device__ __forceinline__ uint32_t order_bucket(uint32_t w, float scale)
{
    return (uint32_t)(kOrderBuckets - 1) - min((uint32_t)(kOrderBuckets - 1), (uint32_t)((float)w * scale));
}

// Each thread takes a contiguous run of bricks, kOrderUnroll counts in flight
// per round: the lanes of one LDS atomic then hold bricks far apart, whose
// buckets mostly differ (neighbouring bricks, which mostly share a bucket,
// would serialise the atomic on one address).
template <typename F>
__device__ __forceinline__ void for_my_bricks(const uint32_t *__restrict__ work, int32_t nb, F &&f)
{
    const int32_t per = (nb + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x;
    const int32_t mine0 = (int32_t)threadIdx.x * per, mine1 = min(nb, mine0 + per);
    for (int32_t b0 = mine0; b0 < mine1; b0 += kOrderUnroll) {
        uint32_t w[kOrderUnroll];
#pragma unroll
        for (int u = 0; u < kOrderUnroll; ++u) w[u] = b0 + u < mine1 ? work[b0 + u] : 0u;
#pragma unroll
        for (int u = 0; u < kOrderUnroll; ++u)
            if (b0 + u < mine1) f(b0 + u, w[u]);
    }
}

// Phase 1 (in the cell-count launch): the scale and the bucket sizes; clears
// the largest count.
__device__ void order_bricks_count(const BrickOrder &O)
{
    __shared__ uint32_t hist[kOrderBuckets];
    if (!O.order) {
        if (threadIdx.x == 0) *O.bmax() = 0u;
        return;
    }
    // buckets per count (a float scale: an integer division per brick would
    // cost more than the whole ordering)
    const float scale = (float)kOrderBuckets / ((float)*O.bmax() + 1.0f);
    if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = 0u;
    __syncthreads();   // every thread has read the largest count
    if (threadIdx.x == 0) {
        *O.bmax() = 0u;
        *O.scale() = __float_as_uint(scale);
    }
    for_my_bricks(O.work, O.nb, [&](int32_t, uint32_t w) { atomicAdd(&hist[order_bucket(w, scale)], 1u); });
    __syncthreads();
    if (threadIdx.x < kOrderBuckets) O.hist()[threadIdx.x] = hist[threadIdx.x];
}

// Phase 2 (in the cell-order launch): bucket starts, then every brick to its
// place.
__device__ void order_bricks_place(const BrickOrder &O)
{
    __shared__ uint32_t cur[kOrderBuckets];
    const float scale = __uint_as_float(*O.scale());
    if (threadIdx.x < 64) {   // exclusive scan of the 64 bucket sizes, one per lane
        const uint32_t h = O.hist()[threadIdx.x];
        uint32_t incl = h;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
            if ((int)threadIdx.x >= off) incl += o;
        }
        cur[threadIdx.x] = incl - h;
    }
    __syncthreads();
    uint32_t *border = O.border();
    for_my_bricks(O.work, O.nb, [&](int32_t b, uint32_t w) {
        border[atomicAdd(&cur[order_bucket(w, scale)], 1u)] = (uint32_t)b;
    });
}

// Particle -> cell id (0xffffffff when outside the grown box) + histogram;
// the atomic's old value is the particle's arrival rank in its cell (an
// arbitrary order that k_cell_order replaces by index order).  With MMAX,
// also records max |m| of the binned particles (as float bits;
// non-negative floats order like unsigned integers) in *mmax for the
// fixed-point splat: reduced over the workgroup first, so one atomic per
// workgroup reaches the single address.
template <bool MMAX>
__global__ __launch_bounds__(256) void k_cell_count(const float *__restrict__ x, const float *__restrict__ y,
                                                    const float *__restrict__ z, const float *__restrict__ m,
                                                    int32_t n, CellGrid cg, uint32_t *__restrict__ cid,
                                                    uint32_t *__restrict__ lrank, uint32_t *__restrict__ count,
                                                    uint32_t *__restrict__ mmax, uint32_t *__restrict__ fail,
                                                    BrickOrder O)
{
    // With brick counts, workgroup 0 runs the first phase of the gather's
    // brick order beside the binning of the others (one workgroup later).
    uint32_t block = blockIdx.x;
    if (O.work) {
        if (block == 0u) {
            order_bricks_count(O);
            return;
        }
        --block;
    }
    // 64-bit: the last workgroup reaches past 2^31 - 1 when n is near it
    const int64_t i = (int64_t)block * blockDim.x + threadIdx.x;
    // the call's scan-failure word starts clear (the scan runs after this launch)
    if (i == 0) *fail = 0u;
    uint32_t mbits = 0u;
    if (i < n) {
        const int cx = cell_coord(x[i], cg.clo[0], cg.inv_cell, cg.nc[0]);
        const int cy = cell_coord(y[i], cg.clo[1], cg.inv_cell, cg.nc[1]);
        const int cz = cell_coord(z[i], cg.clo[2], cg.inv_cell, cg.nc[2]);
        // a particle outside the grown box, or with a mass that is not
        // finite, is in no cell and adds nothing
        const float am = fabsf(m[i]);
        uint32_t id = 0xffffffffu;
        if (cx >= 0 && cy >= 0 && cz >= 0 && isfinite(am)) {
            id = (uint32_t)((cz * cg.nc[1] + cy) * cg.nc[0] + cx);
            lrank[i] = atomicAdd(&count[id], 1u);
            if (MMAX && am > 0.0f) mbits = __float_as_uint(am);
        }
        cid[i] = id;
    }
    if (MMAX) {
        __shared__ uint32_t wmax[4];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mbits = max(mbits, (uint32_t)__shfl_xor((int)mbits, off));
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mbits;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t b = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
            if (b) atomicMax(mmax, b);
        }
    }
}

// Exclusive scan of count[0..n) into start[0..n] (start[n] = total) over
// tiles of SCAN_TILE cells, clearing the counts as it reads them (so the
// histogram starts the next call at zero).  Up to SCAN_ONEPASS_TILES tiles
// it is one launch (k_scan_onepass); beyond, three passes: tile sums, scan of
// the tile sums (one workgroup), then each tile rescanned with its offset.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_PER_THREAD;
constexpr int SCAN_ONEPASS_TILES = 1024;
constexpr size_t SCAN_TAG_OFFSET = 256;   // bytes: ticket counter and failure word, then tile tags or sums

// Inclusive scan of one value per thread across a 256-thread workgroup.
__device__ __forceinline__ uint32_t block_scan_incl(uint32_t v, uint32_t *wave_tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    if (lane == 63) wave_tot[wave] = v;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < wave; ++w) add += wave_tot[w];
    __syncthreads();
    return v + add;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const uint32_t *__restrict__ count, int32_t n,
                                                             uint32_t *__restrict__ tile_sum)
{
    __shared__ uint32_t wt[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k)
        if (base + k < n) s += count[base + k];
    const uint32_t incl = block_scan_incl(s, wt);
    if (threadIdx.x == SCAN_THREADS - 1) tile_sum[blockIdx.x] = incl;
}

// Exclusive scan of the tile sums in place (one workgroup); writes the grand
// total to *total.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile_sums(uint32_t *__restrict__ tile_sum, int32_t ntiles,
                                                                 uint32_t *__restrict__ total)
{
    __shared__ uint32_t wt[4];
    __shared__ uint32_t chunk_total;
    uint32_t carry = 0;
    for (int32_t b = 0; b < ntiles; b += SCAN_THREADS) {
        const int32_t i = b + (int32_t)threadIdx.x;
        const uint32_t v = i < ntiles ? tile_sum[i] : 0u;
        const uint32_t incl = block_scan_incl(v, wt);
        if (i < ntiles) tile_sum[i] = carry + incl - v;
        if (threadIdx.x == SCAN_THREADS - 1) chunk_total = incl;
        __syncthreads();
        carry += chunk_total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(uint32_t *__restrict__ count, int32_t n,
                                                             const uint32_t *__restrict__ tile_off,
                                                             uint32_t *__restrict__ start)
{
    __shared__ uint32_t wt[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        v[k] = base + k < n ? count[base + k] : 0u;
        s += v[k];
    }
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k)
        if (base + k < n) count[base + k] = 0u;
    uint32_t run = tile_off[blockIdx.x] + block_scan_incl(s, wt) - s;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        if (base + k < n) start[base + k] = run;
        run += v[k];
    }
}

// One-launch scan.  Workgroups take tiles in the order they start, from a
// running ticket counter (tile = ticket - base, where base is the counter's
// value at launch), publish their tile's sum tagged with their ticket, and add
// the sums of all lower tiles.  Each lower tile belongs to a workgroup that
// took its ticket earlier and is therefore already running, and it waits only
// on tiles lower still, so every wait ends.  The spin is still bounded
// (spin_limit sleeps per lower tile): a wait that gives up adds nothing,
// sets the call's failure word `fail` (the later kernels of the call then
// skip their work and leave NaN in the field) and stores `serial` into the
// host-visible word `fail_host`, where the library finds it.  tag_bias is 0
// except in the fault test, where it makes every wait give up.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_onepass(uint32_t *__restrict__ count, int32_t n,
                                                               int32_t ntiles, uint32_t *__restrict__ ticket_ctr,
                                                               uint64_t *__restrict__ tags, uint32_t base,
                                                               uint32_t *__restrict__ start, uint32_t spin_limit,
                                                               uint32_t tag_bias, uint32_t *__restrict__ fail,
                                                               uint32_t *fail_host, uint32_t serial)
{
    __shared__ uint32_t wt[4];
    __shared__ uint32_t sh_ticket;
    __shared__ uint32_t sh_lower[4];
    if (threadIdx.x == 0) sh_ticket = atomicAdd(ticket_ctr, 1u);
    __syncthreads();
    const uint32_t ticket = sh_ticket;
    const int32_t tile = (int32_t)(ticket - base);
    const int64_t b0 = (int64_t)tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        v[k] = b0 + k < n ? count[b0 + k] : 0u;
        s += v[k];
    }
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k)
        if (b0 + k < n) count[b0 + k] = 0u;
    const uint32_t incl = block_scan_incl(s, wt);
    // tag = ticket + 1: cleared memory (tag 0) never passes for a sum.  The
    // tag and the sum travel in one 64-bit word, so relaxed device-scope
    // atomics suffice (no fences, which would write back and invalidate L2).
    if (threadIdx.x == SCAN_THREADS - 1)
        __hip_atomic_store(&tags[tile], ((uint64_t)(ticket + 1u) << 32) | incl, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    uint32_t lower = 0;
    bool gave_up = false;
    for (int32_t t = (int32_t)threadIdx.x; t < tile; t += SCAN_THREADS) {
        const uint32_t want = base + (uint32_t)t + 1u + tag_bias;
        bool got = false;
        for (uint32_t spin = 0; spin < spin_limit; ++spin) {
            const uint64_t w = __hip_atomic_load(&tags[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(w >> 32) == want) {
                lower += (uint32_t)w;
                got = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        gave_up = gave_up || !got;
    }
    if (gave_up) {
        __hip_atomic_store(fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fail_host) __hip_atomic_store(fail_host, serial, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lower += (uint32_t)__shfl_xor((int)lower, off);
    if ((threadIdx.x & 63) == 0) sh_lower[threadIdx.x >> 6] = lower;
    __syncthreads();
    const uint32_t offset = sh_lower[0] + sh_lower[1] + sh_lower[2] + sh_lower[3];
    uint32_t run = offset + incl - s;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        if (b0 + k < n) start[b0 + k] = run;
        run += v[k];
    }
    if (tile == ntiles - 1 && threadIdx.x == SCAN_THREADS - 1) start[n] = run;
}

// Every binned particle takes the slot of its cell given by its arrival rank
// (nothing when the scan failed: the starts are then wrong).
__global__ __launch_bounds__(256) void k_cell_scatter(const uint32_t *__restrict__ cid,
                                                      const uint32_t *__restrict__ lrank, int32_t n,
                                                      const uint32_t *__restrict__ start,
                                                      uint32_t *__restrict__ slots, const uint32_t *__restrict__ fail)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || *fail) return;
    uint32_t c = cid[i];
    if (c == 0xffffffffu) return;
    slots[start[c] + lrank[i]] = (uint32_t)i;
}

// One thread per particle: its rank inside its cell is the number of cell
// members with a smaller index, which puts each cell in index order whatever
// order the arrival ranks gave; the particle's (x, y, z, m) record goes there.
__global__ __launch_bounds__(256) void k_cell_order(const uint32_t *__restrict__ cid,
                                                    const uint32_t *__restrict__ start,
                                                    const uint32_t *__restrict__ slots, int32_t n,
                                                    const float *__restrict__ x, const float *__restrict__ y,
                                                    const float *__restrict__ z, const float *__restrict__ m,
                                                    float4 *__restrict__ sorted, const uint32_t *__restrict__ fail,
                                                    BrickOrder O)
{
    // When ordering the gather's bricks, workgroup 0 places them (the second
    // phase) beside the ordering of the particles (one workgroup later).
    uint32_t block = blockIdx.x;
    if (O.order) {
        if (block == 0u) {
            order_bricks_place(O);
            return;
        }
        --block;
    }
    const int64_t i = (int64_t)block * blockDim.x + threadIdx.x;
    if (i >= n || *fail) return;
    const uint32_t c = cid[i];
    if (c == 0xffffffffu) return;
    const uint32_t b = start[c], e = start[c + 1];
    const float4 rec = make_float4(x[i], y[i], z[i], m[i]);
    // Eight slots per round with all eight loads in flight before any compare
    // (the loop is latency-bound); indices are clamped into the cell, which
    // holds at least particle i, and a clamped repeat is not counted.
    uint32_t rank = 0;
    for (uint32_t t = b; t < e; t += 8) {
        uint32_t sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sv[u] = slots[min(t + (uint32_t)u, e - 1u)];
#pragma unroll
        for (int u = 0; u < 8; ++u) rank += (t + (uint32_t)u < e && sv[u] < (uint32_t)i) ? 1u : 0u;
    }
    sorted[b + rank] = rec;
}

// M4 spline (Eq. 12) through two clamped variables.  With q = r / h,
// t = max(1 - q/2, 0) and s = max(1 - q, 0), both in [0, 1]:
//   4 W(q) / sigma = (2 - q)^3 - 4 (1 - q)^3 = 8 t^3 - 4 s^3   (q < 1)
//                  = (2 - q)^3               = 8 t^3           (1 <= q < 2)
//                  = 0                                        (q >= 2),
// so sum_j m_j W = (sigma / 4) (8 A - 4 B) with A = sum m t^3 over the
// support sphere (q < 2) and B = sum m s^3 over the inner sphere (q < 1).
// A lane outside a sphere gets t = 0 (or s = 0) from the clamp and adds an
// exact zero, so a plane needs no per-lane test: a wave-uniform cull decides
// which planes a candidate visits.
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

// Per-lane state of the gather: the column's voxel centres and the two sums
// per voxel.
template <int BZ>
struct Column {
    float cx, cy;
    float cz[BZ];
    float a[BZ], b[BZ];
};

// Candidate q at plane V, dxy = the lane's squared x-y distance to q and
// dz[V] = z_V - z_q (wave-uniform); the inner term too when the inner sphere
// reaches the plane (wave-uniform).
template <int V, int BZ>
__device__ __forceinline__ void plane_terms(Column<BZ> &c, float dxy, const float *dz, const float4 &q, bool inner,
                                            float nhalf_inv_h, float ninv_h)
{
    const float r = __builtin_amdgcn_sqrtf(fmaf(dz[V], dz[V], dxy));
    const float t = clamp01(fmaf(r, nhalf_inv_h, 1.0f));
    c.a[V] = fmaf(q.w, t * t * t, c.a[V]);
    if (inner) {
        const float s = clamp01(fmaf(r, ninv_h, 1.0f));
        c.b[V] = fmaf(q.w, s * s * s, c.b[V]);
    }
}

// The planes of the wave-uniform masks, in order (a uniform branch each).
template <int V, int BZ>
__device__ __forceinline__ void planes(uint32_t om, uint32_t im, Column<BZ> &c, float dxy, const float *dz,
                                       const float4 &q, float nhalf_inv_h, float ninv_h)
{
    if constexpr (V < BZ) {
        if (om & (1u << V)) plane_terms<V, BZ>(c, dxy, dz, q, (im & (1u << V)) != 0u, nhalf_inv_h, ninv_h);
        planes<V + 1, BZ>(om, im, c, dxy, dz, q, nhalf_inv_h, ninv_h);
    }
}

// One candidate: the cull's wave-uniform word holds the planes its support
// sphere reaches (bits 0-7) and those its inner sphere reaches (bits 8-15, a
// subset).
template <int BZ>
__device__ __forceinline__ void gather_candidate(Column<BZ> &c, const float4 &q, const float *dz, uint32_t pk,
                                                 float nhalf_inv_h, float ninv_h)
{
    const float dx = c.cx - q.x, dy = c.cy - q.y;
    const float dxy = fmaf(dx, dx, dy * dy);
    planes<0, BZ>(pk & 0xffu, (pk >> 8) & 0xffu, c, dxy, dz, q, nhalf_inv_h, ninv_h);
}

// One workgroup per brick of 8 x 8 x BZ voxels (BZ = 4 or 8); in each of its
// four waves, lane (lane & 7, lane >> 3) owns the column of BZ voxels along z.
// The brick's cell-list rows near it (each row's x-range cut to the support
// circle) are dealt round-robin to its four waves.  A wave culls a row's
// candidates 64 at a time, one per lane: from the candidate's x-y distance to
// the brick's box of columns it finds the planes its support sphere reaches
// for some column, and those its inner sphere reaches (both as exact as
// testing every lane: a plane is culled only when no lane can be in reach).
// The candidates left are then taken in index order, each as wave-uniform
// scalar loads; its x-y distance is computed once per lane and shared by the
// column; the planes' z offsets, the same for every lane, come from the
// candidate's cull lane through LDS, and each plane in range costs six
// instructions per lane, with no per-lane test or branch.  The four partial
// sums are added in wave order
// through LDS, and each wave adds its terms in row order, then particle index
// order, so the field is bitwise repeatable.  Splitting a brick four ways
// gives four times as many work units as wave slots, so the dispatcher
// balances bricks of unequal cost.  Workgroup i takes brick i: the hardware
// deals workgroups round-robin over the 8 XCDs, so each XCD's share is spread
// over the whole grid (faster than giving each XCD a contiguous run of bricks
// for its own L2: this kernel is bound by instruction issue, not by traffic).
constexpr int SPLAT_WAVES = 4;

template <int BZ>
__global__ __launch_bounds__(64 * SPLAT_WAVES) void k_splat(SplatParams P, const uint32_t *__restrict__ start,
                                                            const float4 *__restrict__ parts, int32_t nbricks,
                                                            float *__restrict__ dn,
                                                            const uint32_t *__restrict__ fail,
                                                            uint32_t *__restrict__ bwork,
                                                            const uint32_t *__restrict__ border)
{
    __shared__ float partial[SPLAT_WAVES - 1][BZ][64];
    __shared__ uint32_t wcand[SPLAT_WAVES];
    // per wave and culled candidate: z_v - z_j for the brick's planes (the
    // same for every lane), read back as a broadcast instead of one
    // subtraction per lane and plane
    __shared__ float4 dzs[SPLAT_WAVES][64][BZ / 4];
    if ((int32_t)blockIdx.x >= nbricks) return;   // uniform over the workgroup
    // the brick of this dispatch slot (heaviest first when an order is given)
    int32_t brick = (int32_t)blockIdx.x;
    if (border) {
        const uint32_t o = __builtin_amdgcn_readfirstlane(border[blockIdx.x]);
        if (o < (uint32_t)nbricks) brick = (int32_t)o;
    }
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t bx = brick % P.nbx;
    const int32_t by = (brick / P.nbx) % P.nby;
    const int32_t bz = brick / (P.nbx * P.nby);
    const int32_t vx = bx * SPLAT_BX + (lane & 7), vy = by * SPLAT_BY + (lane >> 3), vz0 = bz * BZ;
    Column<BZ> col;
    col.cx = P.lo[0] + ((float)vx + 0.5f) * P.sp[0];
    col.cy = P.lo[1] + ((float)vy + 0.5f) * P.sp[1];
#pragma unroll
    for (int v = 0; v < BZ; ++v) {
        col.cz[v] = P.lo[2] + ((float)(vz0 + v) + 0.5f) * P.sp[2];
        col.a[v] = 0.0f;
        col.b[v] = 0.0f;
    }

    // brick AABB of voxel centres (wave-uniform; the x-y faces are the centres
    // of the first and last columns, bit for bit as the lanes compute them)
    float blo[3], bhi[3];
    {
        const int32_t b0[3] = {bx * SPLAT_BX, by * SPLAT_BY, vz0};
        const int32_t bd[3] = {SPLAT_BX, SPLAT_BY, BZ};
        for (int a = 0; a < 3; ++a) {
            const int32_t i1 = min(b0[a] + bd[a] - 1, P.res[a] - 1);
            blo[a] = P.lo[a] + ((float)b0[a] + 0.5f) * P.sp[a];
            bhi[a] = P.lo[a] + ((float)i1 + 0.5f) * P.sp[a];
        }
    }
    const CellGrid &cg = P.cg;
    const float R = 2.0f * P.h;
    const float nhalf_inv_h = -0.5f * P.inv_h, ninv_h = -P.inv_h;
    // cull bounds: squared radii grown by 0.1% and plane ranges by 1% of a
    // plane, so that rounding never drops a plane some lane reaches (a plane
    // visited needlessly adds exact zeros)
    const float ro2 = 1.001f * P.support2, ri2 = 1.001f * P.h * P.h;
    const float inv_spz = 1.0f / P.sp[2];
    // conservative cell ranges (one cell of slack absorbs rounding)
    const int cz0 = max(0, (int)floorf((blo[2] - R - cg.clo[2]) * cg.inv_cell) - 1);
    const int cz1 = min(cg.nc[2] - 1, (int)floorf((bhi[2] + R - cg.clo[2]) * cg.inv_cell) + 1);
    const int cy0 = max(0, (int)floorf((blo[1] - R - cg.clo[1]) * cg.inv_cell) - 1);
    const int cy1 = min(cg.nc[1] - 1, (int)floorf((bhi[1] + R - cg.clo[1]) * cg.inv_cell) + 1);
    const int ny = cy1 - cy0 + 1;

    // rows (kz, ky) in order, every SPLAT_WAVES-th from the wave's index (no rows
    // if the y range is empty, so the row stepping below always advances); no
    // rows, and NaN voxels, when the cell-list scan failed.  Each pass of the
    // loop culls the next 64 candidates of the current row and sums those
    // left, then moves to the next row when the row is done (a row out of
    // reach is culled as empty): one exit, at the bottom, so the sums keep
    // their registers through the loop.
    const bool bad = *fail != 0u;
    int kz = ny >= 1 && !bad ? cz0 : cz1 + 1, ky = cy0 + wave;
    uint32_t c0 = 0u, s1 = 0u;   // the next candidate to cull; the row's end
    uint32_t cand = 0u;          // candidates of this wave's rows (the next call's brick order)
    // moves to the next row; false when there is none
    const auto next_row = [&]() -> bool {
        // (wrapping past the y range without a loop)
        if (ky > cy1 && ny >= 1) {
            const int k = (ky - cy1 + ny - 1) / ny;
            ky -= k * ny;
            kz += k;
        }
        if (kz > cz1) return false;
        const int kyr = ky;
        ky += SPLAT_WAVES;
        const float zl = cg.clo[2] + (float)kz * cg.cell;
        const float gz = fmaxf(0.0f, fmaxf(zl - bhi[2], blo[2] - (zl + cg.cell)));
        const float yl = cg.clo[1] + (float)kyr * cg.cell;
        const float gy = fmaxf(0.0f, fmaxf(yl - bhi[1], blo[1] - (yl + cg.cell)));
        // 1.0001 R^2 keeps the cull conservative under rounding (and the
        // 1-ulp hardware square root)
        const float rem = 1.0001f * P.support2 - gz * gz - gy * gy;
        const float dxm = __builtin_amdgcn_sqrtf(fmaxf(rem, 0.0f));
        const int kx0 = max(0, (int)floorf((blo[0] - dxm - cg.clo[0]) * cg.inv_cell));
        const int kx1 = min(cg.nc[0] - 1, (int)floorf((bhi[0] + dxm - cg.clo[0]) * cg.inv_cell));
        c0 = s1 = 0u;
        if (rem > 0.0f && kx0 <= kx1) {
            const int row = (kz * cg.nc[1] + kyr) * cg.nc[0];
            c0 = __builtin_amdgcn_readfirstlane(start[row + kx0]);
            s1 = __builtin_amdgcn_readfirstlane(start[row + kx1 + 1]);
            cand += s1 - c0;
        }
        return true;
    };
    for (bool more = next_row(); more;) {
        // the cull: lane l takes candidate c0 + l
        const uint32_t idx = c0 + (uint32_t)lane;
        bool reach = false;
        uint32_t pk = 0u;
        if (idx < s1) {
            const float4 p = parts[idx];
            const float ex = fmaxf(fmaxf(blo[0] - p.x, p.x - bhi[0]), 0.0f);
            const float ey = fmaxf(fmaxf(blo[1] - p.y, p.y - bhi[1]), 0.0f);
            const float d2 = fmaf(ex, ex, ey * ey);
            const float zr = (p.z - blo[2]) * inv_spz;   // in planes from plane 0
            const float ho = __builtin_amdgcn_sqrtf(fmaxf(ro2 - d2, 0.0f)) * inv_spz + 0.01f;
            const float hi = __builtin_amdgcn_sqrtf(fmaxf(ri2 - d2, 0.0f)) * inv_spz + 0.01f;
            // planes v0..v1 as a bit mask (empty when v0 > v1)
            const auto span = [](float z0, float z1) -> uint32_t {
                const int v0 = max(0, (int)ceilf(z0)), v1 = min(BZ - 1, (int)floorf(z1));
                return v0 > v1 ? 0u : ((2u << v1) - (1u << v0));
            };
            const uint32_t om = d2 < ro2 ? span(zr - ho, zr + ho) : 0u;
            const uint32_t im = d2 < ri2 ? span(zr - hi, zr + hi) : 0u;
            reach = om != 0u;
            pk = om | (im << 8);
#pragma unroll
            for (int v4 = 0; v4 < BZ / 4; ++v4)
                dzs[wave][lane][v4] = make_float4(col.cz[4 * v4] - p.z, col.cz[4 * v4 + 1] - p.z,
                                                  col.cz[4 * v4 + 2] - p.z, col.cz[4 * v4 + 3] - p.z);
        }
        // the candidates left, in index order
        for (uint64_t mask = __builtin_amdgcn_ballot_w64(reach); mask;) {
            const int i = __builtin_ctzll(mask);
            mask &= ~(1ull << i);
            float dz[BZ];
#pragma unroll
            for (int v4 = 0; v4 < BZ / 4; ++v4) {
                const float4 d = dzs[wave][i][v4];
                dz[4 * v4] = d.x;
                dz[4 * v4 + 1] = d.y;
                dz[4 * v4 + 2] = d.z;
                dz[4 * v4 + 3] = d.w;
            }
            const float4 q = parts[c0 + (uint32_t)i];
            // the record and the offsets in registers here, ahead of the
            // planes' branches
            asm volatile("" ::"s"(q.x), "s"(q.y), "s"(q.z), "s"(q.w));
#pragma unroll
            for (int v = 0; v < BZ; v += 4) asm volatile("" ::"v"(dz[v]), "v"(dz[v + 1]), "v"(dz[v + 2]), "v"(dz[v + 3]));
            gather_candidate<BZ>(col, q, dz, __builtin_amdgcn_readlane(pk, i), nhalf_inv_h, ninv_h);
        }
        c0 += 64u;
        if (c0 >= s1) more = next_row();
    }
    // this wave's share of sum m W / sigma = 2 A - B (the scale is k_gd sigma)
    float part[BZ];
#pragma unroll
    for (int v = 0; v < BZ; ++v) part[v] = fmaf(2.0f, col.a[v], -col.b[v]);
    if (wave > 0) {
#pragma unroll
        for (int v = 0; v < BZ; ++v) partial[wave - 1][v][lane] = part[v];
    }
    if (lane == 0) wcand[wave] = cand;
    __syncthreads();
    if (bwork && threadIdx.x == 0) {
        uint32_t total = 0u;
#pragma unroll
        for (int w = 0; w < SPLAT_WAVES; ++w) total += wcand[w];
        bwork[brick] = total;
        atomicMax(bwork + 2 * (size_t)nbricks, total);
    }
    if (wave == 0 && vx < P.res[0] && vy < P.res[1]) {
        const float sc = bad ? __builtin_nanf("") : P.scale;
#pragma unroll
        for (int v = 0; v < BZ; ++v) {
            float sum = part[v];
#pragma unroll
            for (int w = 0; w < SPLAT_WAVES - 1; ++w) sum += partial[w][v][lane];
            if (vz0 + v < P.res[2]) dn[((int64_t)vy * P.res[0] + vx) * P.res[2] + vz0 + v] = sum * sc;
        }
    }
}

// ---------------------------------------------------------------------------
// scatter splat: one workgroup per voxel tile, particles walk their footprints
// ---------------------------------------------------------------------------
// A workgroup owns a TX x TY x TZ tile of voxels with one 64-bit fixed-point
// accumulator each in LDS.  The candidate particles are the cell-list rows
// overlapping the tile grown by 2h, flattened through a prefix sum in LDS;
// each thread takes candidates in turn and walks the part of the particle's
// support sphere inside the tile row by row, with the exact x-range of each
// row, so only in-support (voxel, particle) pairs are evaluated.  Each term
// m_j W is quantised as round-toward-zero(m_j W / max|m| * 2^31), an exact
// integer; integer addition is associative, so the sum (and the field) is the
// same bits whatever order the threads add in.
constexpr int SC_TX = 16, SC_TY = 16, SC_TZ = 8;
constexpr int SC_THREADS = 256;
constexpr int SC_MAXROWS = 512;

__global__ __launch_bounds__(SC_THREADS) void k_splat_scatter(SplatParams P, const uint32_t *__restrict__ start,
                                                              const float4 *__restrict__ parts,
                                                              const uint32_t *__restrict__ mmax_bits,
                                                              int32_t ntx, int32_t nty, int32_t ntiles,
                                                              int32_t per_xcd, float *__restrict__ dn,
                                                              const uint32_t *__restrict__ fail)
{
    __shared__ unsigned long long acc[SC_TX * SC_TY * SC_TZ];
    __shared__ uint32_t row_first[SC_MAXROWS];
    __shared__ uint32_t row_pref[SC_MAXROWS + 1];
    __shared__ uint32_t wt[4];

    const int32_t tile = (int32_t)(blockIdx.x & 7u) * per_xcd + (int32_t)(blockIdx.x >> 3);
    if (tile >= ntiles) return;
    const int32_t tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int32_t o[3] = {tx * SC_TX, ty * SC_TY, tz * SC_TZ};
    const int32_t tdim[3] = {SC_TX, SC_TY, SC_TZ};
    int32_t nt[3];
    float blo[3], bhi[3];
    for (int a = 0; a < 3; ++a) {
        nt[a] = min(tdim[a], P.res[a] - o[a]);
        blo[a] = P.lo[a] + ((float)o[a] + 0.5f) * P.sp[a];
        bhi[a] = P.lo[a] + ((float)(o[a] + nt[a] - 1) + 0.5f) * P.sp[a];
    }
    for (int v = threadIdx.x; v < SC_TX * SC_TY * SC_TZ; v += SC_THREADS) acc[v] = 0ull;
    if (*fail) {   // the cell-list scan failed: NaN voxels, no particle reads
        for (int v = threadIdx.x; v < SC_TX * SC_TY * SC_TZ; v += SC_THREADS) {
            const int li = v % SC_TX, lj = (v / SC_TX) % SC_TY, lk = v / (SC_TX * SC_TY);
            if (li < nt[0] && lj < nt[1] && lk < nt[2])
                dn[((int64_t)(o[1] + lj) * P.res[0] + (o[0] + li)) * P.res[2] + (o[2] + lk)] = __builtin_nanf("");
        }
        return;
    }

    // cell rows (ky, kz) and x-range of cells overlapping the grown tile (one
    // cell of slack absorbs rounding)
    const CellGrid &cg = P.cg;
    const float R = 2.0f * P.h;
    int c0[3], c1[3];
    for (int a = 0; a < 3; ++a) {
        c0[a] = max(0, (int)floorf((blo[a] - R - cg.clo[a]) * cg.inv_cell) - 1);
        c1[a] = min(cg.nc[a] - 1, (int)floorf((bhi[a] + R - cg.clo[a]) * cg.inv_cell) + 1);
    }
    const int nry = c1[1] - c0[1] + 1, nrz = c1[2] - c0[2] + 1;
    const int nrows = max(0, nry) * max(0, nrz);   // <= SC_MAXROWS (checked on the host)
    uint32_t cnt[2] = {0u, 0u};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int r = threadIdx.x * 2 + k;
        if (r < nrows && c0[0] <= c1[0]) {
            const int ky = c0[1] + r % nry, kz = c0[2] + r / nry;
            const int row = (kz * cg.nc[1] + ky) * cg.nc[0];
            const uint32_t s0 = start[row + c0[0]], s1 = start[row + c1[0] + 1];
            row_first[r] = s0;
            cnt[k] = s1 - s0;
        }
    }
    const uint32_t tsum = cnt[0] + cnt[1];
    const uint32_t incl = block_scan_incl(tsum, wt);
    {
        const int r = threadIdx.x * 2;
        const uint32_t ex = incl - tsum;
        if (r < nrows) row_pref[r] = ex;
        if (r + 1 < nrows) row_pref[r + 1] = ex + cnt[0];
        if (threadIdx.x == SC_THREADS - 1) row_pref[nrows] = incl;
    }
    __syncthreads();
    const uint32_t total = row_pref[nrows];

    const float mref = __uint_as_float(*mmax_bits);
    const float mscale = mref > 0.0f ? 2147483648.0f / mref : 0.0f;
    const float R2 = P.support2;
    for (uint32_t cidx = threadIdx.x; cidx < total; cidx += SC_THREADS) {
        int lo_r = 0, hi_r = nrows - 1;   // last row whose prefix <= cidx
        while (lo_r < hi_r) {
            const int mid = (lo_r + hi_r + 1) >> 1;
            if (row_pref[mid] <= cidx)
                lo_r = mid;
            else
                hi_r = mid - 1;
        }
        const float4 q = parts[row_first[lo_r] + (cidx - row_pref[lo_r])];
        const float pc[3] = {q.x, q.y, q.z};
        int32_t f0[3], f1[3];
        bool empty = false;
        for (int a = 0; a < 3; ++a) {
            // voxel centres within [p - R, p + R] on this axis, clipped to the tile
            f0[a] = max(o[a], (int32_t)ceilf((pc[a] - R - P.lo[a]) / P.sp[a] - 0.5f));
            f1[a] = min(o[a] + nt[a] - 1, (int32_t)floorf((pc[a] + R - P.lo[a]) / P.sp[a] - 0.5f));
            empty |= f0[a] > f1[a];
        }
        if (empty) continue;
        const float ms = q.w * mscale;
        for (int32_t kk = f0[2]; kk <= f1[2]; ++kk) {
            const float dz = P.lo[2] + ((float)kk + 0.5f) * P.sp[2] - q.z;
            for (int32_t jj = f0[1]; jj <= f1[1]; ++jj) {
                const float dy = P.lo[1] + ((float)jj + 0.5f) * P.sp[1] - q.y;
                const float dyz2 = fmaf(dy, dy, dz * dz);
                const float rem = R2 - dyz2;
                if (rem <= 0.0f) continue;
                const float dxm = __builtin_amdgcn_sqrtf(rem);
                const int32_t i0 = max(f0[0], (int32_t)ceilf((q.x - dxm - P.lo[0]) / P.sp[0] - 0.5f));
                const int32_t i1 = min(f1[0], (int32_t)floorf((q.x + dxm - P.lo[0]) / P.sp[0] - 0.5f));
                unsigned long long *rowp = acc + ((kk - o[2]) * SC_TY + (jj - o[1])) * SC_TX - o[0];
                float dx = P.lo[0] + ((float)i0 + 0.5f) * P.sp[0] - q.x;
                for (int32_t ii = i0; ii <= i1; ++ii, dx += P.sp[0]) {
                    const float r2 = fmaf(dx, dx, dyz2);
                    const float qq = __builtin_amdgcn_sqrtf(r2) * P.inv_h;
                    const float a = fmaxf(2.0f - qq, 0.0f);
                    const float b = fmaxf(1.0f - qq, 0.0f);
                    // M4 spline: 1 - 1.5q^2 + 0.75q^3 (q<1), 0.25(2-q)^3 (1<=q<2)
                    const float w = 0.25f * (a * a * a) - b * b * b;
                    const long long term = (long long)(int32_t)(w * ms);
                    atomicAdd(rowp + ii, (unsigned long long)term);
                }
            }
        }
    }
    __syncthreads();
    const double out_scale = (double)P.scale * (double)mref * (1.0 / 2147483648.0);
    for (int v = threadIdx.x; v < SC_TX * SC_TY * SC_TZ; v += SC_THREADS) {
        const int li = v % SC_TX, lj = (v / SC_TX) % SC_TY, lk = v / (SC_TX * SC_TY);
        if (li < nt[0] && lj < nt[1] && lk < nt[2]) {
            const long long sum = (long long)acc[v];
            dn[((int64_t)(o[1] + lj) * P.res[0] + (o[0] + li)) * P.res[2] + (o[2] + lk)] =
                (float)((double)sum * out_scale);
        }
    }
}

// Rows of cells a scatter tile can touch (host check against SC_MAXROWS).
int scatter_max_rows(const SplatParams &P)
{
    int n = 1;
    const int tdim[3] = {SC_TX, SC_TY, SC_TZ};
    for (int a = 1; a < 3; ++a) {
        const float ext = (float)(tdim[a] - 1) * P.sp[a] + 4.0f * P.h;
        n *= (int)ceilf(ext * P.cg.inv_cell) + 4;
    }
    return n;
}

int scatter_rows_limit() { return SC_MAXROWS; }

hipError_t launch_splat_scatter(const SplatParams &P, const uint32_t *start, const float4 *sorted,
                                const uint32_t *mmax_bits, float *dn, const uint32_t *fail, hipStream_t s,
                                const KTimer &t)
{
    const int32_t ntx = (P.res[0] + SC_TX - 1) / SC_TX, nty = (P.res[1] + SC_TY - 1) / SC_TY,
                  ntz = (P.res[2] + SC_TZ - 1) / SC_TZ;
    const int32_t ntiles = ntx * nty * ntz;
    const int32_t per_xcd = (ntiles + 7) / 8;
    hipExtLaunchKernelGGL(k_splat_scatter, dim3((unsigned)(per_xcd * 8)), dim3(SC_THREADS), 0, s, t.start, t.stop, 0,
                          P, start, sorted, mmax_bits, ntx, nty, ntiles, per_xcd, dn, fail);
    return hipGetLastError();
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// A workgroup covers 64 (z) x 4 (x) rows of GP_Y voxels along y: grid
// (ceil(rz/64), ceil(rx/4), ceil(ry/GP_Y)), so no index division; lanes run
// along z, the fastest axis of the packed field, so its stores coalesce.
// Walking along y keeps the y-neighbours in registers (5 loads per voxel, not
// 7).
constexpr int GP_Y = 4;

template <int DT>
__device__ __forceinline__ void store_voxel(void *__restrict__ out, int32_t v, float c, float gx, float gy, float gz,
                                            float scale)
{
    if (DT == DT_F32) {
        reinterpret_cast<float4 *>(out)[v] = make_float4(c, gx, gy, gz);
    } else if (DT == DT_F16) {
        ushort4 h;
        h.x = __half_as_ushort(__float2half_rn(c * scale));
        h.y = __half_as_ushort(__float2half_rn(gx * scale));
        h.z = __half_as_ushort(__float2half_rn(gy * scale));
        h.w = __half_as_ushort(__float2half_rn(gz * scale));
        reinterpret_cast<ushort4 *>(out)[v] = h;
    } else {
        ushort4 h;
        h.x = f32_to_bf16_rne(c * scale);
        h.y = f32_to_bf16_rne(gx * scale);
        h.z = f32_to_bf16_rne(gy * scale);
        h.w = f32_to_bf16_rne(gz * scale);
        reinterpret_cast<ushort4 *>(out)[v] = h;
    }
}

// Inside: (f[i+1] - f[i-1]) / (2 d); faces: one-sided first difference.
__device__ __forceinline__ float central(float fm, float c, float fp, int32_t idx, int32_t n, float inv)
{
    if (idx == 0) return (fp - c) * inv;
    if (idx == n - 1) return (c - fm) * inv;
    return (fp - fm) * (0.5f * inv);
}

// The packed field keeps z fastest: voxel (i, j, k) at (j rx + i) rz + k.  z
// is the cameras' up axis (rays run across it): the 8 x 8 pixel tile a wave
// marches spans a few voxels in z and in one horizontal axis, and with z
// fastest its rows share cache lines whichever horizontal direction the view
// looks along (with x fastest, views along x gathered from twice the lines).
// delta_n is read with strides (dsx, dsy, dsz): z-fast from the splat,
// [z][y][x] from hz_index_field_from_grid.
template <int DT>
__global__ __launch_bounds__(256) void k_grad_pack(const float *__restrict__ dn, int32_t dsx, int32_t dsy,
                                                   int32_t dsz, int32_t rx, int32_t ry, int32_t rz, float ix,
                                                   float iy, float iz, float scale, int32_t gz, int32_t gx,
                                                   int32_t nblocks, int32_t per_xcd, void *__restrict__ out)
{
    // blocks (z, x, y) in that order, each XCD (workgroups are dealt
    // round-robin over the 8 XCDs) taking a contiguous run of them, so that
    // the neighbouring columns a block reads mostly sit in the same L2
    const int32_t blk = (int32_t)(blockIdx.x & 7u) * per_xcd + (int32_t)(blockIdx.x >> 3);
    if (blk >= nblocks) return;
    const int32_t bz = blk % gz, bx = (blk / gz) % gx, by = blk / (gz * gx);
    const int32_t k = bz * 64 + (int32_t)(threadIdx.x & 63);
    const int32_t i = bx * 4 + (int32_t)(threadIdx.x >> 6);
    const int32_t j0 = by * GP_Y;
    if (k >= rz || i >= rx) return;
    // voxel counts are below 2^31 (checked on the host): 32-bit index math
    int32_t u = i * dsx + j0 * dsy + k * dsz;    // delta_n
    int32_t v = (j0 * rx + i) * rz + k;          // packed voxel
    const int32_t vy = rx * rz;
    // x and z neighbours (and the y ones, from the walk) stay inside the
    // grid: a face uses the one-sided difference
    const int32_t xm = i > 0 ? -dsx : 0, xp = i < rx - 1 ? dsx : 0;
    const int32_t zm = k > 0 ? -dsz : 0, zp = k < rz - 1 ? dsz : 0;
    float ym = j0 > 0 ? dn[u - dsy] : 0.0f;
    float c = dn[u];
    const int32_t j1 = min(j0 + GP_Y, ry);
    for (int32_t j = j0; j < j1; ++j) {
        const float yp = j + 1 < ry ? dn[u + dsy] : 0.0f;
        const float gx = central(dn[u + xm], c, dn[u + xp], i, rx, ix);
        const float gy = central(ym, c, yp, j, ry, iy);
        const float gz = central(dn[u + zm], c, dn[u + zp], k, rz, iz);
        store_voxel<DT>(out, v, c, gx, gy, gz, scale);
        ym = c;
        c = yp;
        u += dsy;
        v += vy;
    }
}

// Packed (z-fast) field -> [z][y][x] arrays: one thread per output voxel v.
template <int DT>
__global__ __launch_bounds__(256) void k_field_unpack(const void *__restrict__ in, int32_t rx, int32_t ry,
                                                      int32_t rz, float inv_scale, float *__restrict__ dn,
                                                      float *__restrict__ gx, float *__restrict__ gy,
                                                      float *__restrict__ gz)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nxy = (int64_t)rx * ry;
    if (v >= nxy * rz) return;
    const int64_t k = v / nxy, r = v - k * nxy;
    const int64_t w = r * rz + k;   // r = j rx + i
    float4 f;
    if (DT == DT_F32) {
        f = reinterpret_cast<const float4 *>(in)[w];
    } else {
        const ushort4 h = reinterpret_cast<const ushort4 *>(in)[w];
        if (DT == DT_F16) {
            f = make_float4(__half2float(__ushort_as_half(h.x)), __half2float(__ushort_as_half(h.y)),
                            __half2float(__ushort_as_half(h.z)), __half2float(__ushort_as_half(h.w)));
        } else {
            f = make_float4(__uint_as_float((uint32_t)h.x << 16), __uint_as_float((uint32_t)h.y << 16),
                            __uint_as_float((uint32_t)h.z << 16), __uint_as_float((uint32_t)h.w << 16));
        }
        f.x *= inv_scale;
        f.y *= inv_scale;
        f.z *= inv_scale;
        f.w *= inv_scale;
    }
    if (dn) dn[v] = f.x;
    if (gx) gx[v] = f.y;
    if (gy) gy[v] = f.z;
    if (gz) gz[v] = f.w;
}

// ---------------------------------------------------------------------------
// host launchers (sizes validated by the caller)
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int32_t scan_tiles(int32_t ncells) { return (ncells + SCAN_TILE - 1) / SCAN_TILE; }

size_t scan_scratch_bytes(int32_t ncells) { return SCAN_TAG_OFFSET + 8u * (size_t)scan_tiles(ncells); }

bool scan_is_onepass(int32_t ncells) { return scan_tiles(ncells) <= SCAN_ONEPASS_TILES; }

uint32_t *scan_fail_word(void *scan) { return (uint32_t *)scan + 1; }

hipError_t launch_cell_list(const float *x, const float *y, const float *z, const float *m, int32_t n,
                            const CellGrid &cg, uint32_t *cid, uint32_t *count, int64_t count_clear_words,
                            uint32_t *start, uint32_t *lrank, uint32_t *slots, float4 *sorted, void *scan,
                            bool scan_reset, uint32_t *scan_base, bool want_mmax, const ScanGuard &guard,
                            uint32_t *bwork, int32_t nbricks, bool order, hipStream_t s, const KTimer &t)
{
    // The counts must start at zero; each scan leaves them so.
    // count[ncells+1] holds max |m| (scatter splat only), which the caller
    // clears through count_clear_words.  The scan scratch holds the one-pass
    // scan's ticket counter (word 0), the call's scan-failure word (word 1,
    // cleared by k_cell_count), and from byte SCAN_TAG_OFFSET the tile tags of
    // the one-pass scan (cleared with the counter by scan_reset) or the tile
    // sums of the three-pass one.
    uint32_t *fail = scan_fail_word(scan);
    const BrickOrder O{bwork, nbricks, bwork && order ? 1 : 0};
    const int32_t ntiles = scan_tiles(cg.ncells);
    const bool onepass = ntiles <= SCAN_ONEPASS_TILES;
    bool first = true;
    if (count_clear_words > 0) {
        hipExtLaunchKernelGGL(k_fill_u32, dim3(blocks_for(count_clear_words, 256)), dim3(256), 0, s, t.start, nullptr,
                              0, count, 0u, count_clear_words);
        first = false;
    }
    if (onepass && scan_reset) {
        const int64_t words = (int64_t)(scan_scratch_bytes(cg.ncells) / 4);
        hipExtLaunchKernelGGL(k_fill_u32, dim3(blocks_for(words, 256)), dim3(256), 0, s, first ? t.start : nullptr,
                              nullptr, 0, (uint32_t *)scan, 0u, words);
        first = false;
        *scan_base = 0;
    }
    if (want_mmax)
        hipExtLaunchKernelGGL(k_cell_count<true>, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                              first ? t.start : nullptr, nullptr, 0, x, y, z, m, n, cg, cid, lrank, count,
                              count + cg.ncells + 1, fail, BrickOrder{nullptr, 0, 0});
    else
        hipExtLaunchKernelGGL(k_cell_count<false>, dim3(blocks_for(n, 256) + (bwork ? 1 : 0)), dim3(256), 0, s,
                              first ? t.start : nullptr, nullptr, 0, x, y, z, m, n, cg, cid, lrank, count,
                              count + cg.ncells + 1, fail, O);
    if (onepass) {
        hipLaunchKernelGGL(k_scan_onepass, dim3((unsigned)ntiles), dim3(SCAN_THREADS), 0, s, count, cg.ncells, ntiles,
                           (uint32_t *)scan, (uint64_t *)((char *)scan + SCAN_TAG_OFFSET), *scan_base, start,
                           guard.spin_limit, guard.tag_bias, fail, guard.fail_host, guard.serial);
        *scan_base += (uint32_t)ntiles;
    } else {
        uint32_t *tile_sum = (uint32_t *)((char *)scan + SCAN_TAG_OFFSET);
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(SCAN_THREADS), 0, s, count, cg.ncells,
                           tile_sum);
        hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(SCAN_THREADS), 0, s, tile_sum, ntiles,
                           start + cg.ncells);
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(SCAN_THREADS), 0, s, count, cg.ncells,
                           tile_sum, start);
    }
    hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, cid, lrank, n, start, slots,
                       fail);
    hipExtLaunchKernelGGL(k_cell_order, dim3(blocks_for(n, 256) + (O.order ? 1 : 0)), dim3(256), 0, s, nullptr,
                          t.stop, 0, cid, start, slots, n, x, y, z, m, sorted, fail, O);
    return hipGetLastError();
}

// bwork (optional): receives each brick's candidate count (and their largest
// at bwork[2 nbricks], which the cell-count launch cleared); border
// (optional): the dispatch order of the bricks.
hipError_t launch_splat(const SplatParams &P, const uint32_t *start, const float4 *sorted, float *dn,
                        const uint32_t *fail, uint32_t *bwork, const uint32_t *border, hipStream_t s,
                        const KTimer &t)
{
    const int32_t nbricks = P.nbx * P.nby * P.nbz;
    const dim3 g((unsigned)nbricks), b(64 * SPLAT_WAVES);
    if (P.bz == 8)
        hipExtLaunchKernelGGL(k_splat<8>, g, b, 0, s, t.start, t.stop, 0, P, start, sorted, nbricks, dn,
                              fail, bwork, border);
    else
        hipExtLaunchKernelGGL(k_splat<4>, g, b, 0, s, t.start, t.stop, 0, P, start, sorted, nbricks, dn,
                              fail, bwork, border);
    return hipGetLastError();
}

// dn_zfast: delta_n as the splat writes it (z fastest: (j rx + i) rz + k);
// otherwise [z][y][x].
hipError_t launch_grad_pack(int dtype, const float *dn, bool dn_zfast, const int32_t res[3], const float inv_sp[3],
                            float scale, void *out, hipStream_t s, const KTimer &t)
{
    const int32_t gz = (res[2] + 63) / 64, gx = (res[0] + 3) / 4, gy = (res[1] + GP_Y - 1) / GP_Y;
    const int32_t nblocks = gz * gx * gy, per_xcd = (nblocks + 7) / 8;
    const dim3 g((unsigned)(per_xcd * 8)), b(256);
    const int32_t dsx = dn_zfast ? res[2] : 1, dsy = dn_zfast ? res[0] * res[2] : res[0],
                  dsz = dn_zfast ? 1 : res[0] * res[1];
    if (dtype == DT_F32)
        hipExtLaunchKernelGGL(k_grad_pack<DT_F32>, g, b, 0, s, t.start, t.stop, 0, dn, dsx, dsy, dsz, res[0], res[1],
                              res[2], inv_sp[0], inv_sp[1], inv_sp[2], scale, gz, gx, nblocks, per_xcd, out);
    else if (dtype == DT_F16)
        hipExtLaunchKernelGGL(k_grad_pack<DT_F16>, g, b, 0, s, t.start, t.stop, 0, dn, dsx, dsy, dsz, res[0], res[1],
                              res[2], inv_sp[0], inv_sp[1], inv_sp[2], scale, gz, gx, nblocks, per_xcd, out);
    else
        hipExtLaunchKernelGGL(k_grad_pack<DT_BF16>, g, b, 0, s, t.start, t.stop, 0, dn, dsx, dsy, dsz, res[0],
                              res[1], res[2], inv_sp[0], inv_sp[1], inv_sp[2], scale, gz, gx, nblocks, per_xcd, out);
    return hipGetLastError();
}

hipError_t launch_field_unpack(int dtype, const void *in, const int32_t res[3], float inv_scale, float *dn, float *gx,
                               float *gy, float *gz, hipStream_t s)
{
    const dim3 g(blocks_for((int64_t)res[0] * res[1] * res[2], 256)), b(256);
    if (dtype == DT_F32)
        hipLaunchKernelGGL(k_field_unpack<DT_F32>, g, b, 0, s, in, res[0], res[1], res[2], inv_scale, dn, gx, gy, gz);
    else if (dtype == DT_F16)
        hipLaunchKernelGGL(k_field_unpack<DT_F16>, g, b, 0, s, in, res[0], res[1], res[2], inv_scale, dn, gx, gy, gz);
    else
        hipLaunchKernelGGL(k_field_unpack<DT_BF16>, g, b, 0, s, in, res[0], res[1], res[2], inv_scale, dn, gx, gy,
                           gz);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace haze
