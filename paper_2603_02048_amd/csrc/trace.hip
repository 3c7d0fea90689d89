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
// Three launches per trace:
//   k_raygen  one thread per queue slot: pinhole ray, slab test against the
//             volume; rays that miss are finished at once, rays that enter
//             are binned by their chord length (longest first) and counted;
//             it also clears the counter set of the next launch
//   k_raygen_place  places the entering rays in a hit list sorted by bin
//             (wave ballots + mbcnt ranks, one atomic per workgroup and bin)
//   k_march   persistent waves pull hit rays from the list in batches of
//             64; once refill_min lanes have finished (by default all of
//             them), the idle lanes are refilled together (ballot of idle
//             lanes, one atomic per batch, mbcnt rank); finished rays write
//             their outputs at the next refill.  The length sort keeps the
//             lanes of a batch finishing together, and whole-batch refills
//             keep a wave's lanes one 8x8 pixel tile, whose rays gather from
//             few cache lines (see sample_field).
//             Each ray's arithmetic is independent of which lane or wave runs
//             it, so results are bitwise repeatable.
//
// Positions are float32 metres with a compensated (Kahan) sum of the steps.
// The direction is carried as an unnormalised vector p = wr + dw (entry
// direction plus accumulated turns); since normalize() ignores scale, adding
// |p| ds/n P g to p reproduces Eq. 16 exactly while dw keeps the low-order bits
// of many small turns that a unit vector would round away.
#include "haze_device.h"
#include "ray_geom.h"

#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstring>

namespace haze {

// Exit distance along w from a point in the volume (clamped at 0).
__device__ __forceinline__ float exit_distance(const TraceGrid &G, const float c[3], const float w[3])
{
    // per axis the face the ray heads for, chosen by value (a per-lane choice
    // of address would turn the uniform bounds into vector loads), and the
    // distance by the hardware reciprocal (~2 ulp); axes with w = 0 never exit
    float t = INFINITY;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float face = w[k] > 0.0f ? G.hi[k] : G.lo[k];
        const float tk = (face - c[k]) * __builtin_amdgcn_rcpf(w[k]);
        if (w[k] != 0.0f) t = fminf(t, tk);
    }
    return fmaxf(t, 0.0f);
}

__device__ __forceinline__ float quad_side(const SceneQuad &Q, const float x[3])
{
    return fmaf(Q.n[0], x[0], fmaf(Q.n[1], x[1], fmaf(Q.n[2], x[2], -Q.n0)));
}

__device__ __forceinline__ bool in_quad(const SceneQuad &Q, const float h[3])
{
    const float u = fmaf(Q.du[0], h[0], fmaf(Q.du[1], h[1], fmaf(Q.du[2], h[2], -Q.du0)));
    const float v = fmaf(Q.dv[0], h[0], fmaf(Q.dv[1], h[1], fmaf(Q.dv[2], h[2], -Q.dv0)));
    return u >= 0.0f && u <= 1.0f && v >= 0.0f && v <= 1.0f;
}

// First board met by the straight ray x + t w, t in [0, tmax]; ties go to the
// lower index.  Returns the board index or -1, and t.
__device__ __forceinline__ int cast_quads(const TraceLaunch &L, const float x[3], const float w[3], float tmax,
                                          float &thit)
{
    int best = -1;
    float bt = tmax;
    for (int k = 0; k < L.nquads; ++k) {
        const SceneQuad &Q = L.quads[k];
        const float dn = Q.n[0] * w[0] + Q.n[1] * w[1] + Q.n[2] * w[2];
        if (dn == 0.0f) continue;
        const float t = -quad_side(Q, x) / dn;
        if (!(t >= 0.0f) || t > bt || (t == bt && best >= 0)) continue;
        const float h[3] = {fmaf(t, w[0], x[0]), fmaf(t, w[1], x[1]), fmaf(t, w[2], x[2])};
        if (!in_quad(Q, h)) continue;
        best = k;
        bt = t;
    }
    thit = bt;
    return best;
}

// ---- triangle-mesh scenes ----

__device__ __forceinline__ bool in_tri(const SceneQuad &T, const float h[3])
{
    const float u = fmaf(T.du[0], h[0], fmaf(T.du[1], h[1], fmaf(T.du[2], h[2], -T.du0)));
    const float v = fmaf(T.dv[0], h[0], fmaf(T.dv[1], h[1], fmaf(T.dv[2], h[2], -T.dv0)));
    return u >= 0.0f && v >= 0.0f && u + v <= 1.0f;
}

// Straight ray x + t w against triangle k: keeps the first hit in (best, bt),
// ties to the lower triangle index.
__device__ __forceinline__ void cast_tri(const MeshLaunch &M, int k, const float x[3], const float w[3], int &best,
                                         float &bt)
{
    const SceneQuad &T = M.tris[k];
    const float dn = T.n[0] * w[0] + T.n[1] * w[1] + T.n[2] * w[2];
    if (dn == 0.0f) return;
    const float t = -quad_side(T, x) / dn;
    if (!(t >= 0.0f) || t > bt || (t == bt && best >= 0 && k >= best)) return;
    const float h[3] = {fmaf(t, w[0], x[0]), fmaf(t, w[1], x[1]), fmaf(t, w[2], x[2])};
    if (!in_tri(T, h)) return;
    best = k;
    bt = t;
}

// First triangle met by the straight ray x + t w, t in [0, tmax]: the ray
// walks the shell cells it crosses (3D DDA) and tests their lists, until the
// next cell starts beyond the best hit.  A cell lists every triangle within
// reach of it, so a hit inside a cell is found there whatever the rounding of
// the walk.  Returns the triangle or -1, and t; counts the exact tests.
__device__ int cast_mesh(const MeshLaunch &M, const float x[3], const float w[3], float tmax, float &thit,
                         uint32_t &ntests)
{
    int best = -1;
    float bt = tmax;
    if (M.brute) {
        for (int k = 0; k < M.ntris; ++k) cast_tri(M, k, x, w, best, bt);
        ntests += (uint32_t)M.ntris;
        thit = bt;
        return best;
    }
    float ta = 0.0f, tb = tmax;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = M.lo[a], hi = M.lo[a] + (float)M.res[a] * M.cell;
        if (w[a] == 0.0f) {
            if (x[a] < lo || x[a] > hi) ta = INFINITY;
            continue;
        }
        const float inv = 1.0f / w[a];
        const float t1 = (lo - x[a]) * inv, t2 = (hi - x[a]) * inv;
        ta = fmaxf(ta, fminf(t1, t2));
        tb = fminf(tb, fmaxf(t1, t2));
    }
    if (!(ta <= tb)) {
        thit = bt;
        return -1;
    }
    // per-axis walk state in scalars (an array indexed by the axis chosen at
    // run time would live in private memory)
    auto axis_start = [&](int a, int &ci, int &stp, float &tn, float &td) {
        const float p = fmaf(ta, w[a], x[a]);
        ci = min(max((int)floorf((p - M.lo[a]) * M.inv_cell), 0), M.res[a] - 1);
        if (w[a] > 0.0f) {
            stp = 1;
            tn = (M.lo[a] + (float)(ci + 1) * M.cell - x[a]) / w[a];
            td = M.cell / w[a];
        } else if (w[a] < 0.0f) {
            stp = -1;
            tn = (M.lo[a] + (float)ci * M.cell - x[a]) / w[a];
            td = -M.cell / w[a];
        } else {
            stp = 0;
            tn = INFINITY;
            td = INFINITY;
        }
    };
    int cx, cy, cz, sx, sy, sz;
    float tnx, tny, tnz, tdx, tdy, tdz;
    axis_start(0, cx, sx, tnx, tdx);
    axis_start(1, cy, sy, tny, tdy);
    axis_start(2, cz, sz, tnz, tdz);
    const int rx = M.res[0], ry = M.res[1], rz = M.res[2];
    float tenter = ta;
    for (int it = 0; it < rx + ry + rz + 3; ++it) {
        if (tenter > bt) break;
        const uint32_t cell = ((uint32_t)cz * (uint32_t)ry + (uint32_t)cy) * (uint32_t)rx + (uint32_t)cx;
        const uint32_t e0 = M.start[cell], e1 = M.start[cell + 1];
        for (uint32_t e = e0; e < e1; ++e) cast_tri(M, (int)M.list[e], x, w, best, bt);
        ntests += e1 - e0;
        if (tnx <= tny && tnx <= tnz) {
            tenter = tnx;
            cx += sx;
            tnx += tdx;
            if (cx < 0 || cx >= rx) break;
        } else if (tny <= tnz) {
            tenter = tny;
            cy += sy;
            tny += tdy;
            if (cy < 0 || cy >= ry) break;
        } else {
            tenter = tnz;
            cz += sz;
            tnz += tdz;
            if (cz < 0 || cz >= rz) break;
        }
        if (tenter > tb) break;
    }
    thit = bt;
    return best;
}

// The chord a -> b = a + ds w of one march step against triangle k: the side
// value changes sign (or reaches zero) along it; keeps the first crossing
// (fraction lam, then the lower index) in (best, bl, hp).
__device__ __forceinline__ void chord_tri(const MeshLaunch &M, int k, const float a[3], const float b[3],
                                          const float w[3], float ds, int &best, float &bl, float hp[3])
{
    const SceneQuad &T = M.tris[k];
    const float s0 = quad_side(T, a), s1 = quad_side(T, b);
    if (s0 == 0.0f || (s0 > 0.0f && s1 > 0.0f) || (s0 < 0.0f && s1 < 0.0f)) return;
    const float lam = s0 / (s0 - s1);
    if (!(lam < bl || (lam == bl && k < best))) return;
    const float back = (1.0f - lam) * ds;
    const float h[3] = {fmaf(-back, w[0], b[0]), fmaf(-back, w[1], b[1]), fmaf(-back, w[2], b[2])};
    if (!in_tri(T, h)) return;
    best = k;
    bl = lam;
    hp[0] = h[0]; hp[1] = h[1]; hp[2] = h[2];
}

// Writes a finished ray.  With surf >= 0 the ray already met scene board surf
// at hp; otherwise the straight ray (x, w) is cast against the boards and the
// view's backdrop plane (front side only) and the nearest wins, boards on
// ties.  The image point is re-projected through the pinhole: displacement =
// projected point - pixel centre (Sec. 3.3.2).
// Per-ray count of exact triangle tests of the ray's output, or null.
__device__ __forceinline__ uint32_t *tri_tests_of(const TraceLaunch &L, const Ray &r)
{
    return L.subset ? L.flat.tri_tests : L.jobs[r.job].tri_tests;
}

// SCENE 0: no scene; 1, 2: boards (surf is a board); 3: triangle mesh (surf
// is a triangle, reported by its surface id, and ntests counts the exact
// triangle tests the ray took so far).
template <int SCENE>
__device__ __forceinline__ void finish_ray(const TraceLaunch &L, const TraceJob &J, const Ray &r, const float x[3],
                                           const float w[3], uint32_t steps, int status, const float *hp = nullptr,
                                           int surf = -1, uint32_t ntests = 0u)
{
    constexpr bool BOARDS = SCENE == 1 || SCENE == 2;
    float disp0 = __builtin_nanf(""), disp1 = __builtin_nanf("");
    int sid = 255;
    if (status != 3) {
        float h[3];
        bool hit = surf >= 0;
        if (hit) {
            h[0] = hp[0]; h[1] = hp[1]; h[2] = hp[2];
            sid = (SCENE == 3 ? (int)L.mesh.surf[surf] : surf) + 1;
        } else {
            const float denom = w[0] * J.plane_n[0] + w[1] * J.plane_n[1] + w[2] * J.plane_n[2];
            float tb = -1.0f;
            if (denom < 0.0f) {
                tb = ((J.plane_p[0] - x[0]) * J.plane_n[0] + (J.plane_p[1] - x[1]) * J.plane_n[1] +
                      (J.plane_p[2] - x[2]) * J.plane_n[2]) / denom;
                if (!(tb >= 0.0f)) tb = -1.0f;
            }
            float t = tb;
            hit = tb >= 0.0f;
            sid = 0;
            if (BOARDS) {
                float tq;
                const int q = cast_quads(L, x, w, hit ? tb : INFINITY, tq);
                if (q >= 0) {
                    t = tq;
                    hit = true;
                    sid = q + 1;
                }
            }
            if (SCENE == 3) {
                float tq;
                const int q = cast_mesh(L.mesh, x, w, hit ? tb : INFINITY, tq, ntests);
                if (q >= 0) {
                    t = tq;
                    hit = true;
                    sid = (int)L.mesh.surf[q] + 1;
                }
            }
            if (hit) {
                h[0] = x[0] + t * w[0];
                h[1] = x[1] + t * w[1];
                h[2] = x[2] + t * w[2];
            }
        }
        float zc = 0.0f, xc = 0.0f, yc = 0.0f;
        if (hit) {
            const float hx = h[0] - J.eye[0];
            const float hy = h[1] - J.eye[1];
            const float hz = h[2] - J.eye[2];
            xc = hx * J.r[0] + hy * J.r[1] + hz * J.r[2];
            yc = hx * J.u[0] + hy * J.u[1] + hz * J.u[2];
            zc = hx * J.f[0] + hy * J.f[1] + hz * J.f[2];
            hit = zc > 0.0f;
        }
        if (hit) {
            disp0 = (J.half_w + J.fpx * xc / zc) - ((float)r.p + 0.5f);
            disp1 = (J.half_h - J.fpx * yc / zc) - ((float)r.q + 0.5f);
        } else {
            sid = 255;
            if (status == 0) status = 2;
        }
    }
    float *disp, *ep, *ed;
    uint32_t *st, *tt;
    uint8_t *stat, *sf;
    if (L.subset) {
        disp = L.flat.disp; ep = L.flat.exit_pos; ed = L.flat.exit_dir; st = L.flat.steps; stat = L.flat.status;
        sf = L.flat.surface; tt = L.flat.tri_tests;
    } else {
        disp = J.disp; ep = J.exit_pos; ed = J.exit_dir; st = J.steps; stat = J.status; sf = J.surface;
        tt = J.tri_tests;
    }
    if (BOARDS || sf) {
        if (sf) sf[r.out] = (uint8_t)sid;
    }
    if (SCENE == 3 && tt) tt[r.out] = ntests;   // the whole ray's exact triangle tests
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

// Part of a job table carried in the kernel arguments: the tracer's view
// table reaches the device without a host staging buffer.
constexpr int kTableChunkWords = 240;
struct TableChunk {
    uint32_t offset;   // destination word offset
    uint32_t nwords;
    uint32_t w[kTableChunkWords];
};

__global__ __launch_bounds__(256) void k_put_table(uint32_t *__restrict__ dst, TableChunk c)
{
    for (uint32_t i = threadIdx.x; i < c.nwords; i += blockDim.x) dst[c.offset + i] = c.w[i];
}

// Zero the bin totals, the placement cursors and the march batch head.
__global__ void k_trace_init(uint32_t *counters)
{
    for (int k = threadIdx.x; k <= kMarchHead; k += blockDim.x) *hit_counter(counters, k) = 0u;
}

// Per-wave counts of each bin among the lanes' bins (255: none) into
// wcnt[wave][bin]; returns the lane's rank among the wave's lanes of its bin.
__device__ __forceinline__ uint32_t bin_rank(int bin, uint32_t (*wcnt)[kRayBins])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < kRayBins) wcnt[wave][lane] = 0u;
    // only the bins present in the wave (a wave is a pixel tile, whose rays
    // have similar chords: usually one to three bins)
    uint32_t rank = 0;
    uint64_t todo = __ballot(bin < kRayBins);
    while (todo) {
        const int first = (int)__builtin_ctzll(todo);
        const int b = __builtin_amdgcn_readfirstlane(__shfl(bin, first));
        const uint64_t m = __ballot(bin == b);
        if (lane == 0) wcnt[wave][b] = (uint32_t)__popcll(m);
        if (bin == b)
            rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        todo &= ~m;
    }
    return rank;
}

// SCENE: 0 no scene, 1 boards, 3 triangle mesh (the launch's scene kind, so
// that the common case carries no scene code).
template <int SCENE>
__global__ __launch_bounds__(kRaygenBlock) void k_raygen(TraceLaunch L, const TraceJob *__restrict__ jobs)
{
    // A tile's slots run down its columns (decode_slot), but the rays that
    // miss write their outputs here, by pixel: the 64 threads of a tile take
    // its slots transposed, so neighbouring threads write neighbouring pixels
    // of a row.  (Which thread takes a slot changes nothing else: the counts
    // are per workgroup, and the hit list is placed in slot order.)
    const int l = (int)(threadIdx.x & 63);
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u) +
                         (L.subset ? l : (((l & 7) << 3) | (l >> 3)));
    bool enters = false;
    int bin = 255;
    // one ray: pinhole direction, entry into the volume, the rays that miss
    // (or meet the scene first) finished here
    const auto generate = [&](const TraceJob &J, Ray &r) {
        const float3 d3 = pixel_dir(J, r.p, r.q);
        const float d[3] = {d3.x, d3.y, d3.z};
        float t0, t1 = 0.0f;
        enters = enter_volume(L.grid, J.eye, d, t0, &t1);
        if (enters) bin = kRayBins - 1 - min(kRayBins - 1, max(0, (int)((t1 - t0) * L.inv_len_bin)));
        if (SCENE == 3) {
            if (enters) {
                // the mesh in front of the volume ends the ray before it enters;
                // otherwise the march continues the test count from here
                float tq;
                uint32_t nt = 0u;
                const int q = cast_mesh(L.mesh, J.eye, d, t0, tq, nt);
                if (q >= 0) {
                    const float hp[3] = {J.eye[0] + tq * d[0], J.eye[1] + tq * d[1], J.eye[2] + tq * d[2]};
                    finish_ray<3>(L, J, r, J.eye, d, 0u, 0, hp, q, nt);
                    enters = false;
                } else if (uint32_t *tt = tri_tests_of(L, r)) {
                    tt[r.out] = nt;
                }
            } else {
                finish_ray<3>(L, J, r, J.eye, d, 0u, 0);
            }
        } else if (SCENE == 1 && enters) {
            // a board in front of the volume ends the ray before it enters
            float tq;
            const int q = cast_quads(L, J.eye, d, t0, tq);
            if (q >= 0) {
                const float hp[3] = {J.eye[0] + tq * d[0], J.eye[1] + tq * d[1], J.eye[2] + tq * d[2]};
                finish_ray<1>(L, J, r, J.eye, d, 0u, 0, hp, q);
                enters = false;
            }
        } else if (!enters) {
            finish_ray<SCENE == 1 ? 1 : 0>(L, J, r, J.eye, d, 0u, 0);
        }
    };
    if (!L.subset) {
        // a wave's 64 slots are one 8x8 tile of one view: the view is found,
        // and read, with scalar loads (`jobs` is L.jobs, which nothing here
        // writes)
        const uint32_t base =
            __builtin_amdgcn_readfirstlane((uint32_t)(blockIdx.x * blockDim.x + (threadIdx.x & ~63u)));
        if ((int64_t)base < L.nslots) {
            const int job = job_of_slot(jobs, L.njobs, base);
            const TraceJob &J = jobs[job];
            Ray r;
            if (slot < L.nslots && decode_tile_slot(J, job, slot, r)) generate(J, r);
        }
    } else if (slot < L.nslots) {
        Ray r;
        if (decode_slot(L, slot, r)) {
            generate(L.jobs[r.job], r);
        } else {
            // ray id outside the views: flag it, leave no stale values behind
            const float nan = __builtin_nanf("");
            if (L.flat.disp) L.flat.disp[2 * slot] = L.flat.disp[2 * slot + 1] = nan;
            if (L.flat.exit_pos)
                L.flat.exit_pos[3 * slot] = L.flat.exit_pos[3 * slot + 1] = L.flat.exit_pos[3 * slot + 2] = nan;
            if (L.flat.exit_dir)
                L.flat.exit_dir[3 * slot] = L.flat.exit_dir[3 * slot + 1] = L.flat.exit_dir[3 * slot + 2] = nan;
            if (L.flat.steps) L.flat.steps[slot] = 0u;
            if (L.flat.status) L.flat.status[slot] = 4u;
            if (L.flat.surface) L.flat.surface[slot] = 255u;
            if (L.flat.tri_tests) L.flat.tri_tests[slot] = 0u;
        }
    }
    // the next launch's counter set (this launch's march uses the other one)
    static_assert(kMarchHead < kRaygenBlock, "one workgroup clears a counter set");
    if (blockIdx.x == 0 && threadIdx.x <= kMarchHead) *hit_counter(L.counters_next, threadIdx.x) = 0u;
    // pass 1 of the length sort: remember the bin, count the bins of the
    // workgroup (wave ballots), one atomic per non-empty bin
    if (!enters) bin = 255;
    if (slot < L.nslots) L.slot_bin[slot] = (uint8_t)bin;
    __shared__ uint32_t wcnt[kRaygenBlock / 64][kRayBins];
    bin_rank(bin, wcnt);
    __syncthreads();
    if (threadIdx.x < kRayBins) {
        uint32_t total = 0;
        for (int w = 0; w < kRaygenBlock / 64; ++w) total += wcnt[w][threadIdx.x];
        if (total) atomicAdd(hit_counter(L.counters, threadIdx.x), total);
    }
}

// Pass 2 of the length sort: each entering ray takes its place in its bin's
// range of the hit list (bins in order, longest rays first).  The order inside
// a bin depends on the atomics, which changes no ray's result.
__global__ __launch_bounds__(kRaygenBlock) void k_raygen_place(TraceLaunch L)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int bin = slot < L.nslots ? (int)L.slot_bin[slot] : 255;
    __shared__ uint32_t wcnt[kRaygenBlock / 64][kRayBins];
    __shared__ uint32_t tot[kRayBins];
    __shared__ uint32_t base[kRayBins];
    if (threadIdx.x < kRayBins) tot[threadIdx.x] = *hit_counter(L.counters, threadIdx.x);
    const uint32_t rank = bin_rank(bin, wcnt);
    __syncthreads();
    if (threadIdx.x < kRayBins) {
        const int b = threadIdx.x;
        uint32_t total = 0, start = 0;
        for (int w = 0; w < kRaygenBlock / 64; ++w) total += wcnt[w][b];
        for (int k = 0; k < b; ++k) start += tot[k];
        base[b] = total ? start + atomicAdd(hit_counter(L.counters, kRayBins + b), total) : 0u;
    }
    __syncthreads();
    if (bin < kRayBins) {
        uint32_t off = base[bin] + rank;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) off += wcnt[w][bin];
        L.hits[off] = (uint32_t)slot;
    }
}

__device__ __forceinline__ void wsum(float4 &v, float wgt, const float4 &c)
{
    v.x = fmaf(wgt, c.x, v.x);
    v.y = fmaf(wgt, c.y, v.y);
    v.z = fmaf(wgt, c.z, v.z);
    v.w = fmaf(wgt, c.w, v.w);
}

// Cell of x and the trilinear weights in it: cell index clamped to [0, R-2],
// so the outer half-voxel extrapolates linearly; b is the index of the
// cell's corner voxel in the packed field, whose fastest axis is z
// (k_grad_pack).  (Fields hold fewer than
// 2^31 voxels, checked on the host: 32-bit indices.  A NaN coordinate
// converts to cell 0 and poisons the weights, which the march's finiteness
// test catches.)
__device__ __forceinline__ void cell_of(const TraceGrid &G, const float x[3], uint32_t &b, float t[3])
{
    uint32_t i[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = fmaf(x[a], G.inv_sp[a], G.off[a]);
        const float fl = __builtin_amdgcn_fmed3f(floorf(u), 0.0f, G.maxi[a]);
        i[a] = (uint32_t)fl;
        t[a] = u - fl;
    }
    b = (i[1] * (uint32_t)G.res[0] + i[0]) * (uint32_t)G.res[2] + i[2];
}

// F16/BF16 voxels are 8 bytes; the two z-neighbours of a cell row are one
// 16-byte load (8-byte aligned, which the hardware serves as one dwordx4).
typedef uint32_t u32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));
// The field pointer reaches the kernel through the job table, so the compiler
// cannot prove it is global memory; say so, to get global (not flat) loads.
typedef const u32x4_a8 __attribute__((address_space(1))) *gpair_ptr;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const f32x4 __attribute__((address_space(1))) *gfloat4_ptr;

__device__ __forceinline__ float4 load_f32x4(gfloat4_ptr F, uint32_t i)
{
    const f32x4 v = F[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

template <int DT>
__device__ __forceinline__ float4 half4_to_float4(uint32_t lo, uint32_t hi)
{
    if (DT == DT_F16) {
        return make_float4(__half2float(__ushort_as_half((unsigned short)(lo & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(lo >> 16))),
                           __half2float(__ushort_as_half((unsigned short)(hi & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(hi >> 16))));
    } else {
        return make_float4(__uint_as_float(lo << 16), __uint_as_float(lo & 0xffff0000u), __uint_as_float(hi << 16),
                           __uint_as_float(hi & 0xffff0000u));
    }
}

template <int DT>
__device__ __forceinline__ void load_pair_at(gpair_ptr p, float4 &a, float4 &b)
{
    const u32x4_a8 v = *p;
    a = half4_to_float4<DT>(v.x, v.y);
    b = half4_to_float4<DT>(v.z, v.w);
}

// Trilinear sample of (delta_n, grad n) at x (Sec. 3.3.1): 8 corners, 4 row
// loads of a z-neighbour pair each.  The gathers are bound by how the
// texture-address unit serves a wave's 64 addresses: lanes next to each other
// that fall in one cache line are served together.  The packed field keeps z
// (the cameras' up axis) fastest and the queue orders a tile's pixels
// column-major, so neighbouring lanes are vertically adjacent pixels whose
// rows share lines whatever horizontal direction the view looks along.  (With
// x fastest and row-major tiles only views along y coalesced: single 1280x720
// views along x took 1.8x as long.)
template <int DT>
__device__ __forceinline__ float4 sample_field(const TraceGrid &G, const void *__restrict__ f, const float x[3])
{
    uint32_t b;
    float t[3];
    cell_of(G, x, b, t);
    const uint32_t sx = (uint32_t)G.res[2], sy = (uint32_t)G.res[0] * (uint32_t)G.res[2];
    float4 c000, c100, c010, c110, c001, c101, c011, c111;
    // Addresses by 64-bit pointer steps from the corner voxel: the
    // z-neighbour is the load's immediate offset, and the x and y rows one add
    // each (instead of a 32-bit index and a 64-bit address per load).  The
    // corners keep their names whatever the layout, so the weighted sum below
    // runs in the same order.
    if (DT == DT_F32) {
        const gfloat4_ptr p0 = (gfloat4_ptr)f + b, p1 = p0 + sy;
        const gfloat4_ptr q0 = p0 + sx, q1 = p1 + sx;
        c000 = load_f32x4(p0, 0);
        c001 = load_f32x4(p0, 1);
        c100 = load_f32x4(q0, 0);
        c101 = load_f32x4(q0, 1);
        c010 = load_f32x4(p1, 0);
        c011 = load_f32x4(p1, 1);
        c110 = load_f32x4(q1, 0);
        c111 = load_f32x4(q1, 1);
    } else {
        const gpair_ptr p0 = (gpair_ptr)(reinterpret_cast<const uint16_t *>(f) + 4 * (size_t)b);
        const gpair_ptr p1 = (gpair_ptr)((const uint16_t __attribute__((address_space(1))) *)p0 + 4 * (size_t)sy);
        const gpair_ptr q0 = (gpair_ptr)((const uint16_t __attribute__((address_space(1))) *)p0 + 4 * (size_t)sx);
        const gpair_ptr q1 = (gpair_ptr)((const uint16_t __attribute__((address_space(1))) *)p1 + 4 * (size_t)sx);
        load_pair_at<DT>(p0, c000, c001);
        load_pair_at<DT>(q0, c100, c101);
        load_pair_at<DT>(p1, c010, c011);
        load_pair_at<DT>(q1, c110, c111);
    }
    // trilinear weights, then one FMA per corner and channel
    const float ux = 1.0f - t[0], uy = 1.0f - t[1], uz = 1.0f - t[2];
    const float a00 = ux * uy, a10 = t[0] * uy, a01 = ux * t[1], a11 = t[0] * t[1];
    const float w000 = a00 * uz, w100 = a10 * uz, w010 = a01 * uz, w110 = a11 * uz;
    const float w001 = a00 * t[2], w101 = a10 * t[2], w011 = a01 * t[2], w111 = a11 * t[2];
    float4 v;
    v.x = w000 * c000.x;
    v.y = w000 * c000.y;
    v.z = w000 * c000.z;
    v.w = w000 * c000.w;
    wsum(v, w100, c100);
    wsum(v, w010, c010);
    wsum(v, w110, c110);
    wsum(v, w001, c001);
    wsum(v, w101, c101);
    wsum(v, w011, c011);
    wsum(v, w111, c111);
    if (DT != DT_F32) {
        // stored values are scaled; interpolation is linear, so unscale once
        v.x *= G.inv_scale;
        v.y *= G.inv_scale;
        v.z *= G.inv_scale;
        v.w *= G.inv_scale;
    }
    return v;
}

// Distance from c to the nearest face of the box (negative outside).
__device__ __forceinline__ float face_distance(const TraceGrid &G, const float c[3])
{
    return fminf(fminf(fminf(c[0] - G.lo[0], G.hi[0] - c[0]), fminf(c[1] - G.lo[1], G.hi[1] - c[1])),
                 fminf(c[2] - G.lo[2], G.hi[2] - c[2]));
}

// SCENE 0: no scene boards; 1: boards, none near the volume (met only by the
// straight exit ray); 2: some boards may cross the volume, so the chord of
// every step is tested against those (L.ninner of them) and the first one
// crossed ends the ray at the crossing point.
template <int DT, int SCENE>
__device__ __forceinline__ void march(const TraceLaunch &L)
{
    const TraceGrid &G = L.grid;
    const TraceStep &S = L.step;
    uint32_t nh = 0;
    for (int k = 0; k < kRayBins; ++k) nh += *hit_counter(L.counters, k);
    nh = __builtin_amdgcn_readfirstlane(nh);
    const uint32_t refill_min = (uint32_t)max(1, min(64, L.refill_min));
    const int lane = threadIdx.x & 63;

    // Work distribution over the length-sorted hits.  Wave w first takes
    // hits [64 w, 64 w + 64) with no atomic; later batches of 64 come from one
    // counter past the static range, fetched one batch ahead (the atomic's
    // latency hides behind the march).  Each wave keeps its reserve
    // [next, end) of hit indices.
    const uint32_t blk = blockIdx.x, nblk = gridDim.x;
    const uint32_t nwaves = nblk * (blockDim.x >> 6);
    const uint32_t wave_id = __builtin_amdgcn_readfirstlane(blk * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const uint32_t sb = 64u;
    const uint32_t dyn0 = nwaves * sb;
    uint32_t next = min(wave_id * sb, nh);
    uint32_t end = min(next + sb, nh);
    bool done = next >= nh && dyn0 >= nh;
    bool pending = false;
    uint32_t pend_v = 0;

    bool active = false;
    Ray r{0, 0, 0, 0};
    const void *field = nullptr;
    // direction omega = p / |p| with p = wr + dw: wr is the entry direction and
    // dw accumulates the turns, so small turns keep their low-order bits
    float c[3] = {0, 0, 0}, cc[3] = {0, 0, 0}, w[3] = {0, 0, 1}, wr[3] = {0, 0, 1}, dw[3] = {0, 0, 0};
    float pnorm = 1.0f;
    float safe = 0.0f;   // lower bound of the distance from c to the box faces
    uint32_t steps = 0;
    float side[SCENE == 2 ? kMaxInner : 1];   // side values of the inner boards at c
    // A finished ray keeps its end state (c, w, steps) and writes its outputs
    // only when the wave refills or stops, so the output code runs once for
    // all lanes finished since, not once per finishing lane.
    int fin = -1;        // status of a finished ray not yet written (-1: none)
    int fin_surf = -1;   // its board or triangle (c is then the hit point), -1 for none
    uint32_t ntests = 0u;   // SCENE 3: the ray's exact triangle tests so far

    // Outer loop: refill the wave's idle lanes (wave-uniform bookkeeping);
    // inner loop: step the active lanes until enough of them have finished.
    // The refill and the step are separate loops, so the step loop carries
    // the rays' state alone (no joins with the refill code on every step).
    for (;;) {
        const uint64_t idle = __ballot(!active);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (!done) {
            if (fin >= 0) {
                finish_ray<SCENE>(L, L.jobs[r.job], r, c, w, steps, fin, c, fin_surf, ntests);
                fin = -1;
            }
            if (next == end) {
                uint32_t b;
                if (pending) {
                    b = __shfl(pend_v, 0);
                    pending = false;
                } else {
                    uint32_t v = 0;
                    if (lane == 0) v = dyn0 + atomicAdd(hit_counter(L.counters, kMarchHead), 64u);
                    b = __shfl(v, 0);
                }
                b = __builtin_amdgcn_readfirstlane(b);
                if (b >= nh) {
                    done = true;   // next == end: nothing left to hand out below
                } else {
                    next = b;
                    end = min(b + 64u, nh);
                }
            }
            if (!active && next < end) {
                const uint32_t k = next + __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (k < end) {
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
                    safe = face_distance(G, c);
                    steps = 0;
                    active = true;
                    if (SCENE == 3) {
                        const uint32_t *tt = tri_tests_of(L, r);
                        ntests = tt ? tt[r.out] : 0u;   // the straight part before the volume
                    }
                    if (SCENE == 2) {
#pragma unroll
                        for (int j = 0; j < kMaxInner; ++j)
                            side[j] = j < L.ninner ? quad_side(L.quads[(L.inner_idx >> (8 * j)) & 255u], c) : 0.0f;
                    }
                }
            }
            next = min(next + nidle, end);
            if (!done && next == end && !pending) {
                if (dyn0 >= nh) {
                    done = true;   // the static batches hold every hit: no dynamic work
                } else {
                    if (lane == 0) pend_v = dyn0 + atomicAdd(hit_counter(L.counters, kMarchHead), 64u);
                    pending = true;
                }
            }
        }
        if (done && __ballot(active) == 0ull) {
            if (fin >= 0) finish_ray<SCENE>(L, L.jobs[r.job], r, c, w, steps, fin, c, fin_surf, ntests);
            break;
        }
        // once nothing is left to hand out, step until every lane is done
        const uint32_t want_idle = done ? 64u : refill_min;
        for (;;) {
            if (active) {
                // ---- one step of Eq. 16 with the step of Eq. 18 ----
                int status = -1;
                int hit_surf = -1;
                float te = INFINITY;
                bool near = safe <= S.near_cap;
                if (near) {
                    safe = face_distance(G, c);
                    near = safe <= S.near_cap;
                    if (near) {
                        te = exit_distance(G, c, w);
                        if (te <= S.tau) status = 0;
                    }
                }
                if (status < 0) {
                    const float4 s = sample_field<DT>(G, field, c);
                    const float n = 1.0f + s.x;
                    const float rn = __builtin_amdgcn_rcpf(n);
                    const float wg = w[0] * s.y + w[1] * s.z + w[2] * s.w;
                    const float pg0 = s.y - wg * w[0], pg1 = s.z - wg * w[1], pg2 = s.w - wg * w[2];
                    float ds;
                    if (S.uniform) {
                        ds = S.ds_uniform;
                    } else {
                        const float pgn = __builtin_amdgcn_sqrtf(pg0 * pg0 + pg1 * pg1 + pg2 * pg2);
                        // clamp to [ds_min, ds_max] (ds_min <= ds_max, checked on the host) in
                        // one med3: fminf/fmaxf would also canonicalize both bounds every step
                        ds = __builtin_amdgcn_fmed3f(n * S.theta_max * __builtin_amdgcn_rcpf(pgn + S.eps), S.ds_min,
                                                     S.ds_max);
                    }
                    ds = te < ds ? te : ds;   // min(ds, te) as a select: fminf would canonicalize both
                    // omega_{k+1} = normalize(omega_k + ds/n P g) = normalize(p + |p| ds/n P g)
                    const float a = ds * rn * pnorm;
                    dw[0] = fmaf(a, pg0, dw[0]);
                    dw[1] = fmaf(a, pg1, dw[1]);
                    dw[2] = fmaf(a, pg2, dw[2]);
                    const float p0 = wr[0] + dw[0], p1 = wr[1] + dw[1], p2 = wr[2] + dw[2];
                    const float pn2 = p0 * p0 + p1 * p1 + p2 * p2;
                    const float inv = __builtin_amdgcn_rsqf(pn2);
                    pnorm = pn2 * inv;
                    w[0] = p0 * inv;
                    w[1] = p1 * inv;
                    w[2] = p2 * inv;
                    float cp[3];   // C_k (SCENE 3)
                    if (SCENE == 3) {
                        cp[0] = c[0]; cp[1] = c[1]; cp[2] = c[2];
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        // compensated C += ds * w
                        const float y = fmaf(ds, w[k], -cc[k]);
                        const float t = c[k] + y;
                        cc[k] = (t - c[k]) - y;
                        c[k] = t;
                    }
                    ++steps;
                    safe -= ds;
                    int surf = -1;
                    float hp[3];
                    if (SCENE == 3) {
                        // chord C_k -> C_{k+1} against the triangles that the shell
                        // cell of C_k lists, unless the cell's distance bound
                        // exceeds the step (then no triangle is within reach)
                        const MeshLaunch &M = L.mesh;
                        float bl = 2.0f;
                        if (M.brute) {
                            for (int k = 0; k < M.ntris; ++k) chord_tri(M, k, cp, c, w, ds, surf, bl, hp);
                            ntests += (uint32_t)M.ntris;
                        } else {
                            int ci[3];
                            bool in = true;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                ci[a] = (int)floorf((cp[a] - M.lo[a]) * M.inv_cell);
                                in = in && ci[a] >= 0 && ci[a] < M.res[a];
                            }
                            if (in) {
                                const uint32_t cell = ((uint32_t)ci[2] * (uint32_t)M.res[1] + (uint32_t)ci[1]) *
                                                          (uint32_t)M.res[0] + (uint32_t)ci[0];
                                if (M.dlow[cell] <= ds * 1.001f) {
                                    const uint32_t e0 = M.start[cell], e1 = M.start[cell + 1];
                                    for (uint32_t e = e0; e < e1; ++e)
                                        chord_tri(M, (int)M.list[e], cp, c, w, ds, surf, bl, hp);
                                    ntests += e1 - e0;
                                }
                            }
                        }
                    }
                    if (SCENE == 2) {
                        // chord C_k -> C_{k+1} = C_{k+1} - ds w: the board whose side value
                        // changes sign (or reaches zero) first along it; ties go to the
                        // lower board index
                        float best = 2.0f;
#pragma unroll
                        for (int j = 0; j < kMaxInner; ++j) {
                            if (j >= L.ninner) continue;
                            const int k = (int)((L.inner_idx >> (8 * j)) & 255u);
                            const float s0 = side[j], s1 = quad_side(L.quads[k], c);
                            side[j] = s1;
                            if (s0 == 0.0f || (s0 > 0.0f && s1 > 0.0f) || (s0 < 0.0f && s1 < 0.0f)) continue;
                            const float lam = s0 / (s0 - s1);
                            if (!(lam < best)) continue;
                            const float back = (1.0f - lam) * ds;
                            const float h[3] = {fmaf(-back, w[0], c[0]), fmaf(-back, w[1], c[1]),
                                                fmaf(-back, w[2], c[2])};
                            if (!in_quad(L.quads[k], h)) continue;
                            best = lam;
                            surf = k;
                            hp[0] = h[0]; hp[1] = h[1]; hp[2] = h[2];
                        }
                    }
                    // a non-finite sample makes n or the direction vector p non-finite
                    // (or p zero); otherwise the step, direction and position stay finite
                    if (!(pn2 > 0.0f && pn2 < INFINITY && fabsf(n) < INFINITY))
                        status = 3;
                    else if ((SCENE == 2 || SCENE == 3) && surf >= 0) {
                        c[0] = hp[0]; c[1] = hp[1]; c[2] = hp[2];
                        status = 0;
                        hit_surf = surf;
                    } else if (safe <= S.pos_eps &&
                               (c[0] < G.lo[0] || c[0] > G.hi[0] || c[1] < G.lo[1] || c[1] > G.hi[1] ||
                                c[2] < G.lo[2] || c[2] > G.hi[2]))
                        status = 0;
                    else if ((int32_t)steps >= S.max_steps)
                        status = 1;
                }
                if (status >= 0) {
                    fin = status;
                    fin_surf = hit_surf;
                    active = false;
                }
            }
            if ((uint32_t)__popcll(__ballot(!active)) >= want_idle) break;
        }
    }
}

// Without boards, or with boards only outside the volume, the march fits six
// waves per SIMD (at most 80 VGPRs) with no spills; the board-crossing
// variant fits five (capped at six, it would spill).
#ifndef HZ_MARCH_F32_WAVES
#define HZ_MARCH_F32_WAVES 6
#endif
template <int DT, int SCENE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DT == DT_F32 ? HZ_MARCH_F32_WAVES : 6)))
void k_march(TraceLaunch L)
{
    march<DT, SCENE>(L);
}

template <int DT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_march_boards(TraceLaunch L)
{
    march<DT, 2>(L);
}

template <int DT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_march_mesh(TraceLaunch L)
{
    march<DT, 3>(L);
}

template <int DT, int SCENE>
static constexpr auto march_kernel()
{
    if constexpr (SCENE == 2)
        return &k_march_boards<DT>;
    else if constexpr (SCENE == 3)
        return &k_march_mesh<DT>;
    else
        return &k_march<DT, SCENE>;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

// Copy `bytes` (a multiple of 4) of host memory to device memory at `dst`
// through kernel arguments, in chunks of kTableChunkWords words.
hipError_t launch_put_table(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    TableChunk c;
    const uint32_t total = (uint32_t)(bytes / 4);
    for (uint32_t off = 0; off < total; off += kTableChunkWords) {
        c.offset = off;
        c.nwords = std::min<uint32_t>(kTableChunkWords, total - off);
        std::memcpy(c.w, (const uint32_t *)src + off, 4u * c.nwords);
        hipLaunchKernelGGL(k_put_table, dim3(1), dim3(256), 0, s, (uint32_t *)dst, c);
    }
    return hipGetLastError();
}

// Ray generation for L.nslots > 0 slots; `clear_counters` when the set
// L.counters was not cleared by the previous launch's ray generation (new
// memory, or after a failed launch).
hipError_t launch_raygen(const TraceLaunch &L, bool clear_counters, hipStream_t s, const KTimer &t)
{
    if (L.nslots <= 0) return hipSuccess;
    if (clear_counters)
        hipExtLaunchKernelGGL(k_trace_init, dim3(1), dim3(64), 0, s, t.start, nullptr, 0, L.counters);
    const dim3 g((unsigned)((L.nslots + kRaygenBlock - 1) / kRaygenBlock));
    hipEvent_t e0 = clear_counters ? nullptr : t.start;
    if (L.mesh.ntris > 0)
        hipExtLaunchKernelGGL(k_raygen<3>, g, dim3(kRaygenBlock), 0, s, e0, nullptr, 0, L, L.jobs);
    else if (L.nquads > 0)
        hipExtLaunchKernelGGL(k_raygen<1>, g, dim3(kRaygenBlock), 0, s, e0, nullptr, 0, L, L.jobs);
    else
        hipExtLaunchKernelGGL(k_raygen<0>, g, dim3(kRaygenBlock), 0, s, e0, nullptr, 0, L, L.jobs);
    hipExtLaunchKernelGGL(k_raygen_place, g, dim3(kRaygenBlock), 0, s, nullptr, t.stop, 0, L);
    return hipGetLastError();
}

template <int SCENE>
static void launch_march_t(int dtype, const TraceLaunch &L, int march_blocks, hipStream_t s, const KTimer &t)
{
    if (dtype == DT_F32)
        hipExtLaunchKernelGGL((march_kernel<DT_F32, SCENE>()), dim3(march_blocks), dim3(256), 0, s, t.start, t.stop, 0,
                              L);
    else if (dtype == DT_F16)
        hipExtLaunchKernelGGL((march_kernel<DT_F16, SCENE>()), dim3(march_blocks), dim3(256), 0, s, t.start, t.stop, 0,
                              L);
    else
        hipExtLaunchKernelGGL((march_kernel<DT_BF16, SCENE>()), dim3(march_blocks), dim3(256), 0, s, t.start, t.stop,
                              0, L);
}

hipError_t launch_march(int dtype, const TraceLaunch &L, int march_blocks, hipStream_t s, const KTimer &t)
{
    if (L.mesh.ntris > 0)
        launch_march_t<3>(dtype, L, march_blocks, s, t);
    else if (L.ninner > 0)
        launch_march_t<2>(dtype, L, march_blocks, s, t);
    else if (L.nquads > 0)
        launch_march_t<1>(dtype, L, march_blocks, s, t);
    else
        launch_march_t<0>(dtype, L, march_blocks, s, t);
    return hipGetLastError();
}

int march_scene_mode(const TraceLaunch &L) { return L.mesh.ntris > 0 ? 3 : L.ninner > 0 ? 2 : L.nquads > 0 ? 1 : 0; }

template <int SCENE>
static hipError_t occupancy(int dtype, int *nb)
{
    if (dtype == DT_F32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, march_kernel<DT_F32, SCENE>(), 256, 0);
    if (dtype == DT_F16)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, march_kernel<DT_F16, SCENE>(), 256, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, march_kernel<DT_BF16, SCENE>(), 256, 0);
}

int march_blocks_per_cu(int dtype, int scene_mode)
{
    int nb = 0;
    const hipError_t e = scene_mode == 3   ? occupancy<3>(dtype, &nb)
                         : scene_mode == 2 ? occupancy<2>(dtype, &nb)
                         : scene_mode == 1 ? occupancy<1>(dtype, &nb)
                                           : occupancy<0>(dtype, &nb);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace haze
