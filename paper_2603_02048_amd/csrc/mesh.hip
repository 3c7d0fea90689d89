// mesh.hip -- triangle-mesh scenes and their conservative shell (paper Sec.
// 4.1: exact ray-triangle tests are done only once the refracted ray has
// entered a conservative shell precomputed around the scene geometry).
//
// The shell is a coarse uniform grid over the mesh's box grown by the reach
// (the longest chord it serves) and one cell.  Per cell it holds
//   dlow  a lower bound of the distance from any point of the cell to the
//         mesh: (distance from the cell centre to the nearest triangle) minus
//         half the cell diagonal, minus a rounding margin, at least 0;
//   list  every triangle within reach of the cell: those whose distance from
//         the cell centre is at most half the diagonal plus the reach (plus
//         the margin), in ascending index order.
// A march step of length ds starting at C_k meets no triangle when dlow of
// C_k's cell exceeds ds, and otherwise only triangles of the cell's list; a
// straight ray meets a triangle only in a cell it crosses, whose list holds
// it.  The shell therefore changes which exact tests run, never their
// outcome: with brute_force set, every test runs against every triangle and
// the results are the same bits (tests/test_gpu_mesh.py checks this).
//
// The shell is built on the device: one thread per cell walks all triangles
// twice (counts and bounds, then the lists); the list offsets are a host scan
// of the counts.  The build is a set-up step, done once per mesh.
#include "haze.h"
#include "haze_device.h"
#include "serve.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace haze {

// Geometry of the shell grid for the build kernels.
struct ShellGeom {
    float lo[3];
    float cell;
    int32_t res[3];
    float half_diag;
    float list_radius;   // half_diag + reach + margin
    float margin;
};

// Distance from p to the triangle (a, b, c): the closest point is a vertex,
// a point of an edge or an interior point, according to which region of the
// triangle's plane p projects into (the Voronoi regions of the vertices and
// edges, tested with the dot products of p's offsets with the edges).
__device__ float point_triangle_distance(const float p[3], const float a[3], const float b[3], const float c[3])
{
    // no contraction: both build passes must take the same decisions
#pragma clang fp contract(off)
    float ab[3], ac[3], ap[3], q[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ac[k] = c[k] - a[k];
        ap[k] = p[k] - a[k];
    }
    auto dot = [](const float *u, const float *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    const float d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0f && d2 <= 0.0f) {
        for (int k = 0; k < 3; ++k) q[k] = a[k];
    } else {
        float bp[3], cp[3];
        for (int k = 0; k < 3; ++k) {
            bp[k] = p[k] - b[k];
            cp[k] = p[k] - c[k];
        }
        const float d3 = dot(ab, bp), d4 = dot(ac, bp);
        const float d5 = dot(ab, cp), d6 = dot(ac, cp);
        const float vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
        if (d3 >= 0.0f && d4 <= d3) {                     // vertex b
            for (int k = 0; k < 3; ++k) q[k] = b[k];
        } else if (d6 >= 0.0f && d5 <= d6) {              // vertex c
            for (int k = 0; k < 3; ++k) q[k] = c[k];
        } else if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {   // edge ab
            const float t = d1 / (d1 - d3);
            for (int k = 0; k < 3; ++k) q[k] = a[k] + t * ab[k];
        } else if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {   // edge ac
            const float t = d2 / (d2 - d6);
            for (int k = 0; k < 3; ++k) q[k] = a[k] + t * ac[k];
        } else if (va <= 0.0f && d4 - d3 >= 0.0f && d5 - d6 >= 0.0f) {   // edge bc
            const float t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
            for (int k = 0; k < 3; ++k) q[k] = b[k] + t * (c[k] - b[k]);
        } else {                                          // interior
            const float inv = 1.0f / (va + vb + vc);
            const float v = vb * inv, w = vc * inv;
            for (int k = 0; k < 3; ++k) q[k] = a[k] + ab[k] * v + ac[k] * w;
        }
    }
    const float dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
    return sqrtf(dx * dx + dy * dy + dz * dz);
}

// FILL = false: per cell, the distance bound and the list length; FILL =
// true: the list itself (same distances, bit for bit).
template <bool FILL>
__global__ __launch_bounds__(256) void k_shell(ShellGeom G, const float *__restrict__ verts, int32_t ntris,
                                               float *__restrict__ dlow, uint32_t *__restrict__ count,
                                               const uint32_t *__restrict__ start, uint32_t *__restrict__ list)
{
    const int64_t ncells = (int64_t)G.res[0] * G.res[1] * G.res[2];
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncells) return;
    const int32_t ix = (int32_t)(cell % G.res[0]);
    const int32_t iy = (int32_t)((cell / G.res[0]) % G.res[1]);
    const int32_t iz = (int32_t)(cell / ((int64_t)G.res[0] * G.res[1]));
    const float p[3] = {G.lo[0] + ((float)ix + 0.5f) * G.cell, G.lo[1] + ((float)iy + 0.5f) * G.cell,
                        G.lo[2] + ((float)iz + 0.5f) * G.cell};
    float dmin = INFINITY;
    uint32_t n = 0, out = FILL ? start[cell] : 0u;
    const uint32_t end = FILL ? start[cell + 1] : 0u;
    for (int32_t t = 0; t < ntris; ++t) {
        const float *v = verts + 9 * (int64_t)t;
        const float d = point_triangle_distance(p, v, v + 3, v + 6);
        dmin = fminf(dmin, d);
        if (d <= G.list_radius) {
            if (FILL && out < end) list[out++] = (uint32_t)t;   // never past the cell's counted range
            ++n;
        }
    }
    if (!FILL) {
        dlow[cell] = fmaxf(0.0f, dmin - G.half_diag - G.margin);
        count[cell] = n;
    }
}

}  // namespace haze

using namespace haze;

struct hz_mesh {
    hz_ctx *ctx = nullptr;
    int32_t ntris = 0;
    float reach = 0.0f;
    int32_t brute = 0;
    MeshLaunch launch{};        // device pointers and grid for the tracer
    void *mem = nullptr;        // one device block: triangles, surfaces, dlow, starts, lists
    size_t bytes = 0;
    int64_t list_entries = 0;
    std::vector<CallMark> uses;   // latest call on each stream that traced with it
    std::mutex mu;
};

namespace haze {
const MeshLaunch &mesh_launch(const hz_mesh *m) { return m->launch; }
float mesh_reach(const hz_mesh *m) { return m->reach; }
hz_ctx *mesh_ctx(const hz_mesh *m) { return m->ctx; }
void mesh_use(hz_mesh *m, const CallMark &t)
{
    std::lock_guard<std::mutex> g(m->mu);
    for (CallMark &u : m->uses)
        if (u.stream == t.stream) {
            u = t;
            return;
        }
    m->uses.push_back(t);
}
}  // namespace haze

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" hz_status hz_mesh_create(hz_ctx *c, const hz_triangle *tris, int32_t ntris, const hz_mesh_params *prm,
                                    void *hip_stream, hz_mesh **out)
{
    if (!c || !tris || !prm || !out) return set_error(HZ_E_INVALID, "hz_mesh_create: NULL argument");
    if (ntris < 1 || ntris > kMaxMeshTriangles)
        return set_error(HZ_E_INVALID, "hz_mesh_create: ntris outside [1, 65536]");
    if (!(std::isfinite(prm->reach) && prm->reach > 0.0f))
        return set_error(HZ_E_INVALID, "hz_mesh_create: reach must be > 0");
    if (!(std::isfinite(prm->cell) && prm->cell >= 0.0f))
        return set_error(HZ_E_INVALID, "hz_mesh_create: cell must be >= 0");
    // triangles: validated, and as plane + barycentric functions (double on
    // the host, float for the kernels)
    std::vector<SceneQuad> tq((size_t)ntris);
    std::vector<uint8_t> surf((size_t)ntris);
    std::vector<float> verts(9 * (size_t)ntris);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = 0; i < ntris; ++i) {
        const hz_triangle &t = tris[i];
        double v0[3], e1[3], e2[3];
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(t.v0[a]) || !std::isfinite(t.v1[a]) || !std::isfinite(t.v2[a]))
                return set_error(HZ_E_INVALID, "hz_mesh_create: a triangle has non-finite vertices");
            v0[a] = t.v0[a];
            e1[a] = (double)t.v1[a] - t.v0[a];
            e2[a] = (double)t.v2[a] - t.v0[a];
            verts[9 * (size_t)i + a] = t.v0[a];
            verts[9 * (size_t)i + 3 + a] = t.v1[a];
            verts[9 * (size_t)i + 6 + a] = t.v2[a];
            for (const float v : {t.v0[a], t.v1[a], t.v2[a]}) {
                lo[a] = std::min(lo[a], (double)v);
                hi[a] = std::max(hi[a], (double)v);
            }
        }
        if (t.surface < 0 || t.surface > 253)
            return set_error(HZ_E_INVALID, "hz_mesh_create: surface ids must be in [0, 253]");
        surf[(size_t)i] = (uint8_t)t.surface;
        const double x[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        const double area = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        const double l2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        if (!(area > 1e-9 * l1 * l2) || !(area > 0.0))
            return set_error(HZ_E_INVALID, "hz_mesh_create: a triangle is degenerate (zero area)");
        const double n[3] = {x[0] / area, x[1] / area, x[2] / area};
        // du = (e2 x n) / area, dv = (n x e1) / area: barycentric u, v of a point
        const double du[3] = {(e2[1] * n[2] - e2[2] * n[1]) / area, (e2[2] * n[0] - e2[0] * n[2]) / area,
                              (e2[0] * n[1] - e2[1] * n[0]) / area};
        const double dv[3] = {(n[1] * e1[2] - n[2] * e1[1]) / area, (n[2] * e1[0] - n[0] * e1[2]) / area,
                              (n[0] * e1[1] - n[1] * e1[0]) / area};
        SceneQuad &Q = tq[(size_t)i];
        double on = 0.0, odu = 0.0, odv = 0.0;
        for (int a = 0; a < 3; ++a) {
            Q.n[a] = (float)n[a];
            Q.du[a] = (float)du[a];
            Q.dv[a] = (float)dv[a];
        }
        for (int a = 0; a < 3; ++a) {
            on += (double)Q.n[a] * v0[a];
            odu += (double)Q.du[a] * v0[a];
            odv += (double)Q.dv[a] * v0[a];
        }
        Q.n0 = (float)on;
        Q.du0 = (float)odu;
        Q.dv0 = (float)odv;
    }
    // shell grid: the mesh box grown by reach + one cell; cells of edge
    // `cell` (default four reaches), coarsened until it has at most
    // kMaxShellCells cells and 512 per axis
    ShellGeom G{};
    double cell = prm->cell > 0.0f ? (double)prm->cell : 4.0 * (double)prm->reach;
    double amax = 0.0;
    for (int a = 0; a < 3; ++a) amax = std::max(amax, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
    for (;;) {
        int64_t n = 1;
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            const double ext = hi[a] - lo[a] + 2.0 * ((double)prm->reach + cell);
            const int64_t r = (int64_t)std::ceil(ext / cell);
            ok = ok && r <= 512;
            n *= r;
        }
        if (ok && n <= kMaxShellCells) break;
        cell *= 1.25;
    }
    for (int a = 0; a < 3; ++a) {
        const double glo = lo[a] - ((double)prm->reach + cell);
        const double ext = hi[a] - lo[a] + 2.0 * ((double)prm->reach + cell);
        G.lo[a] = (float)glo;
        G.res[a] = (int32_t)std::ceil(ext / cell);
    }
    G.cell = (float)cell;
    G.half_diag = (float)(0.5 * std::sqrt(3.0) * cell);
    // rounding of the float distance and cell-centre arithmetic: a few ulps of
    // the coordinates involved, far below the reach
    G.margin = (float)(1e-5 * cell + 4e-6 * (amax + 2.0 * cell + (double)prm->reach));
    G.list_radius = G.half_diag + prm->reach + G.margin;
    const int64_t ncells = (int64_t)G.res[0] * G.res[1] * G.res[2];

    if (hipSetDevice(ctx_device(c)) != hipSuccess) return set_error(HZ_E_DEVICE, "hz_mesh_create: hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    // build buffers (freed at the end) and the first part of the mesh block
    const size_t vbytes = 4 * verts.size();
    void *build = nullptr;
    hz_status st = ctx_alloc(c, &build, align256(vbytes) + 4 * (size_t)(ncells + 1));
    if (st != HZ_OK) return st;
    float *dverts = (float *)build;
    uint32_t *dcount = (uint32_t *)((char *)build + align256(vbytes));
    const size_t off_surf = align256(sizeof(SceneQuad) * (size_t)ntris);
    const size_t off_dlow = off_surf + align256((size_t)ntris);
    const size_t off_start = off_dlow + align256(4 * (size_t)ncells);
    const size_t off_list = off_start + align256(4 * (size_t)(ncells + 1));
    std::vector<uint32_t> counts((size_t)ncells);
    hz_mesh *m = new hz_mesh();
    m->ctx = c;
    m->ntris = ntris;
    m->reach = prm->reach;
    m->brute = prm->brute_force ? 1 : 0;
    void *pre = nullptr;
    st = ctx_alloc(c, &pre, off_list);
    auto fail_all = [&](hz_status e) {
        if (pre) ctx_free(c, pre, off_list);
        ctx_free(c, build, align256(vbytes) + 4 * (size_t)(ncells + 1));
        delete m;
        return e;
    };
    if (st != HZ_OK) return fail_all(st);
    const unsigned blocks = (unsigned)((ncells + 255) / 256);
    if (hipMemcpyAsync(dverts, verts.data(), vbytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail_all(set_error(HZ_E_DEVICE, "hz_mesh_create: copy of the vertices failed"));
    hipLaunchKernelGGL(k_shell<false>, dim3(blocks), dim3(256), 0, s, G, (const float *)dverts, ntris,
                       (float *)((char *)pre + off_dlow), dcount, (const uint32_t *)nullptr, (uint32_t *)nullptr);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(counts.data(), dcount, 4 * (size_t)ncells, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail_all(set_error(HZ_E_DEVICE, "hz_mesh_create: shell bound pass failed"));
    std::vector<uint32_t> starts((size_t)ncells + 1);
    uint64_t total = 0;
    for (int64_t k = 0; k < ncells; ++k) {
        starts[(size_t)k] = (uint32_t)total;
        total += counts[(size_t)k];
    }
    if (total > 0xffffffffull / 2)
        return fail_all(set_error(HZ_E_UNSUPPORTED, "hz_mesh_create: shell lists too long (use a coarser cell)"));
    starts[(size_t)ncells] = (uint32_t)total;
    // the final block: triangles, surfaces, bounds, starts, lists
    const size_t bytes = off_list + align256(4 * (size_t)std::max<uint64_t>(total, 1));
    void *mem = nullptr;
    st = ctx_alloc(c, &mem, bytes);
    if (st != HZ_OK) return fail_all(st);
    bool ok = hipMemcpyAsync(mem, pre, off_list, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(mem, tq.data(), sizeof(SceneQuad) * tq.size(), hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync((char *)mem + off_surf, surf.data(), surf.size(), hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync((char *)mem + off_start, starts.data(), 4 * starts.size(), hipMemcpyHostToDevice, s) ==
                  hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_shell<true>, dim3(blocks), dim3(256), 0, s, G, (const float *)dverts, ntris,
                           (float *)nullptr, (uint32_t *)nullptr, (const uint32_t *)((char *)mem + off_start),
                           (uint32_t *)((char *)mem + off_list));
        ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
    }
    if (!ok) {
        ctx_free(c, mem, bytes);
        return fail_all(set_error(HZ_E_DEVICE, "hz_mesh_create: shell list pass failed"));
    }
    ctx_free(c, pre, off_list);
    pre = nullptr;
    ctx_free(c, build, align256(vbytes) + 4 * (size_t)(ncells + 1));
    m->mem = mem;
    m->bytes = bytes;
    m->list_entries = (int64_t)total;
    MeshLaunch &M = m->launch;
    M.tris = (const SceneQuad *)mem;
    M.surf = (const uint8_t *)((char *)mem + off_surf);
    M.dlow = (const float *)((char *)mem + off_dlow);
    M.start = (const uint32_t *)((char *)mem + off_start);
    M.list = (const uint32_t *)((char *)mem + off_list);
    for (int a = 0; a < 3; ++a) {
        M.lo[a] = G.lo[a];
        M.res[a] = G.res[a];
    }
    M.cell = G.cell;
    M.inv_cell = (float)(1.0 / cell);
    M.ntris = ntris;
    M.brute = m->brute;
    *out = m;
    return HZ_OK;
}

extern "C" hz_status hz_mesh_info(const hz_mesh *m, int32_t *ntris, int32_t shell_res[3], float *shell_cell,
                                  int64_t *list_entries, uint64_t *bytes)
{
    if (!m) return set_error(HZ_E_INVALID, "hz_mesh_info: mesh is NULL");
    if (ntris) *ntris = m->ntris;
    if (shell_res)
        for (int a = 0; a < 3; ++a) shell_res[a] = m->launch.res[a];
    if (shell_cell) *shell_cell = m->launch.cell;
    if (list_entries) *list_entries = m->list_entries;
    if (bytes) *bytes = m->bytes;
    return HZ_OK;
}

extern "C" hz_status hz_mesh_release(hz_ctx *c, hz_mesh *m)
{
    if (!c || !m) return set_error(HZ_E_INVALID, "hz_mesh_release: NULL argument");
    if (m->ctx != c) return set_error(HZ_E_INVALID, "hz_mesh_release: mesh belongs to another context");
    if (server_waiting_use(c, nullptr, m))
        return set_error(HZ_E_INVALID, "hz_mesh_release: a request waiting in the serving loop reads the mesh");
    (void)hipSetDevice(ctx_device(c));
    std::vector<CallMark> uses;
    {
        std::lock_guard<std::mutex> g(m->mu);
        uses = m->uses;
    }
    for (const CallMark &t : uses) (void)ctx_mark_sync(c, t);
    ctx_free(c, m->mem, m->bytes);
    delete m;
    return HZ_OK;
}
