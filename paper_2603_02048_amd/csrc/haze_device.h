// haze_device.h -- structures shared by the gfx950 kernels and the host runtime
// of libhaze.so (internal; the public ABI is include/haze.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace haze {

// Timing events of a group of launches: the first launch records `start` when
// it begins and the last records `stop` when it ends (AMD dispatch-packet
// timestamps, no extra packets in the stream); null when profiling is off.
struct KTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Completion mark of a library call: the call's place in the context's
// numbering and the stream its work went to (seq 0: no call).
struct CallMark {
    uint64_t seq = 0;
    hipStream_t stream = nullptr;
};

// ---------------------------------------------------------------------------
// splat: particle cell list and brick gather
// ---------------------------------------------------------------------------

// Cell list over the grid box grown by the kernel support 2h on every side.
// Cells are cubes of edge `cell`; cell (cx, cy, cz) spans
// clo + (cx, cy, cz) * cell.  Particles outside the grown box are not binned.
struct CellGrid {
    float clo[3];
    float cell;
    float inv_cell;
    int32_t nc[3];
    int32_t ncells;
};

// Gather-splat brick: 8 x 8 lanes in x-y, each lane a column of bz voxels in z
// (4 or 8, whichever makes the brick closer to a cube).
constexpr int SPLAT_BX = 8, SPLAT_BY = 8;

// Bounded wait of the one-pass cell-list scan: spin_limit sleeps per lower
// tile before the wait gives up (tag_bias != 0 only in the fault test, where no
// tag matches); a wait that gives up stores `serial` into fail_host, a word
// of host memory the library reads at its next call.
struct ScanGuard {
    uint32_t spin_limit;
    uint32_t tag_bias;
    uint32_t *fail_host;
    uint32_t serial;
};

// Geometry and constants of one splat launch.
struct SplatParams {
    float lo[3];          // grid box corner
    float sp[3];          // voxel spacing
    int32_t res[3];
    int32_t bz;            // gather brick depth: 4 or 8 voxels
    int32_t nbx, nby, nbz; // gather bricks (SPLAT_BX x SPLAT_BY x bz voxels) per axis
    float h;
    float inv_h;
    float support2;       // (2h)^2
    float scale;          // k_gd / (pi h^3)
    CellGrid cg;
};

// ---------------------------------------------------------------------------
// trace: launch-uniform grid/step data and per-view jobs
// ---------------------------------------------------------------------------

// One view of one request.  Everything a ray of this view needs besides the
// launch-uniform grid and step data.  Host code fills it; 16-byte aligned.
struct alignas(16) TraceJob {
    float eye[3];
    float fpx;            // focal length in pixels: (H/2) / tan(vfov/2)
    float f[3];           // unit forward
    float half_w;         // W/2
    float r[3];           // unit right = normalize(f x up)
    float half_h;         // H/2
    float u[3];           // unit up = r x f
    int32_t width;
    float plane_p[3];
    int32_t height;
    float plane_n[3];
    int32_t tiles_x;      // 8x8 pixel tiles per row
    const void *field;    // packed (delta_n, grad) voxels of this view's field
    int64_t slot_begin;   // first queue slot (8x8 tile order) of this view
    int64_t ray_begin;    // first global ray id (row-major order) of this view
    float *disp;          // outputs of this view, indexed q * width + p
    float *exit_pos;
    float *exit_dir;
    uint32_t *steps;
    uint8_t *status;
    uint8_t *surface;     // optional: 0 backdrop, k + 1 scene quad k (or mesh surface k), 255 none
    uint32_t *tri_tests;  // optional (mesh scenes): exact ray-triangle tests the ray took
};

struct TraceGrid {
    float lo[3], hi[3];
    float inv_sp[3];       // 1 / spacing
    float off[3];          // -lo / spacing - 1/2  (u = x * inv_sp + off)
    float maxi[3];         // res - 2 (largest cell index) as float
    int32_t res[3];
    float inv_scale;       // 1 / store_scale
};

struct TraceStep {
    int32_t uniform;
    float theta_max, ds_min, ds_max, eps, ds_uniform, tau;
    int32_t max_steps;
    float near_cap;        // a point closer than this to a face may need the exit clamp
    float pos_eps;         // rounding margin of coordinates inside the box
};

struct TraceOutFlat {      // outputs indexed by queue position (ray-subset mode)
    float *disp;
    float *exit_pos;
    float *exit_dir;
    uint32_t *steps;
    uint8_t *status;
    uint8_t *surface;
    uint32_t *tri_tests;
};

// A planar scene board (parallelogram), as affine functions of the position:
//   side(x) = n . x - n0    (n unit normal; the board's plane is side = 0)
//   u(x)    = du . x - du0,  v(x) = dv . x - dv0   (board = 0 <= u, v <= 1)
// Up to kMaxQuads boards per launch, of which at most kMaxInner may come
// within a voxel of the volume (those are tested on every step).
constexpr int kMaxQuads = 8;
constexpr int kMaxInner = 4;
struct SceneQuad {
    float n[3], n0;
    float du[3], du0;
    float dv[3], dv0;
};

// A triangle-mesh scene (paper Sec. 4.1): each triangle as a SceneQuad whose
// u, v functions are the barycentric coordinates (inside: u, v >= 0,
// u + v <= 1), and a conservative shell on a coarse grid: per cell a lower
// bound of the distance from any point of the cell to the mesh, and the list
// of triangles within `reach` (the longest chord served) of the cell.  A chord
// of a march step starting in a cell whose bound exceeds the step length
// cannot meet the mesh and takes no exact test; straight rays walk the cells
// they cross (3D DDA) and test the cells' lists.  brute = 1: no shell, every
// test against every triangle (for comparison).
constexpr int32_t kMaxMeshTriangles = 65536;
constexpr int64_t kMaxShellCells = (int64_t)1 << 22;
struct MeshLaunch {
    const SceneQuad *tris;
    const uint8_t *surf;       // surface id of each triangle (a hit reports it + 1)
    const float *dlow;         // per cell
    const uint32_t *start;     // per cell, ncells + 1 entries
    const uint32_t *list;      // triangle indices, ascending within a cell
    float lo[3];               // shell grid corner
    float cell;                // cell edge
    float inv_cell;
    int32_t res[3];
    int32_t ntris;
    int32_t brute;
};

struct TraceLaunch {
    const TraceJob *jobs;
    int32_t njobs;
    int32_t subset;        // 1: slots are positions in ray_ids; 0: 8x8 tile order over jobs
    int64_t nslots;
    const int64_t *ray_ids;
    TraceOutFlat flat;
    uint32_t *hits;        // slots of the rays that enter the volume, sorted by length bin
    uint8_t *slot_bin;     // per slot: length bin of an entering ray, 255 otherwise
    uint32_t *counters;    // bin totals, placement cursors, march batch head (hit_counter)
    uint32_t *counters_next;   // the other set, cleared here for the next launch
    float inv_len_bin;     // kRayBins / (box diagonal): chord length -> bin
    TraceGrid grid;
    TraceStep step;
    int32_t refill_min;    // refill a wave once this many lanes are idle
    int32_t nquads;        // scene boards, tested before, inside and after the volume
    int32_t ninner;        // boards that may cross the volume: tested on every step
    uint32_t inner_idx;    // their indices, one byte each (lowest byte first)
    const SceneQuad *quads;  // device copy of the nquads boards
    MeshLaunch mesh;       // triangle-mesh scene (mesh.ntris > 0), exclusive of boards
};

// Ray generation sorts the entering rays by their straight chord through the
// volume (a proxy for their step count), longest first, in kRayBins bins: the
// march then hands out rays of similar length to each wave, so lanes finish
// together, and the longest rays start first.  Pass 1 finishes the rays that
// miss and counts the bins (one atomic per workgroup and non-empty bin); pass
// 2 places each ray in its bin's range of the hit list.  Counters sit
// kCounterStride words (256 B) apart so that no two share a cache line:
// bin totals [0, kRayBins), placement cursors [kRayBins, 2 kRayBins), and the
// march's dynamic batch head at 2 kRayBins.  Counter memory holds two such
// sets used by alternate launches: ray generation clears the set the next
// launch will use, so no launch of its own clears counters (new memory is
// cleared once by k_trace_init).
constexpr int kRayBins = 32;
constexpr int kCounterStride = 64;
constexpr int kRaygenBlock = 1024;
constexpr int kMarchHead = 2 * kRayBins;
constexpr size_t kCounterSetWords = (size_t)(kMarchHead + 1) * kCounterStride;
constexpr size_t kCounterBytes = 2 * kCounterSetWords * 4;
__host__ __device__ inline uint32_t *hit_counter(uint32_t *counters, int k) { return counters + k * kCounterStride; }

// Field storage types (match hz_dtype).
enum { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

}  // namespace haze
