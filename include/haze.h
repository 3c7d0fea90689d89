/*
 * haze.h -- C ABI of the MI355X (gfx950) splat-and-trace library `libhaze.so`.
 *
 * The library turns SPH particles into a refractive-index field and traces
 * curved camera rays through it:
 *
 *   1. hz_splat_index_field: density at voxel centres by SPH kernel splatting,
 *      mapped to the refractive-index excess delta_n = n - 1 = K_GD rho by the
 *      Gladstone-Dale relation (paper Sec. 3.3.1, Eq. 12), and its gradient
 *      grad n = K_GD grad rho by finite differences on the grid (Eq. 13).
 *   2. hz_trace_views: per pixel of every view, a ray that is straight outside
 *      the volume (Fig. 1 caption) and inside it follows the explicit update
 *        omega_{k+1} = normalize(omega_k + ds_k/n_k (I - omega_k omega_k^T) g_k)
 *        C_{k+1}     = C_k + ds_k omega_{k+1}                       (Eq. 16)
 *      with n_k, g_k trilinearly sampled (Sec. 3.3.1) and the step
 *        ds_k = clamp(n_k theta_max / (|(I - omega omega^T) g_k| + eps),
 *                     ds_min, ds_max)                     (Eqs. 17-18)
 *      or a fixed step (Sec. 4.1).  The image is formed only by bending
 *      (Sec. 3.3.2, last paragraph): the exit ray is intersected with a
 *      backdrop plane and re-projected through the same pinhole, giving a
 *      per-pixel displacement.
 *   3. hz_submit / hz_poll: the same trace as a request to a serving loop that
 *      batches concurrent multi-view requests into shared launches.
 *
 * Conventions
 *   - Lengths in metres, angles in radians, float32 unless stated.
 *   - "device" pointers are HIP device memory on the context's GPU; "host"
 *     pointers are ordinary process memory.  Structs passed by pointer are
 *     host memory and are only read during the call.
 *   - Grids are regular: voxel (i, j, k) has its centre at
 *     lo + (i + 1/2, j + 1/2, k + 1/2) * (hi - lo) / res; exported arrays are
 *     linear [z][y][x] (x fastest).
 *   - Work is enqueued on `hip_stream` (a hipStream_t, NULL = the default
 *     stream) and the call returns without waiting for it.  Device faults show
 *     up as HZ_E_DEVICE on a later call.  A call that reads a field built on
 *     another stream makes its own stream wait for the field; the traces
 *     generate their rays (which read no field data) before that wait, so ray
 *     generation can run while the field is still being built.
 *   - Every call returns an hz_status; nothing throws or aborts across the
 *     ABI.  On an error return no output has been written and no work queued,
 *     except for HZ_E_DEVICE from a failed launch or stream wait, which can
 *     come after part of the call's work was queued.
 *     hz_last_error() describes the most recent failure on the calling thread.
 *   - A context is not thread-safe, except hz_submit and hz_poll, which may be
 *     called from any thread.
 */
#ifndef HAZE_H
#define HAZE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HZ_OK = 0,
    HZ_PENDING = 1,         /* hz_poll: the request has not completed yet */
    HZ_E_INVALID = -1,      /* bad argument (null pointer, size, range) */
    HZ_E_NOMEM = -2,        /* the device allocator failed */
    HZ_E_BUDGET = -3,       /* the request can never fit the context's HBM budget */
    HZ_E_DEVICE = -4,       /* no usable GPU, or a HIP runtime/device error */
    HZ_E_NOTFOUND = -5,     /* unknown ticket */
    HZ_E_UNSUPPORTED = -6   /* valid but not supported by the library */
} hz_status;

/* Storage type of the index field.  Integration is always float32. */
typedef enum {
    HZ_F32 = 0,   /* 16 B per voxel: (delta_n, dn/dx, dn/dy, dn/dz) */
    HZ_F16 = 1,   /* 8 B per voxel, each channel stored as half(value * store_scale) */
    HZ_BF16 = 2   /* 8 B per voxel, each channel stored as bfloat16(value * store_scale) */
} hz_dtype;

/* Per-ray status codes written to hz_trace_out.status. */
enum {
    HZ_RAY_OK = 0,
    HZ_RAY_MAXSTEPS = 1,    /* max_steps reached inside the volume */
    HZ_RAY_NOHIT = 2,       /* exit ray misses the backdrop plane; disp is NaN */
    HZ_RAY_NONFINITE = 3,   /* position or direction became non-finite */
    HZ_RAY_BAD_ID = 4       /* ray_ids[i] is not a ray of the views; outputs are NaN */
};

typedef struct hz_ctx hz_ctx;       /* device, HBM ledger, scratch, serving loop */
typedef struct hz_field hz_field;   /* device-resident (delta_n, grad n) grid, immutable */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the library itself allocates (fields, scratch, serving buffers);
 * 0 means "free device memory at creation minus 1 GiB".
 * Errors: HZ_E_INVALID (out == NULL), HZ_E_DEVICE (no such device / no GPU). */
hz_status hz_ctx_create(int device, uint64_t hbm_budget_bytes, hz_ctx **out);

/* Wait for the context's outstanding work, release every field it still owns
 * and free the context.  NULL is ignored. */
void hz_ctx_destroy(hz_ctx *ctx);

/* Message for the last failure on the calling thread ("" if none).  The
 * string stays valid until the thread's next failing call. */
const char *hz_last_error(void);

/* Bytes of device memory the library currently holds for this context, and
 * its budget. */
hz_status hz_ctx_memory(const hz_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);

/* Tuning knobs.  The march knobs change speed only, never results; the splat
 * method and brick depth change only how delta_n is rounded (all meet the same
 * accuracy and each is bitwise repeatable):
 *   "march.refill_min"     refill a wave once this many of its 64 lanes are
 *                          idle, 1..64 (default 64: whole batches, so a
 *                          wave's lanes stay one pixel tile)
 *   "march.blocks_per_cu"  cap on resident 256-thread workgroups per CU,
 *                          0 = as many as fit (default 0)
 *   "splat.method"         0 or 1: gather (one workgroup per 8x8xBZ voxel
 *                          brick, fixed FP32 summation order; the default), 2: scatter
 *                          (voxel tiles with 64-bit fixed-point accumulation in
 *                          LDS; slower, for a support of up to ~16 cells per
 *                          tile axis, HZ_E_UNSUPPORTED beyond); both are
 *                          bitwise repeatable
 *   "splat.brick_z"        gather brick depth BZ: 4 or 8 voxels, 0 = the one
 *                          that brings the brick closer to twice as deep as
 *                          wide (default 0)
 *   "splat.order"          1: the gather hands out its bricks heaviest first,
 *                          by each brick's candidate count in the context's
 *                          previous gather over the same bricks (up to 65,536
 *                          bricks); 0: in index order.  The field is the same
 *                          bits either way (default 1)
 *   "splat.scan_fault_test" 1: the next splat calls' one-pass cell-list scans
 *                          wait for tile sums that never come, with a short
 *                          bound, so that the failure path runs (default 0;
 *                          for tests).  A scan whose bounded wait gives up
 *                          leaves NaN in the field it builds, the field is
 *                          marked unusable, and the first library call that
 *                          runs after the failing work has completed returns
 *                          HZ_E_DEVICE (as does every later call given that
 *                          field).
 * Errors: HZ_E_INVALID (unknown key or value out of range). */
hz_status hz_ctx_tune(hz_ctx *ctx, const char *key, int64_t value);

/* Per-kernel timing with HIP events that the launches themselves record (the
 * start of a group's first kernel, the end of its last), on the caller's
 * stream; groups: "cell_list", "splat", "grad_pack", "raygen" (ray generation
 * and the length sort), "march"; the serving loop's launches as
 * "serve_batch".  hz_profile_read waits for the recorded events and returns the
 * summed milliseconds and launch count of `kernel` since the last reset
 * (reset != 0 clears all sums after reading). */
hz_status hz_profile_enable(hz_ctx *ctx, int32_t enable);
/* Time only the listed groups (comma-separated names as above; NULL or ""
 * selects all, the default).  Each timed group costs its stream a few
 * microseconds per launch, so a run that needs one kernel's time selects it
 * alone.  Errors: HZ_E_INVALID (unknown group name). */
hz_status hz_profile_select(hz_ctx *ctx, const char *groups);
hz_status hz_profile_read(hz_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches, int32_t reset);

/* ---------------------------------------------------------------------- */
/* Index field (paper Sec. 3.3.1, Eqs. 12-13)                             */
/* ---------------------------------------------------------------------- */

/* Particle set, structure of arrays.  x, y, z, m are device pointers to n
 * float32 values each (positions in metres, masses in kg), caller-owned and
 * only read.  Particles farther than 2h from the grid box, or whose mass is
 * not finite, contribute nothing and are skipped. */
typedef struct {
    int64_t n;
    const float *x, *y, *z, *m;
} hz_particles;

/* Regular grid over the box [lo, hi] with res[0] x res[1] x res[2] voxels:
 * 2 <= res[a] <= 65535 on each axis and fewer than 2^31 voxels in all. */
typedef struct {
    double lo[3], hi[3];
    int32_t res[3];
} hz_grid;

/* Splat parameters.  The kernel is the M4 cubic spline with smoothing length
 * h (support 2h, normalisation 1/(pi h^3)).  store_scale multiplies every
 * channel before it is stored as F16/BF16 (it is divided out when the tracer
 * reads it); it must be 1 for F32. */
typedef struct {
    float k_gd;
    float h;
    hz_dtype dtype;
    float store_scale;
} hz_splat_params;

/* Build the index field of a particle set:
 *   delta_n(c) = k_gd * sum_j m_j W(|c - x_j|, h)  at every voxel centre c,
 *   grad n     = second-order central differences inside the grid and
 *                first-order one-sided differences on its faces.
 * The sum over particles runs in a fixed order, so the field is bitwise
 * identical across calls.  On success *out is a new field owned by the
 * context (release it with hz_field_release).
 * Errors: HZ_E_INVALID (null pointers, n < 1, res < 2 on an axis, hi <= lo,
 * h <= 0, non-finite k_gd, store_scale <= 0 or != 1 for F32, more than
 * 2^31 - 1 particles or voxels), HZ_E_BUDGET, HZ_E_NOMEM, HZ_E_DEVICE. */
hz_status hz_splat_index_field(hz_ctx *ctx, const hz_particles *particles, const hz_grid *grid,
                               const hz_splat_params *params, void *hip_stream, hz_field **out);

/* Build the index field from a given delta_n grid: `dn` is a device array of
 * res[0]*res[1]*res[2] float32 values, linear [z][y][x]; the gradient and the
 * storage conversion are computed as in hz_splat_index_field.  For callers
 * (and tests) that already have a density grid.
 * Errors: as hz_splat_index_field. */
hz_status hz_index_field_from_grid(hz_ctx *ctx, const float *dn, const hz_grid *grid, hz_dtype dtype,
                                   float store_scale, void *hip_stream, hz_field **out);

/* Export a field as four device arrays of res[0]*res[1]*res[2] float32 values,
 * linear [z][y][x], decoded to physical units (any of them may be NULL).
 * Errors: HZ_E_INVALID, HZ_E_DEVICE. */
hz_status hz_field_read(hz_ctx *ctx, const hz_field *field, float *dn, float *gx, float *gy, float *gz,
                        void *hip_stream);

/* Grid and storage type of a field. */
hz_status hz_field_info(const hz_field *field, hz_grid *grid, hz_dtype *dtype, float *store_scale,
                        uint64_t *bytes);

/* Release a field.  Does not block: the field's memory returns to the
 * context's pool and is reused (by a later field of the same size) only by
 * work ordered after every launch already queued that reads the field.
 * Pooled memory stays charged to the budget until the context needs the room
 * or is destroyed.  Errors: HZ_E_INVALID (NULL arguments, unknown field, or a
 * request still waiting in the serving loop reads the field). */
hz_status hz_field_release(hz_ctx *ctx, hz_field *field);

/* ---------------------------------------------------------------------- */
/* Curved-ray tracing (paper Sec. 3.3.2-3.3.3, Eqs. 15-18)                */
/* ---------------------------------------------------------------------- */

/* Pinhole camera with a backdrop plane.  fwd is the viewing direction, up
 * fixes the roll (right = normalize(fwd x up)), vfov is the vertical field of
 * view; pixel (p, q) has q = 0 at the top.  The backdrop is the plane through
 * plane_p with unit normal plane_n facing the camera. */
typedef struct {
    float eye[3], fwd[3], up[3];
    float vfov;
    int32_t width, height;
    float plane_p[3], plane_n[3];
} hz_view;

/* Step control.  uniform != 0 selects the fixed step ds_uniform; otherwise
 * ds = clamp(n theta_max / (|(I - w w^T) g| + eps), ds_min, ds_max).  A step
 * never runs past the volume: it is shortened to the exit distance along the
 * current direction, and the march ends when that distance is <= tau_term or
 * the new position is outside the volume, or after max_steps steps. */
typedef struct {
    int32_t uniform;
    float theta_max, ds_min, ds_max, eps, ds_uniform;
    int32_t max_steps;
    float tau_term;
} hz_step;

/* Per-ray outputs, device arrays with one entry per traced ray:
 *   disp      2 floats: displacement (px) of the scene point seen through the
 *             volume from where the straight ray would see it, (+x right,
 *             +y down); NaN when status is HZ_RAY_NOHIT
 *   exit_pos  3 floats: where the ray leaves the volume (the eye for rays that
 *             miss the volume)
 *   exit_dir  3 floats: unit direction there
 *   steps     number of update steps taken inside the volume
 *   status    HZ_RAY_* code
 * Any pointer may be NULL to skip that output. */
typedef struct {
    float *disp;
    float *exit_pos;
    float *exit_dir;
    uint32_t *steps;
    uint8_t *status;
} hz_trace_out;

/* Trace views[0..nviews) through `field` in one launch whose persistent waves
 * share one queue of the rays of every view.  Rays are numbered by
 * concatenating the views in order, each view row-major (ray id =
 * offset_of_view + q * width + p).  If ray_ids (device, int64) is NULL all
 * rays are traced and output i belongs to ray id i (nrays must equal the total
 * pixel count); otherwise output i belongs to ray id ray_ids[i] for i <
 * nrays.  `views` and `step` are host memory.  Results are bitwise identical
 * across calls and launch shapes.
 * Errors: HZ_E_INVALID (null ctx/field/views/step/out, nviews < 1 or > 4096,
 * width/height < 1, vfov outside (0, pi), zero fwd or fwd parallel to up,
 * zero plane_n, ds_min <= 0, ds_max < ds_min, theta_max <= 0, eps < 0,
 * ds_uniform <= 0 with uniform set, max_steps < 1, tau_term < 0, nrays
 * mismatch, more than 2^31 - 1 rays), HZ_E_BUDGET, HZ_E_NOMEM, HZ_E_DEVICE. */
hz_status hz_trace_views(hz_ctx *ctx, const hz_field *field, const hz_view *views, int32_t nviews,
                         const hz_step *step, const int64_t *ray_ids, int64_t nrays, const hz_trace_out *out,
                         void *hip_stream);

/* hz_trace_views for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results (bitwise equal to hz_trace_views), but the
 * launch scratch (ray counters, view table, hit list, length bins) lives in
 * one static device array of the library, about 40 MiB, that each GPU the
 * library runs on holds until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine; the view table
 * reaches the device in kernel arguments).  Limits: at most 64 views and
 * 2^23 queue slots (each view is padded to 8 x 8 pixel tiles; with ray_ids,
 * nrays slots); beyond them it returns HZ_E_UNSUPPORTED without doing
 * anything.  Every call on one GPU shares that GPU's array, and the array
 * keeps the last call's contents: calls that overlap on one GPU (on two
 * streams, or from two contexts) race and give wrong results, so order them.
 * Arguments, outputs and other errors as hz_trace_views. */
hz_status hz_trace_views_noalloc(hz_ctx *ctx, const hz_field *field, const hz_view *views, int32_t nviews,
                                 const hz_step *step, const int64_t *ray_ids, int64_t nrays,
                                 const hz_trace_out *out, void *hip_stream);

/* Scene boards (paper Sec. 3.3.2: the image is formed where the bent ray meets
 * the scene; Sec. 4.2: boards at two depths, or one slanted board, viewed
 * through the volume).  A board is the parallelogram
 *     origin + u edge_u + v edge_v,  0 <= u, v <= 1,
 * in metres, seen from either side. */
#define HZ_MAX_QUADS 8
typedef struct {
    float origin[3];
    float edge_u[3];
    float edge_v[3];
} hz_quad;

/* Up to HZ_MAX_QUADS boards shared by all views of a call; host memory, read
 * during the call only. */
typedef struct {
    int32_t nquads;
    const hz_quad *quads;
} hz_scene;

/* hz_trace_views with scene boards.  A board can be met anywhere along a ray:
 * before the volume (straight ray from the eye), inside it (the straight chord
 * C_k -> C_{k+1} of each update step of Eq. 16 is tested, and the first board
 * crossed ends the ray at the crossing point), or after it (the straight exit
 * ray is cast against the boards and the view's backdrop plane, and the
 * nearest wins; boards win ties).  Outputs as hz_trace_views, except:
 *   exit_pos, exit_dir  for a ray that met a board inside the volume: the
 *                       crossing point and the direction omega_{k+1} of that
 *                       step; for a board met before the volume: the eye and
 *                       the pixel direction (steps = 0)
 *   disp                displacement of the board point the ray met
 *   surface (device, uint8, one per output; may be NULL): 0 backdrop plane,
 *                       k + 1 board k, 255 nothing met (HZ_RAY_NOHIT,
 *                       HZ_RAY_NONFINITE, HZ_RAY_BAD_ID)
 * `scene` may be NULL or hold 0 boards, which is hz_trace_views plus the
 * surface output.  Errors: as hz_trace_views, and HZ_E_INVALID for nquads
 * outside [0, HZ_MAX_QUADS], a NULL quads pointer with nquads > 0, non-finite
 * board values or edges that are zero or parallel. */
hz_status hz_trace_scene(hz_ctx *ctx, const hz_field *field, const hz_view *views, int32_t nviews,
                         const hz_scene *scene, const hz_step *step, const int64_t *ray_ids, int64_t nrays,
                         const hz_trace_out *out, uint8_t *surface, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Triangle-mesh scenes with a conservative shell (paper Sec. 4.1)        */
/* ---------------------------------------------------------------------- */

/* A scene triangle, seen from either side; `surface` (0..253) names the part
 * of the scene it belongs to, and a ray that meets it reports surface + 1. */
typedef struct {
    float v0[3], v1[3], v2[3];
    int32_t surface;
} hz_triangle;

/* reach: the longest march step the shell must serve, in metres: a trace
 *   whose largest step (ds_max, or ds_uniform for the fixed step) exceeds it
 *   is refused.
 * cell: edge of the shell's grid cells in metres; 0 = 4 x reach.  Coarsened
 *   by factors of 1.25 until the grid has at most 512 cells per axis and
 *   2^22 cells.
 * brute_force: 1 = no shell: every chord and straight segment is tested
 *   against every triangle (same results, for comparison). */
typedef struct {
    float reach;
    float cell;
    int32_t brute_force;
} hz_mesh_params;

typedef struct hz_mesh hz_mesh;   /* device-resident triangles and their shell */

/* Build a mesh scene from ntris host triangles (1..65536) and precompute its
 * conservative shell (paper Sec. 4.1): a coarse grid over the mesh's box
 * grown by reach + one cell, holding per cell a lower bound of the distance
 * from any point of the cell to the mesh, and the triangles within reach of
 * the cell.  During the march, a step starting in a cell whose bound exceeds
 * the step cannot meet the mesh and takes no exact test; otherwise the
 * step's chord is tested against the cell's triangles.  Straight parts of the
 * ray (before the volume, rays that miss it, the exit ray) walk the cells
 * they cross.  Built on the device in two passes over all triangles per cell
 * (cost cells x triangles); synchronises hip_stream.
 * Errors: HZ_E_INVALID (NULL arguments, ntris out of range, non-finite or
 * degenerate triangles, surface outside [0, 253], reach <= 0, cell < 0),
 * HZ_E_UNSUPPORTED (lists too long), HZ_E_BUDGET, HZ_E_NOMEM, HZ_E_DEVICE. */
hz_status hz_mesh_create(hz_ctx *ctx, const hz_triangle *tris, int32_t ntris, const hz_mesh_params *params,
                         void *hip_stream, hz_mesh **out);

/* Triangles, shell grid size and cell, total length of the shell's lists,
 * and device bytes of a mesh (any pointer may be NULL). */
hz_status hz_mesh_info(const hz_mesh *mesh, int32_t *ntris, int32_t shell_res[3], float *shell_cell,
                       int64_t *list_entries, uint64_t *bytes);

/* Release a mesh; waits for the traces that use it.  Errors: HZ_E_INVALID
 * (NULL arguments, a mesh of another context, or a request still waiting in
 * the serving loop reads the mesh). */
hz_status hz_mesh_release(hz_ctx *ctx, hz_mesh *mesh);

/* hz_trace_scene with a triangle mesh instead of boards.  The first triangle
 * met ends the ray: met before the volume (straight ray from the eye), on the
 * chord C_k -> C_{k+1} of a step of Eq. 16 inside it (first crossing along the
 * chord; equal crossings go to the lower triangle index), or after it (the
 * straight exit ray against the mesh and the view's backdrop plane; the mesh
 * wins ties).  Outputs as hz_trace_scene (surface: 0 backdrop, s + 1 a
 * triangle of surface s, 255 nothing met), plus, if tri_tests (device, one
 * uint32 per output) is not NULL, the number of exact ray-triangle tests each
 * ray took.  Errors: as hz_trace_views, and HZ_E_INVALID for a NULL mesh, a
 * mesh of another context, or steps longer than the mesh's reach. */
hz_status hz_trace_mesh(hz_ctx *ctx, const hz_field *field, const hz_view *views, int32_t nviews,
                        const hz_mesh *mesh, const hz_step *step, const int64_t *ray_ids, int64_t nrays,
                        const hz_trace_out *out, uint8_t *surface, uint32_t *tri_tests, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Measurement: achievable bandwidth of the memory levels the tracer uses   */
/* ---------------------------------------------------------------------- */

/* Achievable read bandwidth (GB/s) of a device buffer of `bytes` read `reps`
 * times by a plain streaming kernel: buffers far above the 256 MB MALL measure
 * HBM, field-sized ones measure the caches that serve the tracer.  Allocates
 * (and frees) the buffer against the budget; synchronises `hip_stream`.
 * Errors: HZ_E_INVALID (bytes < 4096, reps outside [1, 10000]), HZ_E_BUDGET,
 * HZ_E_NOMEM, HZ_E_DEVICE. */
hz_status hz_membench(hz_ctx *ctx, uint64_t bytes, int32_t reps, double *read_gbps, void *hip_stream);

/* Achievable gather bandwidth (GB/s) of the tracer's access pattern with no
 * arithmetic around it, replaying the tracer's own rays: every pixel of
 * views[0..nviews) casts the pinhole ray hz_trace_views casts (one thread per
 * pixel, 8 x 8 pixel tiles per wave, view after view) and, if the ray enters
 * the box of `grid`, walks straight through it in steps of step_len metres
 * from the entry point, reading at every sample the 8 corner voxels of its
 * cell the way the marcher does.  The grid holds voxel_bytes-byte voxels (16
 * as F32 fields, 8 as F16/BF16 ones).  Counted as samples x 8 x voxel_bytes
 * per launch (*samples, may be NULL, gets the samples per launch); one
 * warm-up launch, then `reps` timed ones.  Allocates (and frees) the grid
 * against the budget; synchronises hip_stream.
 * Errors: HZ_E_INVALID (NULL grid/views/gather_gbps, voxel_bytes not 8 or 16,
 * res outside [2, 65535] or a grid of 2^31 voxels or more, bad views, nviews
 * outside [1, 4096], step_len outside [1e-3, 1e3] voxels, reps outside
 * [1, 10000]; after the run: no ray enters the grid), HZ_E_BUDGET,
 * HZ_E_NOMEM, HZ_E_DEVICE. */
hz_status hz_membench_gather(hz_ctx *ctx, const hz_grid *grid, int32_t voxel_bytes, const hz_view *views,
                             int32_t nviews, float step_len, int32_t reps, double *gather_gbps, int64_t *samples,
                             void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of multi-view requests                   */
/* ---------------------------------------------------------------------- */
/* The paper defines no serving interface.  What it fixes is the use: every
 * camera renders through the same time-varying 3D volume, so views of one
 * frame are consistent by construction (Sec. 1; multi-view results, Sec. 4.2),
 * at interactive frame rates (abstract; Sec. 4.1).  The request, batching,
 * admission and release semantics below are this library's own design for
 * that use: requests for fields of one grid and storage type are traced in
 * shared launches, and each request's result is the one hz_trace_views gives
 * for it alone. */

typedef uint64_t hz_ticket;

/* Start the context's serving loop: at most `slots` launches in flight at
 * once (each on its own stream), each batching up to `max_batch_rays` rays of
 * whole requests.  Requests are admitted while their output buffers and the
 * launch scratch fit the HBM budget.  Errors: HZ_E_INVALID (slots < 1 or >
 * 16, max_batch_rays < 1), HZ_E_BUDGET, HZ_E_NOMEM, HZ_E_DEVICE. */
hz_status hz_server_start(hz_ctx *ctx, int32_t slots, int64_t max_batch_rays);

/* Submit a request: trace all pixels of views[0..nviews) through `field` with
 * `step`.  Non-blocking; views and step are copied.  The library allocates
 * the request's outputs (see hz_request_outputs).  hz_field_release refuses
 * `field` while the request waits to be launched; once it is launched, a
 * release of the field defers its reuse past the request's work.  Requests that arrive while others run join
 * the next launch whose slot and memory are free; requests for different
 * fields of the same grid and storage type share launches.
 * Errors: HZ_E_INVALID (as hz_trace_views, or no server), HZ_E_BUDGET (the
 * request alone exceeds the budget or a batch). */
hz_status hz_submit(hz_ctx *ctx, const hz_field *field, const hz_view *views, int32_t nviews,
                    const hz_step *step, hz_ticket *out);

/* hz_submit with scene boards (as hz_trace_scene; `scene` is copied).  Only
 * requests with the same boards (and grid, storage type and step control)
 * share a launch.  Errors: as hz_submit, and as hz_trace_scene for the
 * boards. */
hz_status hz_submit_scene(hz_ctx *ctx, const hz_field *field, const hz_view *views, int32_t nviews,
                          const hz_scene *scene, const hz_step *step, hz_ticket *out);

/* hz_submit with a triangle mesh (as hz_trace_mesh, without tri_tests; the
 * request's surface array reports the mesh surfaces).  hz_mesh_release refuses
 * `mesh` while the request waits to be launched, and waits for its work once
 * it is launched.  Only requests with the same mesh (and grid,
 * storage type and step control) share a launch.  Errors: as hz_submit, and
 * HZ_E_INVALID for a NULL mesh, a mesh of another context, or steps longer
 * than the mesh's reach. */
hz_status hz_submit_mesh(hz_ctx *ctx, const hz_field *field, const hz_view *views, int32_t nviews,
                         const hz_mesh *mesh, const hz_step *step, hz_ticket *out);

/* Poll a request: HZ_PENDING until its results are complete on the device,
 * then HZ_OK with *latency_s = seconds from submit to completion (may be
 * NULL).  Errors: HZ_E_NOTFOUND (unknown or already released ticket),
 * HZ_E_DEVICE. */
hz_status hz_poll(hz_ctx *ctx, hz_ticket ticket, double *latency_s);

/* Device output arrays of a completed request (layout as hz_trace_views with
 * ray_ids == NULL); valid until hz_request_release.  *nrays gets the number
 * of rays.  Errors: HZ_E_NOTFOUND, HZ_E_INVALID (not complete yet). */
hz_status hz_request_outputs(hz_ctx *ctx, hz_ticket ticket, hz_trace_out *out, int64_t *nrays);

/* Device array (uint8, one per ray) of the surface each ray of a completed
 * request met, as hz_trace_scene's `surface` (0 backdrop, k + 1 board k, 255
 * nothing); valid until hz_request_release.  Errors: HZ_E_NOTFOUND,
 * HZ_E_INVALID (not complete). */
hz_status hz_request_surface(hz_ctx *ctx, hz_ticket ticket, uint8_t **surface);

/* Device timestamps (milliseconds from the server's start, on the GPU's own
 * clock) of the first and last kernel of the launch that carried a completed
 * request; requests batched together share them, and launches on different
 * slots may overlap.  Errors: HZ_E_NOTFOUND, HZ_E_INVALID (not complete). */
hz_status hz_request_timing(hz_ctx *ctx, hz_ticket ticket, double *device_start_ms, double *device_end_ms);

/* Release a completed (or still pending) request and forget its ticket.  Its
 * output memory goes back to the server's pool and is reused by later
 * requests, so every read of the outputs (including device work queued on
 * other streams) must have completed first.  Never blocks on the device. */
hz_status hz_request_release(hz_ctx *ctx, hz_ticket ticket);

/* Stop the serving loop after the requests already admitted have finished;
 * pending requests are completed first. */
hz_status hz_server_stop(hz_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* HAZE_H */
