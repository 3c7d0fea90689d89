// serve.hip -- serving loop: continuous batching of multi-view trace requests.
//
// hz_submit enqueues a request (views of one field, one step control) and
// returns at once.  A scheduler thread owns `slots` launch slots, each with
// its own HIP stream, job table, hit list and counters.  Whenever a slot is
// free it takes the oldest pending request and every later pending request
// that can share its launch (same grid, storage type and step control; the
// fields may differ, e.g. different frames), as long as the batch fits the
// slot and the requests' output buffers fit the context's HBM budget; the
// batch is traced by one persistent launch (ray generation + march, the same
// kernels as hz_trace_views).  Requests arriving while others run are
// admitted as soon as a slot and memory free up, and launches on different
// slots overlap on the device.  A request's rays are computed exactly as in a
// solo hz_trace_views call, whatever else shares the launch.
//
// Nothing on the serving path frees device memory or waits for the device
// while holding the server lock: request outputs come from a pool of
// size-classed blocks that released requests return to (a released request's
// batch has completed), and blocks that must go (budget pressure, a slot's
// grown view table) are freed by the scheduler with the lock dropped.
#include "haze_device.h"
#include "serve.h"
#include "serve_policy.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace haze {
hipError_t launch_raygen(const TraceLaunch &, bool, hipStream_t, const KTimer &);
hipError_t launch_march(int, const TraceLaunch &, int, hipStream_t, const KTimer &);
hz_status check_step(const hz_step *st, const char *fn);
hz_status build_scene(const hz_scene *scene, const hz_grid &g, TraceLaunch *L, std::vector<SceneQuad> &qs,
                      const char *fn);
hz_status make_job(const hz_view *v, const void *field, int64_t slot_begin, int64_t ray_begin, TraceJob *J,
                   const char *fn, int index);
void make_trace_grid(const hz_grid &g, float store_scale, TraceGrid *G);
float length_bin_scale(const hz_grid &g);
void make_trace_step(const hz_step &st, const hz_grid &g, TraceStep *S);

enum ReqState { REQ_PENDING = 0, REQ_RUNNING = 1, REQ_DONE = 2, REQ_FAILED = 3 };

struct Request {
    hz_ticket id = 0;
    hz_field *field = nullptr;
    std::vector<hz_view> views;
    std::vector<hz_quad> quads;   // scene boards (none: the backdrop only)
    hz_mesh *mesh = nullptr;      // or a triangle-mesh scene
    hz_step step{};
    BatchKey key = zero_key();
    int64_t nrays = 0, nslots = 0, out_bytes = 0;
    void *out_mem = nullptr;
    size_t out_cap = 0;         // size class of out_mem
    hz_trace_out out{};
    uint8_t *surface = nullptr;  // surface each ray met (after status in out_mem)
    double t_submit = 0.0, t_done = 0.0;
    double dev_start_ms = 0.0, dev_end_ms = 0.0;   // its launch on the device, from the server's reference
    int state = REQ_PENDING;
    hz_status err = HZ_OK;
};

// A device block held by the server for reuse (request outputs) or to be
// freed with the lock dropped.
using Block = PoolBlock;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t t_start = nullptr, t_stop = nullptr;   // dispatch timestamps of the batch's first and last kernel
    bool busy = false;
    std::vector<Request *> reqs;
    void *jobs = nullptr;       // device job table
    size_t jobs_cap = 0;
    void *pinned = nullptr;     // host staging of the job table
    size_t pinned_cap = 0;
    void *hits = nullptr;       // u32 per queue slot
    void *bins = nullptr;       // u8 per queue slot (length bins of the ray sort)
    void *counters = nullptr;      // two counter sets, used alternately
    int counter_set = 0;
    bool counters_clean = false;   // the set in turn is zero
    size_t scratch_bytes = 0;
};

struct Server {
    hz_ctx *ctx = nullptr;
    int64_t slot_capacity = 0;  // queue slots per launch
    std::vector<Slot> slots;
    std::deque<Request *> pending;
    std::unordered_map<hz_ticket, Request *> reqs;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    hz_ticket next_id = 1;
    hz_status fatal = HZ_OK;
    hipEvent_t t_ref = nullptr;        // device time origin of the batch timestamps
    OutputPool out_pool;               // released request outputs, by size class
    std::vector<Block> to_free;        // device blocks the scheduler frees unlocked
    std::vector<void *> to_free_host;  // pinned host blocks likewise
    size_t trim_fields = 0;            // bytes of pooled (released) field memory to give back, unlocked
};

// Whether a request still waiting in the serving loop (not yet launched: a
// launched one has left its completion mark on the field and the mesh) reads
// field f or mesh m.
bool server_waiting_use(hz_ctx *c, const hz_field *f, const hz_mesh *m)
{
    Server *S = ctx_server(c);
    if (!S) return false;
    std::lock_guard<std::mutex> g(S->mu);
    for (const Request *r : S->pending)
        if ((f && r->field == f) || (m && r->mesh == m)) return true;
    return false;
}

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static BatchKey make_key(const hz_field *f, const hz_step &st, const std::vector<hz_quad> &quads, const hz_mesh *mesh)
{
    BatchKey k = zero_key();
    const hz_grid &g = field_grid(f);
    for (int a = 0; a < 3; ++a) {
        k.lo[a] = g.lo[a];
        k.hi[a] = g.hi[a];
        k.res[a] = g.res[a];
    }
    k.dtype = (int32_t)field_dtype(f);
    k.store_scale = field_scale(f);
    k.uniform = st.uniform ? 1 : 0;
    k.theta_max = st.theta_max;
    k.ds_min = st.ds_min;
    k.ds_max = st.ds_max;
    k.eps = st.eps;
    k.ds_uniform = st.ds_uniform;
    k.max_steps = st.max_steps;
    k.tau_term = st.tau_term;
    k.nquads = (int32_t)quads.size();
    k.mesh = (uint64_t)(uintptr_t)mesh;
    for (size_t q = 0; q < quads.size(); ++q)
        for (int a = 0; a < 3; ++a) {
            k.quads[q][a] = quads[q].origin[a];
            k.quads[q][3 + a] = quads[q].edge_u[a];
            k.quads[q][6 + a] = quads[q].edge_v[a];
        }
    return k;
}

// Return a request's outputs to the pool (its batch has completed; the caller
// has finished reading them).  Called with the server lock held.
static void pool_outputs(Server *S, Request *r)
{
    if (r->out_mem) S->out_pool.put(r->out_mem, r->out_cap);
    r->out_mem = nullptr;
    r->out_cap = 0;
}

// A request's outputs: one block of its size class, from the pool or newly
// allocated (never by giving back other memory: that waits for the device).
// Called with the server lock held.
static hz_status alloc_outputs(Server *S, Request *r)
{
    const size_t cls = out_class(r->out_bytes);
    r->out_mem = S->out_pool.take(cls);
    if (!r->out_mem) {
        hz_status st = ctx_alloc_nowait(S->ctx, &r->out_mem, cls);
        if (st != HZ_OK) return st;
    }
    r->out_cap = cls;
    char *base = (char *)r->out_mem;
    const int64_t n = r->nrays;
    r->out.disp = (float *)base;
    r->out.exit_pos = (float *)(base + 8 * n);
    r->out.exit_dir = (float *)(base + 20 * n);
    r->out.steps = (uint32_t *)(base + 32 * n);
    r->out.status = (uint8_t *)(base + 36 * n);
    r->surface = (uint8_t *)(base + 37 * n);
    return HZ_OK;
}

// Launch one batch on a free slot; called with the server lock held.
static hz_status launch_batch(Server *S, Slot &sl, std::vector<Request *> &batch)
{
    std::vector<TraceJob> jobs;
    int64_t slot = 0, ray = 0;
    for (Request *r : batch) {
        int64_t local_ray = 0;
        for (size_t i = 0; i < r->views.size(); ++i) {
            TraceJob J;
            hz_status st = make_job(&r->views[i], field_data(r->field), slot, ray, &J, "serve", (int)i);
            if (st != HZ_OK) return st;
            J.disp = r->out.disp + 2 * local_ray;
            J.exit_pos = r->out.exit_pos + 3 * local_ray;
            J.exit_dir = r->out.exit_dir + 3 * local_ray;
            J.steps = r->out.steps + local_ray;
            J.status = r->out.status + local_ray;
            J.surface = r->surface + local_ray;
            jobs.push_back(J);
            const int64_t nr = (int64_t)r->views[i].width * r->views[i].height;
            slot += view_slots(r->views[i].width, r->views[i].height);
            ray += nr;
            local_ray += nr;
        }
    }
    // the batch's boards (all its requests share them: same key) after the
    // views, or its mesh
    Request *head = batch[0];
    TraceLaunch L{};
    std::vector<SceneQuad> qs;
    if (!head->quads.empty()) {
        hz_scene sc{(int32_t)head->quads.size(), head->quads.data()};
        hz_status st = build_scene(&sc, field_grid(head->field), &L, qs, "serve");
        if (st != HZ_OK) return st;
    }
    if (head->mesh) L.mesh = mesh_launch(head->mesh);
    const size_t view_bytes = sizeof(TraceJob) * jobs.size();
    const size_t job_bytes = view_bytes + sizeof(SceneQuad) * qs.size();
    if (sl.jobs_cap < job_bytes) {
        // the slot is idle, so its old table is no longer read; it is freed
        // later with the lock dropped
        const size_t want = std::max(job_bytes, 2 * sl.jobs_cap);
        void *p = nullptr;
        hz_status st = ctx_alloc_nowait(S->ctx, &p, want);
        if (st != HZ_OK) return st;
        if (sl.jobs) S->to_free.push_back({sl.jobs, sl.jobs_cap});
        sl.jobs = p;
        sl.jobs_cap = want;
    }
    if (sl.pinned_cap < job_bytes) {
        const size_t want = std::max(job_bytes, 2 * sl.pinned_cap);
        void *p = nullptr;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess)
            return set_error(HZ_E_NOMEM, "serve: hipHostMalloc failed");
        if (sl.pinned) S->to_free_host.push_back(sl.pinned);
        sl.pinned = p;
        sl.pinned_cap = want;
    }
    for (Request *r : batch) {
        hz_status st = field_ready(r->field, sl.stream);
        if (st != HZ_OK) return st;
    }
    // the slot is idle, so its previous copy out of `pinned` has completed
    std::memcpy(sl.pinned, jobs.data(), view_bytes);
    if (!qs.empty()) std::memcpy((char *)sl.pinned + view_bytes, qs.data(), sizeof(SceneQuad) * qs.size());
    if (hipMemcpyAsync(sl.jobs, sl.pinned, job_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
        return set_error(HZ_E_DEVICE, "serve: hipMemcpyAsync failed");

    L.jobs = (const TraceJob *)sl.jobs;
    L.quads = qs.empty() ? nullptr : (const SceneQuad *)((const char *)sl.jobs + view_bytes);
    L.njobs = (int32_t)jobs.size();
    L.subset = 0;
    L.nslots = slot;
    L.ray_ids = nullptr;
    L.hits = (uint32_t *)sl.hits;
    L.counters = (uint32_t *)sl.counters + (size_t)sl.counter_set * kCounterSetWords;
    L.counters_next = (uint32_t *)sl.counters + (size_t)(1 - sl.counter_set) * kCounterSetWords;
    L.slot_bin = (uint8_t *)sl.bins;
    L.inv_len_bin = length_bin_scale(field_grid(head->field));
    make_trace_grid(field_grid(head->field), field_scale(head->field), &L.grid);
    make_trace_step(head->step, field_grid(head->field), &L.step);
    L.refill_min = 64;
    const int dt = (int)field_dtype(head->field);
    const int mode = L.mesh.ntris > 0 ? 3 : L.ninner > 0 ? 2 : L.nquads > 0 ? 1 : 0;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((slot + 255) / 256, march_blocks(S->ctx, dt, mode)));
    const bool clear = !sl.counters_clean;
    sl.counters_clean = false;
    // the dispatch packets of the first and last kernel record the batch's
    // device start and end (no extra packets)
    if (launch_raygen(L, clear, sl.stream, KTimer{sl.t_start, nullptr}) != hipSuccess ||
        launch_march(dt, L, blocks, sl.stream, KTimer{nullptr, sl.t_stop}) != hipSuccess)
        return set_error(HZ_E_DEVICE, "serve: trace launch failed");
    sl.counter_set = 1 - sl.counter_set;
    sl.counters_clean = true;
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return set_error(HZ_E_DEVICE, "serve: hipEventRecord");
    CallMark done;
    hz_status st = ctx_mark(S->ctx, sl.stream, &done);
    if (st != HZ_OK) return st;
    for (Request *r : batch) {
        field_use(r->field, done);
        r->state = REQ_RUNNING;
    }
    if (head->mesh) mesh_use(head->mesh, done);
    sl.reqs = batch;
    sl.busy = true;
    return HZ_OK;
}

// Free the blocks queued for freeing, with the server lock dropped (freeing
// device memory waits for the device).
static void free_deferred(Server *S, std::unique_lock<std::mutex> &lk)
{
    if (S->to_free.empty() && S->to_free_host.empty() && !S->trim_fields) return;
    std::vector<Block> dev;
    std::vector<void *> host;
    dev.swap(S->to_free);
    host.swap(S->to_free_host);
    const size_t trim = S->trim_fields;
    S->trim_fields = 0;
    lk.unlock();
    for (const Block &b : dev) ctx_free(S->ctx, b.ptr, b.bytes);
    for (void *h : host) (void)hipHostFree(h);
    if (trim) ctx_trim_pool(S->ctx, trim);
    lk.lock();
}

static void scheduler(Server *S)
{
    (void)hipSetDevice(ctx_device(S->ctx));
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progressed = false, any_busy = false;
        for (Slot &sl : S->slots) {
            if (!sl.busy) continue;
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipSuccess || e != hipErrorNotReady) {
                const double t = now_s();
                float ms0 = 0.0f, ms1 = 0.0f;
                if (e == hipSuccess && hipEventElapsedTime(&ms0, S->t_ref, sl.t_start) == hipSuccess &&
                    hipEventElapsedTime(&ms1, S->t_ref, sl.t_stop) == hipSuccess)
                    profile_add(S->ctx, "serve_batch", (double)(ms1 - ms0));
                for (Request *r : sl.reqs) {
                    r->t_done = t;
                    r->dev_start_ms = ms0;
                    r->dev_end_ms = ms1;
                    r->state = e == hipSuccess ? REQ_DONE : REQ_FAILED;
                    if (e != hipSuccess) r->err = HZ_E_DEVICE;
                }
                sl.reqs.clear();
                sl.busy = false;
                progressed = true;
            } else {
                any_busy = true;
            }
        }
        for (Slot &sl : S->slots) {
            if (sl.busy || S->pending.empty()) continue;
            std::vector<PendingInfo> info;
            const size_t window = std::min<size_t>(S->pending.size(), 256);
            for (size_t i = 0; i < window; ++i)
                info.push_back({S->pending[i]->key, S->pending[i]->nslots, (int64_t)out_class(S->pending[i]->out_bytes)});
            // pooled output blocks count as free memory: they are reused, or
            // given back when an allocation finds the budget short
            const std::vector<size_t> pick =
                plan_batch(info, S->slot_capacity, (int64_t)(ctx_mem_avail(S->ctx) + S->out_pool.bytes), 256);
            if (pick.empty()) {
                // the oldest request waits for memory; when stopping with nothing
                // running, no memory will come back: fail what is left
                if (S->stop && !any_busy) {
                    for (Request *r : S->pending) {
                        r->state = REQ_FAILED;
                        r->err = HZ_E_BUDGET;
                        r->t_done = now_s();
                    }
                    S->pending.clear();
                }
                break;
            }
            std::vector<Request *> batch;
            bool short_mem = false;
            for (size_t i : pick) {
                Request *r = S->pending[i];
                if (alloc_outputs(S, r) != HZ_OK) {   // memory went away: launch what we have
                    short_mem = true;
                    break;
                }
                batch.push_back(r);
            }
            if (short_mem) {
                // pooled output blocks of other sizes, or released fields,
                // hold the budget: give them back (below, unlocked); the rest
                // waits for the next round
                const std::vector<Block> held = S->out_pool.drain();
                S->to_free.insert(S->to_free.end(), held.begin(), held.end());
                S->trim_fields = (size_t)out_class(S->pending[pick[batch.size()]]->out_bytes);
                progressed = progressed || !S->to_free.empty();
            }
            if (batch.empty()) break;
            // remove the launched requests from the pending queue (keep order of the rest)
            std::deque<Request *> rest;
            for (Request *r : S->pending)
                if (std::find(batch.begin(), batch.end(), r) == batch.end()) rest.push_back(r);
            S->pending.swap(rest);
            const hz_status st = launch_batch(S, sl, batch);
            if (st != HZ_OK) {
                for (Request *r : batch) {
                    r->state = REQ_FAILED;
                    r->err = st;
                    r->t_done = now_s();
                }
            } else {
                any_busy = true;
            }
            progressed = true;
        }
        free_deferred(S, lk);
        if (S->stop && S->pending.empty() && !any_busy) break;
        if (!progressed) S->cv.wait_for(lk, any_busy ? std::chrono::microseconds(20) : std::chrono::milliseconds(2));
    }
}

void server_destroy(Server *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    for (Slot &sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.jobs) ctx_free(S->ctx, sl.jobs, sl.jobs_cap);
        if (sl.hits) ctx_free(S->ctx, sl.hits, sl.scratch_bytes);
        if (sl.bins) ctx_free(S->ctx, sl.bins, (size_t)S->slot_capacity);
        if (sl.counters) ctx_free(S->ctx, sl.counters, kCounterBytes);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.t_start) (void)hipEventDestroy(sl.t_start);
        if (sl.t_stop) (void)hipEventDestroy(sl.t_stop);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto &kv : S->reqs) {
        pool_outputs(S, kv.second);
        delete kv.second;
    }
    for (const Block &b : S->out_pool.drain()) ctx_free(S->ctx, b.ptr, b.bytes);
    for (const Block &b : S->to_free) ctx_free(S->ctx, b.ptr, b.bytes);
    for (void *h : S->to_free_host) (void)hipHostFree(h);
    if (S->t_ref) (void)hipEventDestroy(S->t_ref);
    delete S;
}

}  // namespace haze

using namespace haze;

extern "C" hz_status hz_server_start(hz_ctx *c, int32_t nslots, int64_t max_batch_rays)
{
    if (!c) return set_error(HZ_E_INVALID, "hz_server_start: ctx is NULL");
    if (nslots < 1 || nslots > 16) return set_error(HZ_E_INVALID, "hz_server_start: slots must be in [1, 16]");
    if (max_batch_rays < 1 || max_batch_rays > INT32_MAX / 2)
        return set_error(HZ_E_INVALID, "hz_server_start: max_batch_rays must be in [1, 2^30]");
    if (ctx_server(c)) return set_error(HZ_E_INVALID, "hz_server_start: the server is already running");
    if (hipSetDevice(ctx_device(c)) != hipSuccess) return set_error(HZ_E_DEVICE, "hz_server_start: hipSetDevice");
    Server *S = new Server();
    S->ctx = c;
    S->slot_capacity = (max_batch_rays + 63) / 64 * 64;
    S->slots.resize((size_t)nslots);
    for (Slot &sl : S->slots) {
        sl.scratch_bytes = 4u * (size_t)S->slot_capacity;
        hz_status st = ctx_alloc(c, &sl.hits, sl.scratch_bytes);
        if (st == HZ_OK) st = ctx_alloc(c, &sl.bins, (size_t)S->slot_capacity);
        if (st == HZ_OK) st = ctx_alloc(c, &sl.counters, kCounterBytes);
        if (st == HZ_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
            st = set_error(HZ_E_DEVICE, "hz_server_start: hipStreamCreate failed");
        if (st == HZ_OK && (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
                            hipEventCreate(&sl.t_start) != hipSuccess || hipEventCreate(&sl.t_stop) != hipSuccess))
            st = set_error(HZ_E_DEVICE, "hz_server_start: hipEventCreate failed");
        if (st != HZ_OK) {
            server_destroy(S);
            return st;
        }
    }
    if (hipEventCreate(&S->t_ref) != hipSuccess || hipEventRecord(S->t_ref, S->slots[0].stream) != hipSuccess ||
        hipEventSynchronize(S->t_ref) != hipSuccess) {
        server_destroy(S);
        return set_error(HZ_E_DEVICE, "hz_server_start: reference event failed");
    }
    ctx_server(c) = S;
    S->th = std::thread(scheduler, S);
    return HZ_OK;
}

extern "C" hz_status hz_server_stop(hz_ctx *c)
{
    if (!c) return set_error(HZ_E_INVALID, "hz_server_stop: ctx is NULL");
    Server *S = ctx_server(c);
    if (!S) return set_error(HZ_E_INVALID, "hz_server_stop: no server running");
    server_destroy(S);
    ctx_server(c) = nullptr;
    return HZ_OK;
}

static hz_status submit_impl(hz_ctx *c, const hz_field *f, const hz_view *views, int32_t nviews,
                             const hz_scene *scene, const hz_mesh *mesh, const hz_step *step, hz_ticket *out,
                             const char *fn)
{
    if (!c || !f || !views || !out) return set_error(HZ_E_INVALID, "hz_submit: NULL argument");
    Server *S = ctx_server(c);
    if (!S) return set_error(HZ_E_INVALID, "hz_submit: no server running (hz_server_start)");
    if (field_ctx(f) != c) return set_error(HZ_E_INVALID, "hz_submit: field belongs to another context");
    if (nviews < 1 || nviews > 4096) return set_error(HZ_E_INVALID, "hz_submit: nviews outside [1, 4096]");
    hz_status st = check_step(step, fn);
    if (st != HZ_OK) return st;
    st = field_usable(c, f, fn);
    if (st != HZ_OK) return st;
    if (mesh) {   // checked now, not at launch
        if (mesh_ctx(mesh) != c) return set_error(HZ_E_INVALID, "hz_submit_mesh: mesh belongs to another context");
        const float longest = step->uniform ? step->ds_uniform : step->ds_max;
        if (longest > mesh_reach(mesh))
            return set_error(HZ_E_INVALID, "hz_submit_mesh: the step is longer than the mesh's shell serves");
    }
    if (scene && scene->nquads > 0) {   // the boards are checked now, not at launch
        TraceLaunch probe{};
        std::vector<SceneQuad> qs;
        st = build_scene(scene, field_grid(f), &probe, qs, fn);
        if (st != HZ_OK) return st;
    }
    Request *r = new Request();
    r->field = const_cast<hz_field *>(f);
    r->views.assign(views, views + nviews);
    if (scene && scene->nquads > 0) r->quads.assign(scene->quads, scene->quads + scene->nquads);
    r->mesh = const_cast<hz_mesh *>(mesh);
    r->step = *step;
    for (int i = 0; i < nviews; ++i) {
        TraceJob J;
        st = make_job(&views[i], field_data(f), 0, 0, &J, fn, i);
        if (st != HZ_OK) {
            delete r;
            return st;
        }
        r->nrays += (int64_t)views[i].width * views[i].height;
        r->nslots += view_slots(views[i].width, views[i].height);
    }
    r->out_bytes = r->nrays * kOutBytesPerRay;
    r->key = make_key(f, *step, r->quads, r->mesh);
    uint64_t budget = 0;
    hz_ctx_memory(c, nullptr, &budget);
    if (r->nslots > S->slot_capacity || (uint64_t)out_class(r->out_bytes) > budget) {
        delete r;
        return set_error(HZ_E_BUDGET, "hz_submit: the request exceeds the batch capacity or the HBM budget");
    }
    {
        std::lock_guard<std::mutex> g(S->mu);
        r->id = S->next_id++;
        r->t_submit = now_s();
        S->reqs[r->id] = r;
        S->pending.push_back(r);
        *out = r->id;
    }
    S->cv.notify_all();
    return HZ_OK;
}

extern "C" hz_status hz_submit(hz_ctx *c, const hz_field *f, const hz_view *views, int32_t nviews,
                               const hz_step *step, hz_ticket *out)
{
    return submit_impl(c, f, views, nviews, nullptr, nullptr, step, out, "hz_submit");
}

extern "C" hz_status hz_submit_scene(hz_ctx *c, const hz_field *f, const hz_view *views, int32_t nviews,
                                     const hz_scene *scene, const hz_step *step, hz_ticket *out)
{
    return submit_impl(c, f, views, nviews, scene, nullptr, step, out, "hz_submit_scene");
}

extern "C" hz_status hz_submit_mesh(hz_ctx *c, const hz_field *f, const hz_view *views, int32_t nviews,
                                    const hz_mesh *mesh, const hz_step *step, hz_ticket *out)
{
    if (!mesh) return set_error(HZ_E_INVALID, "hz_submit_mesh: mesh is NULL");
    return submit_impl(c, f, views, nviews, nullptr, mesh, step, out, "hz_submit_mesh");
}

extern "C" hz_status hz_poll(hz_ctx *c, hz_ticket t, double *latency_s)
{
    if (!c) return set_error(HZ_E_INVALID, "hz_poll: ctx is NULL");
    Server *S = ctx_server(c);
    if (!S) return set_error(HZ_E_INVALID, "hz_poll: no server running");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return set_error(HZ_E_NOTFOUND, "hz_poll: unknown ticket");
    Request *r = it->second;
    if (r->state == REQ_FAILED) return set_error(r->err, "hz_poll: the request failed");
    if (r->state != REQ_DONE) return HZ_PENDING;
    if (latency_s) *latency_s = r->t_done - r->t_submit;
    return HZ_OK;
}

extern "C" hz_status hz_request_outputs(hz_ctx *c, hz_ticket t, hz_trace_out *out, int64_t *nrays)
{
    if (!c || !out) return set_error(HZ_E_INVALID, "hz_request_outputs: NULL argument");
    Server *S = ctx_server(c);
    if (!S) return set_error(HZ_E_INVALID, "hz_request_outputs: no server running");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return set_error(HZ_E_NOTFOUND, "hz_request_outputs: unknown ticket");
    Request *r = it->second;
    if (r->state != REQ_DONE) return set_error(HZ_E_INVALID, "hz_request_outputs: the request is not complete");
    *out = r->out;
    if (nrays) *nrays = r->nrays;
    return HZ_OK;
}

extern "C" hz_status hz_request_surface(hz_ctx *c, hz_ticket t, uint8_t **surface)
{
    if (!c || !surface) return set_error(HZ_E_INVALID, "hz_request_surface: NULL argument");
    Server *S = ctx_server(c);
    if (!S) return set_error(HZ_E_INVALID, "hz_request_surface: no server running");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return set_error(HZ_E_NOTFOUND, "hz_request_surface: unknown ticket");
    if (it->second->state != REQ_DONE)
        return set_error(HZ_E_INVALID, "hz_request_surface: the request is not complete");
    *surface = it->second->surface;
    return HZ_OK;
}

extern "C" hz_status hz_request_timing(hz_ctx *c, hz_ticket t, double *device_start_ms, double *device_end_ms)
{
    if (!c) return set_error(HZ_E_INVALID, "hz_request_timing: ctx is NULL");
    Server *S = ctx_server(c);
    if (!S) return set_error(HZ_E_INVALID, "hz_request_timing: no server running");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return set_error(HZ_E_NOTFOUND, "hz_request_timing: unknown ticket");
    const Request *r = it->second;
    if (r->state != REQ_DONE) return set_error(HZ_E_INVALID, "hz_request_timing: the request is not complete");
    if (device_start_ms) *device_start_ms = r->dev_start_ms;
    if (device_end_ms) *device_end_ms = r->dev_end_ms;
    return HZ_OK;
}

extern "C" hz_status hz_request_release(hz_ctx *c, hz_ticket t)
{
    if (!c) return set_error(HZ_E_INVALID, "hz_request_release: ctx is NULL");
    Server *S = ctx_server(c);
    if (!S) return set_error(HZ_E_INVALID, "hz_request_release: no server running");
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto it = S->reqs.find(t);
        if (it == S->reqs.end()) return set_error(HZ_E_NOTFOUND, "hz_request_release: unknown ticket");
        Request *r = it->second;
        if (r->state == REQ_RUNNING) return set_error(HZ_E_INVALID, "hz_request_release: the request is running");
        if (r->state == REQ_PENDING) S->pending.erase(std::find(S->pending.begin(), S->pending.end(), r));
        pool_outputs(S, r);
        S->reqs.erase(it);
        delete r;
    }
    S->cv.notify_all();   // returned memory may admit a waiting request
    return HZ_OK;
}
