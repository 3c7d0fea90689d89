// runtime.hip -- host side of libhaze.so: the C ABI of include/haze.h.
//
// Owns the context (device, HBM ledger, scratch), field objects, argument
// validation, per-view job tables and the launches of splat.hip / trace.hip.
// Every entry point validates its arguments before touching the device, so an
// error return leaves outputs untouched and queues no work.
#include "haze.h"
#include "haze_device.h"
#include "serve.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace haze {
hipError_t launch_cell_list(const float *, const float *, const float *, const float *, int32_t, const CellGrid &,
                            uint32_t *, uint32_t *, int64_t, uint32_t *, uint32_t *, uint32_t *, float4 *, void *,
                            bool, uint32_t *, bool, const ScanGuard &, uint32_t *, int32_t, bool, hipStream_t,
                            const KTimer &);
int32_t scan_tiles(int32_t ncells);
size_t scan_scratch_bytes(int32_t ncells);
bool scan_is_onepass(int32_t ncells);
uint32_t *scan_fail_word(void *scan);
hipError_t launch_splat(const SplatParams &, const uint32_t *, const float4 *, float *, const uint32_t *, uint32_t *,
                        const uint32_t *, hipStream_t, const KTimer &);
hipError_t launch_splat_scatter(const SplatParams &, const uint32_t *, const float4 *, const uint32_t *, float *,
                                const uint32_t *, hipStream_t, const KTimer &);
int scatter_max_rows(const SplatParams &P);
int scatter_rows_limit();
hipError_t launch_grad_pack(int, const float *, bool, const int32_t[3], const float[3], float, void *, hipStream_t,
                            const KTimer &);
hipError_t launch_field_unpack(int, const void *, const int32_t[3], float, float *, float *, float *, float *,
                               hipStream_t);
hipError_t launch_raygen(const TraceLaunch &, bool, hipStream_t, const KTimer &);
hipError_t launch_march(int, const TraceLaunch &, int, hipStream_t, const KTimer &);
hipError_t launch_put_table(void *dst, const void *src, size_t bytes, hipStream_t s);
int march_blocks_per_cu(int, int);
const MeshLaunch &mesh_launch(const hz_mesh *m);
float mesh_reach(const hz_mesh *m);
hz_ctx *mesh_ctx(const hz_mesh *m);
void mesh_use(hz_mesh *m, const CallMark &t);
}  // namespace haze

using namespace haze;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static hz_status fail(hz_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

static hz_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? HZ_E_NOMEM : HZ_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HZ_HIP(call, what)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, what);    \
    } while (0)

extern "C" const char *hz_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// context, ledger and scratch
// ---------------------------------------------------------------------------

// A device buffer reused across calls.  `last` is the mark of the call that
// used it last: a reuse on another stream, or freeing it, waits for that.
struct Scratch {
    void *ptr = nullptr;
    size_t cap = 0;
    CallMark last;
    bool clean = false;   // holds what its kernels expect on entry (new memory: no)
};

struct PinnedSlot {
    void *host = nullptr;
    size_t cap = 0;
    CallMark last;
};

// Events of the completion marks (a ring; see mark_issue).
constexpr uint64_t kMarkRing = 64;
// largest brick count the gather dispatches by weight (each phase of the
// ordering runs in one workgroup beside a cell-list kernel)
constexpr int32_t kMaxOrderedBricks = 1 << 16;

struct hz_field {
    hz_ctx *ctx = nullptr;
    void *data = nullptr;
    uint64_t bytes = 0;
    hz_grid grid{};
    hz_dtype dtype = HZ_F32;
    float store_scale = 1.0f;
    CallMark made;                 // the call that wrote the field
    std::vector<CallMark> uses;    // the latest call on each stream that touched it
    std::mutex mu;
    uint32_t serial = 0;           // splat call that built it (0: built from a grid)
    bool bad = false;              // that call's cell-list scan failed: the field holds NaN
};

struct hz_ctx {
    int device = 0;
    int num_cus = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    std::mutex ledger_mu;
    // splat scratch; `count` is clean when all zero, `tiles` when the one-pass
    // scan's ticket counter equals scan_base and its tags are older
    Scratch cid, count, start, lrank, slots, sorted, dn, tiles;
    // the gather's per-brick candidate counts, dispatch order and largest
    // count; `clean` while the counts belong to the bricks in brick_dims
    // (from the last gather, which issued all its launches)
    Scratch bricks;
    int32_t brick_dims[4] = {0, 0, 0, 0};
    uint32_t scan_base = 0;
    // trace scratch; `counters` holds two counter sets used alternately,
    // counter_set the one the next launch uses
    Scratch jobs, hits, bins, counters;
    int counter_set = 0;
    std::vector<PinnedSlot> pinned;
    size_t pinned_next = 0;
    hipEvent_t marks[kMarkRing] = {};
    uint64_t mark_next = 1;
    std::mutex mark_mu;
    int march_bpc[3] = {0, 0, 0};          // by dtype, no scene boards
    int march_bpc_scene[3][3] = {};      // by scene mode (outer boards / inner boards / mesh) and dtype
    // march tuning (hz_ctx_tune)
    int32_t refill_min = 64;
    int32_t blocks_per_cu = 0;   // 0: as many as fit
    int32_t splat_method = 0;    // 0: auto, 1: gather, 2: scatter
    int32_t splat_brick_z = 0;   // gather brick depth: 0 auto, 4 or 8
    int32_t splat_order = 1;     // gather bricks heaviest first (by the previous gather's counts)
    int32_t scan_fault_test = 0; // 1: the one-pass scan's waits give up (fault test)
    // host-visible word (pinned, device-mapped) where a failed scan leaves
    // the serial number of its splat call; splat calls are numbered from 1
    uint32_t *fault_word = nullptr;
    uint32_t *fault_word_dev = nullptr;
    uint32_t splat_serial = 0;
    std::vector<hz_field *> fields;
    std::mutex fields_mu;
    // memory of released fields, reused in stream order (no host sync)
    struct PoolBlock {
        void *ptr;
        size_t bytes;
        std::vector<CallMark> uses;   // the block's last use on each stream
    };
    std::vector<PoolBlock> pool;
    std::mutex pool_mu;
    // optional per-kernel event timing
    struct ProfRec {
        std::string name;
        hipEvent_t a, b;
    };
    bool prof_on = false;
    std::vector<std::string> prof_only;   // empty: every group
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_free;
    std::map<std::string, std::pair<double, int64_t>> prof_acc;
    std::mutex prof_mu;
    Server *server = nullptr;
};

static bool ledger_take(hz_ctx *c, uint64_t bytes)
{
    std::lock_guard<std::mutex> g(c->ledger_mu);
    if (c->used.load() + bytes > c->budget) return false;
    c->used += bytes;
    return true;
}

static void ledger_give(hz_ctx *c, uint64_t bytes)
{
    std::lock_guard<std::mutex> g(c->ledger_mu);
    c->used -= std::min<uint64_t>(bytes, c->used.load());
}

static void pool_trim(hz_ctx *c, size_t need);
static uint64_t pool_bytes(hz_ctx *c);

namespace haze {
// Device allocation charged to the context's budget (used by serve.hip too).
// Pooled memory of released fields is given back first when the budget is
// short.
hz_status ctx_alloc(hz_ctx *c, void **p, size_t bytes)
{
    if (!ledger_take(c, bytes)) {
        pool_trim(c, bytes);
        if (!ledger_take(c, bytes))
            return fail(HZ_E_BUDGET, "allocation of %zu bytes exceeds the HBM budget (%llu of %llu bytes in use)",
                        bytes, (unsigned long long)c->used.load(), (unsigned long long)c->budget);
    }
    hipError_t e = hipMalloc(p, bytes == 0 ? 256 : bytes);
    if (e != hipSuccess) {
        ledger_give(c, bytes);
        *p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    return HZ_OK;
}

// ctx_alloc without giving back pooled field memory: never waits for the
// device or frees anything (HZ_E_BUDGET when the budget has no room).
hz_status ctx_alloc_nowait(hz_ctx *c, void **p, size_t bytes)
{
    if (!ledger_take(c, bytes))
        return fail(HZ_E_BUDGET, "allocation of %zu bytes exceeds the HBM budget (%llu of %llu bytes in use)",
                    bytes, (unsigned long long)c->used.load(), (unsigned long long)c->budget);
    hipError_t e = hipMalloc(p, bytes == 0 ? 256 : bytes);
    if (e != hipSuccess) {
        ledger_give(c, bytes);
        *p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    return HZ_OK;
}

void ctx_free(hz_ctx *c, void *p, size_t bytes)
{
    if (p) (void)hipFree(p);
    ledger_give(c, bytes);
}

int ctx_device(const hz_ctx *c) { return c->device; }

// Give back pooled (released) field memory until `bytes` more fit the budget;
// waits for the blocks' last uses.
void ctx_trim_pool(hz_ctx *c, size_t bytes) { pool_trim(c, bytes); }

// Budget left, counting pooled (released) field memory as available.
uint64_t ctx_mem_avail(const hz_ctx *c)
{
    hz_ctx *cc = const_cast<hz_ctx *>(c);
    const uint64_t used = c->used.load(), pooled = pool_bytes(cc);
    const uint64_t held = used > pooled ? used - pooled : 0;
    return c->budget > held ? c->budget - held : 0;
}
int ctx_num_cus(const hz_ctx *c) { return c->num_cus; }
}  // namespace haze

// ---------------------------------------------------------------------------
// completion marks
// ---------------------------------------------------------------------------
// Each call that enqueues work records ONE event after its last launch, its
// mark, and stamps every buffer and field it used with it.  A later call
// orders itself after a mark only when it runs on another stream or must
// free the memory; on the same stream the order is already there.  (An event
// record is a marker packet that costs the stream microseconds, so one per
// call rather than one per buffer.)  The events form a ring: issuing mark q
// first waits for mark q - kMarkRing, so a mark whose event has been
// recorded again is known to be complete.
static hz_status mark_issue(hz_ctx *c, hipStream_t s, CallMark *out)
{
    std::lock_guard<std::mutex> g(c->mark_mu);
    const uint64_t q = c->mark_next;
    hipEvent_t &e = c->marks[q % kMarkRing];
    if (!e)
        HZ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    else
        HZ_HIP(hipEventSynchronize(e), "hipEventSynchronize");
    HZ_HIP(hipEventRecord(e, s), "hipEventRecord");
    c->mark_next = q + 1;
    *out = CallMark{q, s};
    return HZ_OK;
}

// The event still holding mark t, or null when t is known to be complete.
static hipEvent_t mark_event_locked(hz_ctx *c, const CallMark &t)
{
    if (t.seq == 0 || t.seq + kMarkRing < c->mark_next) return nullptr;
    return c->marks[t.seq % kMarkRing];
}

// Order `stream` after mark t.
static hz_status mark_wait(hz_ctx *c, const CallMark &t, hipStream_t stream)
{
    if (t.seq == 0 || t.stream == stream) return HZ_OK;
    std::lock_guard<std::mutex> g(c->mark_mu);
    hipEvent_t e = mark_event_locked(c, t);
    if (e && hipEventQuery(e) != hipSuccess) HZ_HIP(hipStreamWaitEvent(stream, e, 0), "hipStreamWaitEvent");
    return HZ_OK;
}

// Whether mark t's work is known to be done (a query; never waits).
static bool mark_done(hz_ctx *c, const CallMark &t)
{
    std::lock_guard<std::mutex> g(c->mark_mu);
    hipEvent_t e = mark_event_locked(c, t);
    return !e || hipEventQuery(e) == hipSuccess;
}

// Block the host until mark t's work is done.  Should the event be recorded
// again meanwhile, its issuer has already waited for t.
static hz_status mark_sync(hz_ctx *c, const CallMark &t)
{
    hipEvent_t e;
    {
        std::lock_guard<std::mutex> g(c->mark_mu);
        e = mark_event_locked(c, t);
    }
    if (e) HZ_HIP(hipEventSynchronize(e), "hipEventSynchronize");
    return HZ_OK;
}

// Make `s` at least `bytes` large and order its use on `stream` after its
// previous use.  Growing waits for the previous user before freeing.
static hz_status scratch_acquire(hz_ctx *c, Scratch &s, size_t bytes, hipStream_t stream)
{
    if (s.cap < bytes) {
        hz_status st = mark_sync(c, s.last);
        if (st != HZ_OK) return st;
        if (s.ptr) {
            ctx_free(c, s.ptr, s.cap);
            s.ptr = nullptr;
            s.cap = 0;
        }
        size_t want = std::max<size_t>(bytes, 4096);
        want = (want + 4095) & ~(size_t)4095;
        s.clean = false;
        st = ctx_alloc(c, &s.ptr, want);
        if (st != HZ_OK) return st;
        s.cap = want;
        return HZ_OK;
    }
    return mark_wait(c, s.last, stream);
}

static void scratch_free(hz_ctx *c, Scratch &s)
{
    (void)mark_sync(c, s.last);
    if (s.ptr) ctx_free(c, s.ptr, s.cap);
    s = Scratch{};
}

static hz_status noalloc_setup(int device);

extern "C" hz_status hz_ctx_create(int device, uint64_t hbm_budget_bytes, hz_ctx **out)
{
    if (!out) return fail(HZ_E_INVALID, "hz_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(HZ_E_DEVICE, "hz_ctx_create: no HIP device available (%s)",
                                              e != hipSuccess ? hipGetErrorString(e) : "0 devices");
    if (device < 0 || device >= n) return fail(HZ_E_DEVICE, "hz_ctx_create: device %d out of range [0, %d)", device, n);
    HZ_HIP(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    HZ_HIP(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    size_t free_b = 0, total_b = 0;
    HZ_HIP(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    hz_ctx *c = new hz_ctx();
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    const uint64_t gib = 1ull << 30;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (free_b > gib ? free_b - gib : free_b / 2);
    for (int d = 0; d < 3; ++d) {
        c->march_bpc[d] = march_blocks_per_cu(d, 0);
        c->march_bpc_scene[0][d] = march_blocks_per_cu(d, 1);
        c->march_bpc_scene[1][d] = march_blocks_per_cu(d, 2);
        c->march_bpc_scene[2][d] = march_blocks_per_cu(d, 3);
    }
    c->pinned.resize(8);
    // the completion-mark events exist from the start, so issuing a mark
    // never creates one (hz_trace_views_noalloc issues marks)
    for (hipEvent_t &ev : c->marks) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            for (hipEvent_t &x : c->marks)
                if (x) (void)hipEventDestroy(x);
            delete c;
            return fail(HZ_E_DEVICE, "hz_ctx_create: hipEventCreate failed");
        }
    }
    void *fw = nullptr, *fwd = nullptr;
    if (hipHostMalloc(&fw, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(&fwd, fw, 0) != hipSuccess) {
        if (fw) (void)hipHostFree(fw);
        delete c;
        return fail(HZ_E_NOMEM, "hz_ctx_create: pinned host word for device fault reports");
    }
    c->fault_word = (uint32_t *)fw;
    c->fault_word_dev = (uint32_t *)fwd;
    *c->fault_word = 0u;
    const hz_status st = noalloc_setup(device);
    if (st != HZ_OK) {
        hz_ctx_destroy(c);
        return st;
    }
    *out = c;
    return HZ_OK;
}

// A failed cell-list scan (k_scan_onepass gave up a bounded wait) leaves the
// serial number of its splat call in the context's host-visible word: the
// field that call built is marked bad and the calling entry point reports
// HZ_E_DEVICE (once per failure).
static hz_status take_device_fault(hz_ctx *c, const char *fn)
{
    const uint32_t serial = __atomic_exchange_n(c->fault_word, 0u, __ATOMIC_ACQ_REL);
    if (!serial) return HZ_OK;
    {
        std::lock_guard<std::mutex> g(c->fields_mu);
        for (hz_field *f : c->fields)
            if (f->serial == serial) f->bad = true;
    }
    return fail(HZ_E_DEVICE,
                "%s: the cell-list scan of an earlier hz_splat_index_field call (serial %u) gave up waiting for a "
                "tile sum; the field it built holds NaN and is unusable", fn, serial);
}

// Entry check of a call that reads a field: pending fault reports first, then
// the field's own state.
static hz_status check_field_usable(hz_ctx *c, const hz_field *f, const char *fn)
{
    hz_status st = take_device_fault(c, fn);
    if (st != HZ_OK) return st;
    if (f->bad)
        return fail(HZ_E_DEVICE, "%s: the field was built by a splat call whose cell-list scan failed", fn);
    return HZ_OK;
}

static void field_destroy(hz_field *f)
{
    std::vector<CallMark> uses;
    {
        std::lock_guard<std::mutex> g(f->mu);
        uses = f->uses;
    }
    for (const CallMark &t : uses) (void)mark_sync(f->ctx, t);
    if (f->data) ctx_free(f->ctx, f->data, f->bytes);
    delete f;
}

// Return a field's memory to the context pool; its latest uses order any
// reuse after the work that read it, so releasing never blocks the host.
static void field_recycle(hz_field *f)
{
    hz_ctx *c = f->ctx;
    std::vector<CallMark> uses;
    {
        std::lock_guard<std::mutex> g(f->mu);
        uses.swap(f->uses);
    }
    if (uses.empty()) {
        field_destroy(f);
        return;
    }
    {
        std::lock_guard<std::mutex> g(c->pool_mu);
        c->pool.push_back({f->data, (size_t)f->bytes, std::move(uses)});
    }
    delete f;
}

// Free pooled blocks (waiting for their last use) until `need` more bytes fit
// the budget or the pool is empty.
static void pool_trim(hz_ctx *c, size_t need)
{
    if (need > c->budget) need = c->budget;
    std::lock_guard<std::mutex> g(c->pool_mu);
    while (!c->pool.empty() && c->used.load() + need > c->budget) {
        hz_ctx::PoolBlock b = c->pool.back();
        c->pool.pop_back();
        for (const CallMark &t : b.uses) (void)mark_sync(c, t);
        ctx_free(c, b.ptr, b.bytes);
    }
}

static void pool_free_all(hz_ctx *c) { pool_trim(c, (size_t)-1 / 2); }

static uint64_t pool_bytes(hz_ctx *c)
{
    std::lock_guard<std::mutex> g(c->pool_mu);
    uint64_t b = 0;
    for (const hz_ctx::PoolBlock &p : c->pool) b += p.bytes;
    return b;
}

// ---------------------------------------------------------------------------
// per-kernel event timing
// ---------------------------------------------------------------------------
// Kernels are timed by the events their dispatch packets record (no marker
// packets between kernels, so profiling does not stretch the stream).
static hipEvent_t prof_event_locked(hz_ctx *c)
{
    hipEvent_t e = nullptr;
    if (!c->prof_free.empty()) {
        e = c->prof_free.back();
        c->prof_free.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    return e;
}

// A start/stop pair for a group of launches, or nulls when profiling is off.
static KTimer prof_timer(hz_ctx *c, const char *name)
{
    KTimer t;
    if (!c->prof_on) return t;
    std::lock_guard<std::mutex> g(c->prof_mu);
    if (!c->prof_only.empty() && std::find(c->prof_only.begin(), c->prof_only.end(), name) == c->prof_only.end())
        return t;
    t.start = prof_event_locked(c);
    t.stop = prof_event_locked(c);
    if (!t.start || !t.stop) {
        if (t.start) c->prof_free.push_back(t.start);
        if (t.stop) c->prof_free.push_back(t.stop);
        return KTimer{};
    }
    return t;
}

static void prof_flush_locked(hz_ctx *c)
{
    for (hz_ctx::ProfRec &r : c->prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto &acc = c->prof_acc[r.name];
            acc.first += ms;
            acc.second += 1;
        }
        c->prof_free.push_back(r.a);
        c->prof_free.push_back(r.b);
    }
    c->prof_pending.clear();
}

// Queue a launched timer's pair for accumulation under `name`.
static void prof_commit(hz_ctx *c, const char *name, const KTimer &t)
{
    if (!t.start) return;
    std::lock_guard<std::mutex> g(c->prof_mu);
    c->prof_pending.push_back({name, t.start, t.stop});
    if (c->prof_pending.size() > 65536) prof_flush_locked(c);
}

extern "C" hz_status hz_profile_enable(hz_ctx *c, int32_t enable)
{
    if (!c) return fail(HZ_E_INVALID, "hz_profile_enable: ctx is NULL");
    std::lock_guard<std::mutex> g(c->prof_mu);
    c->prof_on = enable != 0;
    return HZ_OK;
}

extern "C" hz_status hz_profile_select(hz_ctx *c, const char *groups)
{
    if (!c) return fail(HZ_E_INVALID, "hz_profile_select: ctx is NULL");
    static const char *const known[] = {"cell_list", "splat", "grad_pack", "raygen", "march", "serve_batch"};
    std::vector<std::string> sel;
    const std::string all = groups ? groups : "";
    size_t a = 0;
    while (a < all.size()) {
        size_t b = all.find(',', a);
        if (b == std::string::npos) b = all.size();
        const std::string name = all.substr(a, b - a);
        if (std::find(std::begin(known), std::end(known), name) == std::end(known))
            return fail(HZ_E_INVALID, "hz_profile_select: unknown group '%s'", name.c_str());
        sel.push_back(name);
        a = b + 1;
    }
    std::lock_guard<std::mutex> g(c->prof_mu);
    c->prof_only = std::move(sel);
    return HZ_OK;
}

extern "C" hz_status hz_profile_read(hz_ctx *c, const char *kernel, double *total_ms, int64_t *launches,
                                     int32_t reset)
{
    if (!c || !kernel) return fail(HZ_E_INVALID, "hz_profile_read: NULL argument");
    std::lock_guard<std::mutex> g(c->prof_mu);
    prof_flush_locked(c);
    auto it = c->prof_acc.find(kernel);
    if (total_ms) *total_ms = it == c->prof_acc.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == c->prof_acc.end() ? 0 : it->second.second;
    if (reset) c->prof_acc.clear();
    return HZ_OK;
}

extern "C" void hz_ctx_destroy(hz_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->server) {
        server_destroy(c->server);
        c->server = nullptr;
    }
    {
        std::lock_guard<std::mutex> g(c->fields_mu);
        for (hz_field *f : c->fields) field_destroy(f);
        c->fields.clear();
    }
    pool_free_all(c);
    {
        std::lock_guard<std::mutex> g(c->prof_mu);
        prof_flush_locked(c);
        for (hipEvent_t e : c->prof_free) (void)hipEventDestroy(e);
        c->prof_free.clear();
    }
    for (Scratch *s : {&c->cid, &c->count, &c->start, &c->lrank, &c->slots, &c->sorted, &c->dn, &c->tiles, &c->bricks,
                       &c->jobs, &c->hits, &c->bins, &c->counters})
        scratch_free(c, *s);
    for (PinnedSlot &p : c->pinned) {
        (void)mark_sync(c, p.last);
        if (p.host) (void)hipHostFree(p.host);
    }
    for (hipEvent_t e : c->marks)
        if (e) (void)hipEventDestroy(e);
    if (c->fault_word) (void)hipHostFree(c->fault_word);
    delete c;
}

extern "C" hz_status hz_ctx_tune(hz_ctx *c, const char *key, int64_t value)
{
    if (!c || !key) return fail(HZ_E_INVALID, "hz_ctx_tune: NULL argument");
    const std::string k(key);
    if (k == "march.refill_min") {
        if (value < 1 || value > 64) return fail(HZ_E_INVALID, "hz_ctx_tune: march.refill_min must be in [1, 64]");
        c->refill_min = (int32_t)value;
    } else if (k == "march.blocks_per_cu") {
        if (value < 0 || value > 64) return fail(HZ_E_INVALID, "hz_ctx_tune: march.blocks_per_cu must be in [0, 64]");
        c->blocks_per_cu = (int32_t)value;
    } else if (k == "splat.brick_z") {
        if (value != 0 && value != 4 && value != 8)
            return fail(HZ_E_INVALID, "hz_ctx_tune: splat.brick_z must be 0, 4 or 8");
        c->splat_brick_z = (int32_t)value;
    } else if (k == "splat.order") {
        if (value < 0 || value > 1) return fail(HZ_E_INVALID, "hz_ctx_tune: splat.order must be 0 or 1");
        c->splat_order = (int32_t)value;
    } else if (k == "splat.method") {
        if (value < 0 || value > 2) return fail(HZ_E_INVALID, "hz_ctx_tune: splat.method must be 0, 1 or 2");
        c->splat_method = (int32_t)value;
    } else if (k == "splat.scan_fault_test") {
        if (value != 0 && value != 1) return fail(HZ_E_INVALID, "hz_ctx_tune: splat.scan_fault_test must be 0 or 1");
        c->scan_fault_test = (int32_t)value;
    } else {
        return fail(HZ_E_INVALID, "hz_ctx_tune: unknown key '%s'", key);
    }
    return HZ_OK;
}

extern "C" hz_status hz_ctx_memory(const hz_ctx *c, uint64_t *used_bytes, uint64_t *budget_bytes)
{
    if (!c) return fail(HZ_E_INVALID, "hz_ctx_memory: ctx is NULL");
    if (used_bytes) *used_bytes = c->used.load();
    if (budget_bytes) *budget_bytes = c->budget;
    return HZ_OK;
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
static hz_status check_grid(const hz_grid *g, const char *fn)
{
    if (!g) return fail(HZ_E_INVALID, "%s: grid is NULL", fn);
    int64_t nv = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(std::isfinite(g->lo[a]) && std::isfinite(g->hi[a]) && g->hi[a] > g->lo[a]))
            return fail(HZ_E_INVALID, "%s: grid axis %d needs finite lo < hi", fn, a);
        if (g->res[a] < 2 || g->res[a] > 65535)
            return fail(HZ_E_INVALID, "%s: grid res[%d] = %d outside [2, 65535]", fn, a, g->res[a]);
        nv *= g->res[a];
        if (nv > INT32_MAX) return fail(HZ_E_INVALID, "%s: more than 2^31 - 1 voxels", fn);
    }
    return HZ_OK;
}

static hz_status check_dtype(hz_dtype dt, float scale, const char *fn)
{
    if (dt != HZ_F32 && dt != HZ_F16 && dt != HZ_BF16) return fail(HZ_E_INVALID, "%s: unknown dtype %d", fn, (int)dt);
    if (!(std::isfinite(scale) && scale > 0.0f)) return fail(HZ_E_INVALID, "%s: store_scale must be > 0", fn);
    if (dt == HZ_F32 && scale != 1.0f) return fail(HZ_E_INVALID, "%s: store_scale must be 1 for HZ_F32", fn);
    return HZ_OK;
}

static uint64_t field_bytes(const hz_grid *g, hz_dtype dt)
{
    return (uint64_t)g->res[0] * g->res[1] * g->res[2] * (dt == HZ_F32 ? 16u : 8u);
}

static hz_status new_field(hz_ctx *c, const hz_grid *g, hz_dtype dt, float scale, hipStream_t s, hz_field **out)
{
    hz_field *f = new hz_field();
    f->ctx = c;
    f->grid = *g;
    f->dtype = dt;
    f->store_scale = scale;
    f->bytes = field_bytes(g, dt);
    {
        // Reuse a released block of the same size, ordered after its last uses
        // (which stay with the field until its producer has run).  A block
        // still in use on another stream is taken only when the budget has no
        // room for a new one, so that frames on two streams can overlap.
        std::lock_guard<std::mutex> lk(c->pool_mu);
        long pick = -1;
        bool busy = false;
        for (size_t i = 0; i < c->pool.size() && pick < 0; ++i) {
            if (c->pool[i].bytes != f->bytes) continue;
            bool idle = true;
            for (const CallMark &t : c->pool[i].uses) idle = idle && (t.stream == s || mark_done(c, t));
            if (idle) pick = (long)i;
            busy = busy || !idle;
        }
        if (pick < 0 && busy) {
            const bool room = c->used.load() + f->bytes <= c->budget;
            for (size_t i = 0; i < c->pool.size() && pick < 0 && !room; ++i)
                if (c->pool[i].bytes == f->bytes) pick = (long)i;
        }
        if (pick >= 0) {
            f->data = c->pool[(size_t)pick].ptr;
            f->uses = std::move(c->pool[(size_t)pick].uses);
            c->pool.erase(c->pool.begin() + pick);
        }
    }
    if (f->data) {
        for (const CallMark &t : f->uses) {
            hz_status st = mark_wait(c, t, s);
            if (st != HZ_OK) {
                field_destroy(f);
                return st;
            }
        }
        *out = f;
        return HZ_OK;
    }
    pool_trim(c, f->bytes);
    hz_status st = ctx_alloc(c, &f->data, f->bytes);
    if (st != HZ_OK) {
        delete f;
        return st;
    }
    *out = f;
    return HZ_OK;
}

// The call with mark t wrote the field; it ran after every earlier use.
static void field_mark_made(hz_field *f, const CallMark &t)
{
    std::lock_guard<std::mutex> g(f->mu);
    f->made = t;
    f->uses.assign(1, t);
}

// The call with mark t read the field.
static void field_mark_used(hz_field *f, const CallMark &t)
{
    std::lock_guard<std::mutex> g(f->mu);
    for (CallMark &u : f->uses)
        if (u.stream == t.stream) {
            u = t;
            return;
        }
    f->uses.push_back(t);
}

// Order a read of the field on `s` after the call that wrote it.
static hz_status field_order_read(hz_ctx *c, hz_field *f, hipStream_t s)
{
    CallMark m;
    {
        std::lock_guard<std::mutex> g(f->mu);
        m = f->made;
    }
    return mark_wait(c, m, s);
}

static void register_field(hz_ctx *c, hz_field *f)
{
    std::lock_guard<std::mutex> g(c->fields_mu);
    c->fields.push_back(f);
}

// ---------------------------------------------------------------------------
// index field
// ---------------------------------------------------------------------------

// dn_zfast: delta_n as the splat leaves it (z fastest); otherwise [z][y][x].
static hz_status pack_field(hz_ctx *c, const float *dn, bool dn_zfast, const hz_grid *g, hz_field *f, hipStream_t s)
{
    int32_t res[3] = {g->res[0], g->res[1], g->res[2]};
    float inv_sp[3];
    for (int a = 0; a < 3; ++a) inv_sp[a] = (float)((double)g->res[a] / (g->hi[a] - g->lo[a]));
    const KTimer t = prof_timer(c, "grad_pack");
    HZ_HIP(launch_grad_pack((int)f->dtype, dn, dn_zfast, res, inv_sp, f->store_scale, f->data, s, t), "grad/pack launch");
    prof_commit(c, "grad_pack", t);
    return HZ_OK;
}

extern "C" hz_status hz_splat_index_field(hz_ctx *c, const hz_particles *P, const hz_grid *g,
                                          const hz_splat_params *prm, void *hip_stream, hz_field **out)
{
    const char *fn = "hz_splat_index_field";
    if (!c || !P || !prm || !out) return fail(HZ_E_INVALID, "%s: NULL argument", fn);
    hz_status st = check_grid(g, fn);
    if (st != HZ_OK) return st;
    if (P->n < 1) return fail(HZ_E_INVALID, "%s: particle count %lld < 1", fn, (long long)P->n);
    if (P->n > INT32_MAX) return fail(HZ_E_INVALID, "%s: more than 2^31 - 1 particles", fn);
    if (!P->x || !P->y || !P->z || !P->m) return fail(HZ_E_INVALID, "%s: NULL particle array", fn);
    if (!(std::isfinite(prm->h) && prm->h > 0.0f)) return fail(HZ_E_INVALID, "%s: h must be > 0", fn);
    if (!std::isfinite(prm->k_gd)) return fail(HZ_E_INVALID, "%s: k_gd must be finite", fn);
    st = check_dtype(prm->dtype, prm->store_scale, fn);
    if (st != HZ_OK) return st;
    st = take_device_fault(c, fn);
    if (st != HZ_OK) return st;

    // cell list over the grid box grown by the support 2h, cells of edge h
    CellGrid cg{};
    const double h = prm->h;
    const double cell = h;
    int64_t ncells = 1;
    for (int a = 0; a < 3; ++a) {
        const double lo = g->lo[a] - 2.0 * h, hi = g->hi[a] + 2.0 * h;
        const int64_t nc = (int64_t)std::ceil((hi - lo) / cell) + 1;
        if (nc > (1 << 20)) return fail(HZ_E_INVALID, "%s: h too small for the grid box (%lld cells on axis %d)", fn,
                                        (long long)nc, a);
        cg.clo[a] = (float)lo;
        cg.nc[a] = (int32_t)nc;
        ncells *= nc;
    }
    if (ncells > (1ll << 28)) return fail(HZ_E_INVALID, "%s: h too small for the grid box (%lld cells)", fn,
                                         (long long)ncells);
    cg.cell = (float)cell;
    cg.inv_cell = (float)(1.0 / cell);
    cg.ncells = (int32_t)ncells;

    SplatParams sp{};
    for (int a = 0; a < 3; ++a) {
        sp.lo[a] = (float)g->lo[a];
        sp.sp[a] = (float)((g->hi[a] - g->lo[a]) / g->res[a]);
        sp.res[a] = g->res[a];
    }
    sp.nbx = (g->res[0] + SPLAT_BX - 1) / SPLAT_BX;
    sp.nby = (g->res[1] + SPLAT_BY - 1) / SPLAT_BY;
    // brick depth: the one of 4 or 8 voxels that brings the brick closer to
    // twice as deep as wide (8 unless the z spacing exceeds 2 sqrt(2) times
    // the x-y spacing); the deeper brick shares each candidate's cull and x-y
    // distance among more planes
    if (c->splat_brick_z == 4 || c->splat_brick_z == 8)
        sp.bz = c->splat_brick_z;
    else
        sp.bz = (double)sp.sp[2] <= 2.82842712 * 0.5 * ((double)sp.sp[0] + (double)sp.sp[1]) ? 8 : 4;
    sp.nbz = (g->res[2] + sp.bz - 1) / sp.bz;
    sp.h = prm->h;
    sp.inv_h = (float)(1.0 / h);
    sp.support2 = (float)(4.0 * h * h);
    sp.scale = (float)((double)prm->k_gd / (M_PI * h * h * h));
    sp.cg = cg;

    HZ_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    const int32_t n = (int32_t)P->n;
    const int64_t nv = (int64_t)g->res[0] * g->res[1] * g->res[2];
    Scratch *bufs[8] = {&c->cid, &c->count, &c->start, &c->lrank, &c->slots, &c->sorted, &c->dn, &c->tiles};
    const size_t sizes[8] = {4u * (size_t)n, 4u * (size_t)(ncells + 2), 4u * (size_t)(ncells + 1),
                             4u * (size_t)n, 4u * (size_t)n, 16u * (size_t)n, 4u * (size_t)nv,
                             scan_scratch_bytes((int32_t)ncells)};
    for (int i = 0; i < 8; ++i) {
        st = scratch_acquire(c, *bufs[i], sizes[i], s);
        if (st != HZ_OK) return st;
    }
    // the gather is the default (faster on gfx950); the scatter on request
    const bool scatter = c->splat_method == 2;
    if (scatter && scatter_max_rows(sp) > scatter_rows_limit())
        return fail(HZ_E_UNSUPPORTED, "%s: h too large for the scatter splat's tile (use splat.method 1)", fn);
    // Up to kMaxOrderedBricks bricks, the gather records each brick's
    // candidate count, and the next gather over the same bricks dispatches
    // them heaviest first (the order is computed by an extra workgroup of the
    // cell-count launch and one of the cell-order launch).
    const int32_t nbricks = sp.nbx * sp.nby * sp.nbz;
    uint32_t *bwork = nullptr, *border = nullptr;
    bool ordered = false;
    const bool record = !scatter && nbricks <= kMaxOrderedBricks;
    if (record) {
        const bool same = c->brick_dims[0] == sp.nbx && c->brick_dims[1] == sp.nby && c->brick_dims[2] == sp.nbz &&
                          c->brick_dims[3] == sp.bz;
        // counts, order, largest count, scale, 64 bucket sizes
        st = scratch_acquire(c, c->bricks, 8u * (size_t)nbricks + 4u * 66u, s);
        if (st != HZ_OK) return st;
        bwork = (uint32_t *)c->bricks.ptr;
        border = bwork + nbricks;
        ordered = c->splat_order && same && c->bricks.clean;
        c->bricks.clean = false;   // until this call's launches are issued
    }
    hz_field *f = nullptr;
    st = new_field(c, g, prm->dtype, prm->store_scale, s, &f);
    if (st != HZ_OK) return st;

    // Histogram memory is cleared only when not known to be zero (new, or after
    // a scatter-splat call, which leaves max |m| behind); the scan clears what
    // it reads.  The one-pass scan's counter is reset when new, after a
    // three-pass scan, or before its tickets would wrap.
    const int32_t ntiles = scan_tiles((int32_t)ncells);
    const int64_t clear_words = (c->count.clean && !scatter) ? 0 : (int64_t)(c->count.cap / 4);
    // (the fault test also resets the scan, so that no stale tag can match the
    // biased ones it waits for)
    const bool scan_reset = !c->tiles.clean || c->scan_base > 0xffffffffu - (uint32_t)ntiles - 1u ||
                            c->scan_fault_test;
    c->count.clean = false;
    c->tiles.clean = false;
    if (++c->splat_serial == 0) c->splat_serial = 1;
    f->serial = c->splat_serial;
    ScanGuard guard{1u << 26, 0u, c->fault_word_dev, f->serial};
    if (c->scan_fault_test) {
        guard.spin_limit = 64;
        guard.tag_bias = 1u << 30;
    }
    const KTimer t0 = prof_timer(c, "cell_list");
    hipError_t e = launch_cell_list(P->x, P->y, P->z, P->m, n, cg, (uint32_t *)c->cid.ptr, (uint32_t *)c->count.ptr,
                                    clear_words, (uint32_t *)c->start.ptr, (uint32_t *)c->lrank.ptr,
                                    (uint32_t *)c->slots.ptr, (float4 *)c->sorted.ptr, c->tiles.ptr, scan_reset,
                                    &c->scan_base, scatter, guard, bwork, nbricks, ordered, s, t0);
    prof_commit(c, "cell_list", t0);
    if (e == hipSuccess) {
        c->count.clean = !scatter;
        c->tiles.clean = scan_is_onepass((int32_t)ncells);
    }
    if (e == hipSuccess) {
        const KTimer t1 = prof_timer(c, "splat");
        const uint32_t *fail_word = scan_fail_word(c->tiles.ptr);
        if (scatter)
            e = launch_splat_scatter(sp, (const uint32_t *)c->start.ptr, (const float4 *)c->sorted.ptr,
                                     (const uint32_t *)c->count.ptr + ncells + 1, (float *)c->dn.ptr, fail_word, s,
                                     t1);
        else
            e = launch_splat(sp, (const uint32_t *)c->start.ptr, (const float4 *)c->sorted.ptr, (float *)c->dn.ptr,
                             fail_word, bwork, ordered ? border : nullptr, s, t1);
        prof_commit(c, "splat", t1);
    }
    if (e != hipSuccess) {
        field_destroy(f);
        return hip_fail(e, "splat launch");
    }
    st = pack_field(c, (const float *)c->dn.ptr, true, g, f, s);
    if (st != HZ_OK) {
        field_destroy(f);
        return st;
    }
    CallMark done;
    st = mark_issue(c, s, &done);
    if (st != HZ_OK) {
        field_destroy(f);
        return st;
    }
    for (int i = 0; i < 8; ++i) bufs[i]->last = done;
    if (record) {
        c->bricks.last = done;
        c->bricks.clean = true;
        c->brick_dims[0] = sp.nbx;
        c->brick_dims[1] = sp.nby;
        c->brick_dims[2] = sp.nbz;
        c->brick_dims[3] = sp.bz;
    }
    field_mark_made(f, done);
    register_field(c, f);
    *out = f;
    return HZ_OK;
}

extern "C" hz_status hz_index_field_from_grid(hz_ctx *c, const float *dn, const hz_grid *g, hz_dtype dtype,
                                              float store_scale, void *hip_stream, hz_field **out)
{
    const char *fn = "hz_index_field_from_grid";
    if (!c || !dn || !out) return fail(HZ_E_INVALID, "%s: NULL argument", fn);
    hz_status st = check_grid(g, fn);
    if (st != HZ_OK) return st;
    st = check_dtype(dtype, store_scale, fn);
    if (st != HZ_OK) return st;
    st = take_device_fault(c, fn);
    if (st != HZ_OK) return st;
    HZ_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    hz_field *f = nullptr;
    st = new_field(c, g, dtype, store_scale, s, &f);
    if (st != HZ_OK) return st;
    st = pack_field(c, dn, false, g, f, s);
    CallMark done;
    if (st == HZ_OK) st = mark_issue(c, s, &done);
    if (st != HZ_OK) {
        field_destroy(f);
        return st;
    }
    field_mark_made(f, done);
    register_field(c, f);
    *out = f;
    return HZ_OK;
}

extern "C" hz_status hz_field_read(hz_ctx *c, const hz_field *fc, float *dn, float *gx, float *gy, float *gz,
                                   void *hip_stream)
{
    if (!c || !fc) return fail(HZ_E_INVALID, "hz_field_read: NULL argument");
    hz_field *f = const_cast<hz_field *>(fc);
    if (f->ctx != c) return fail(HZ_E_INVALID, "hz_field_read: field belongs to another context");
    hz_status st = check_field_usable(c, f, "hz_field_read");
    if (st != HZ_OK) return st;
    HZ_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    st = field_order_read(c, f, s);
    if (st != HZ_OK) return st;
    HZ_HIP(launch_field_unpack((int)f->dtype, f->data, f->grid.res, 1.0f / f->store_scale, dn, gx, gy, gz, s),
           "unpack launch");
    CallMark done;
    st = mark_issue(c, s, &done);
    if (st == HZ_OK) field_mark_used(f, done);
    return st;
}

extern "C" hz_status hz_field_info(const hz_field *f, hz_grid *grid, hz_dtype *dtype, float *store_scale,
                                   uint64_t *bytes)
{
    if (!f) return fail(HZ_E_INVALID, "hz_field_info: field is NULL");
    if (grid) *grid = f->grid;
    if (dtype) *dtype = f->dtype;
    if (store_scale) *store_scale = f->store_scale;
    if (bytes) *bytes = f->bytes;
    return HZ_OK;
}

extern "C" hz_status hz_field_release(hz_ctx *c, hz_field *f)
{
    if (!c || !f) return fail(HZ_E_INVALID, "hz_field_release: NULL argument");
    if (server_waiting_use(c, f, nullptr))
        return fail(HZ_E_INVALID, "hz_field_release: a request waiting in the serving loop reads the field");
    {
        std::lock_guard<std::mutex> g(c->fields_mu);
        auto it = std::find(c->fields.begin(), c->fields.end(), f);
        if (it == c->fields.end()) return fail(HZ_E_INVALID, "hz_field_release: unknown field");
        c->fields.erase(it);
    }
    (void)hipSetDevice(c->device);
    field_recycle(f);
    return HZ_OK;
}

// ---------------------------------------------------------------------------
// tracing
// ---------------------------------------------------------------------------
namespace haze {

hz_status check_step(const hz_step *st, const char *fn)
{
    if (!st) return fail(HZ_E_INVALID, "%s: step is NULL", fn);
    if (st->uniform) {
        if (!(std::isfinite(st->ds_uniform) && st->ds_uniform > 0.0f))
            return fail(HZ_E_INVALID, "%s: ds_uniform must be > 0", fn);
    } else {
        if (!(std::isfinite(st->ds_min) && st->ds_min > 0.0f))
            return fail(HZ_E_INVALID, "%s: ds_min must be > 0", fn);
        if (!(std::isfinite(st->ds_max) && st->ds_max >= st->ds_min))
            return fail(HZ_E_INVALID, "%s: ds_max must be >= ds_min", fn);
        if (!(std::isfinite(st->theta_max) && st->theta_max > 0.0f))
            return fail(HZ_E_INVALID, "%s: theta_max must be > 0", fn);
        if (!(std::isfinite(st->eps) && st->eps >= 0.0f)) return fail(HZ_E_INVALID, "%s: eps must be >= 0", fn);
    }
    if (st->max_steps < 1) return fail(HZ_E_INVALID, "%s: max_steps must be >= 1", fn);
    if (!(std::isfinite(st->tau_term) && st->tau_term >= 0.0f))
        return fail(HZ_E_INVALID, "%s: tau_term must be >= 0", fn);
    return HZ_OK;
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Camera frame of a view, computed on the host in double precision.
hz_status make_job(const hz_view *v, const void *field, int64_t slot_begin, int64_t ray_begin, TraceJob *J,
                   const char *fn, int index)
{
    if (v->width < 1 || v->height < 1)
        return fail(HZ_E_INVALID, "%s: view %d has size %dx%d", fn, index, v->width, v->height);
    if (!(std::isfinite(v->vfov) && v->vfov > 0.0f && v->vfov < (float)M_PI))
        return fail(HZ_E_INVALID, "%s: view %d vfov must be in (0, pi)", fn, index);
    double f[3], up[3], pn[3];
    for (int a = 0; a < 3; ++a) {
        f[a] = v->fwd[a];
        up[a] = v->up[a];
        pn[a] = v->plane_n[a];
        if (!std::isfinite(v->eye[a]) || !std::isfinite(f[a]) || !std::isfinite(up[a]) ||
            !std::isfinite(v->plane_p[a]) || !std::isfinite(pn[a]))
            return fail(HZ_E_INVALID, "%s: view %d has non-finite values", fn, index);
    }
    const double fl = std::sqrt(dot3(f, f));
    if (!(fl > 0.0)) return fail(HZ_E_INVALID, "%s: view %d fwd is zero", fn, index);
    if (!(dot3(pn, pn) > 0.0)) return fail(HZ_E_INVALID, "%s: view %d plane_n is zero", fn, index);
    for (double &x : f) x /= fl;
    double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    const double rl = std::sqrt(dot3(r, r));
    if (!(rl > 1e-6 * std::sqrt(dot3(up, up))) || !(rl > 0.0))
        return fail(HZ_E_INVALID, "%s: view %d fwd is parallel to up", fn, index);
    for (double &x : r) x /= rl;
    const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    std::memset(J, 0, sizeof *J);
    for (int a = 0; a < 3; ++a) {
        J->eye[a] = v->eye[a];
        J->f[a] = (float)f[a];
        J->r[a] = (float)r[a];
        J->u[a] = (float)u[a];
        J->plane_p[a] = v->plane_p[a];
        J->plane_n[a] = v->plane_n[a];
    }
    J->fpx = (float)(0.5 * (double)v->height / std::tan(0.5 * (double)v->vfov));
    J->half_w = 0.5f * (float)v->width;
    J->half_h = 0.5f * (float)v->height;
    J->width = v->width;
    J->height = v->height;
    J->tiles_x = (v->width + 7) / 8;
    J->field = field;
    J->slot_begin = slot_begin;
    J->ray_begin = ray_begin;
    return HZ_OK;
}

// Chord length -> length bin of the ray sort: kRayBins bins over the box diagonal.
float length_bin_scale(const hz_grid &g)
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) d2 += (g.hi[a] - g.lo[a]) * (g.hi[a] - g.lo[a]);
    return (float)(kRayBins / std::sqrt(d2));
}

void make_trace_grid(const hz_grid &g, float store_scale, TraceGrid *G)
{
    for (int a = 0; a < 3; ++a) {
        const double sp = (g.hi[a] - g.lo[a]) / g.res[a];
        G->lo[a] = (float)g.lo[a];
        G->hi[a] = (float)g.hi[a];
        G->inv_sp[a] = (float)(1.0 / sp);
        G->off[a] = (float)(-g.lo[a] / sp - 0.5);
        G->maxi[a] = (float)(g.res[a] - 2);
        G->res[a] = g.res[a];
    }
    G->inv_scale = 1.0f / store_scale;
}

void make_trace_step(const hz_step &st, const hz_grid &g, TraceStep *S)
{
    S->uniform = st.uniform ? 1 : 0;
    S->theta_max = st.theta_max;
    S->ds_min = st.ds_min;
    S->ds_max = st.ds_max;
    S->eps = st.eps;
    S->ds_uniform = st.ds_uniform;
    S->tau = st.tau_term;
    S->max_steps = st.max_steps;
    // rounding margin: 8 ulps of the largest coordinate of the box
    double amax = 0.0;
    for (int a = 0; a < 3; ++a) amax = std::max(amax, std::max(std::fabs(g.lo[a]), std::fabs(g.hi[a])));
    S->pos_eps = (float)(8.0 * amax * 1.1920928955078125e-7);
    const float cap = std::max(st.uniform ? st.ds_uniform : st.ds_max, st.tau_term);
    S->near_cap = cap * 1.001f + 2.0f * S->pos_eps;
}

}  // namespace haze

// Copy `bytes` from host to device through a pinned staging slot; the caller
// stamps *slot with its call's mark.
static hz_status staged_copy(hz_ctx *c, void *dst, const void *src, size_t bytes, hipStream_t s, PinnedSlot **slot)
{
    PinnedSlot &p = c->pinned[c->pinned_next];
    c->pinned_next = (c->pinned_next + 1) % c->pinned.size();
    hz_status st = mark_sync(c, p.last);
    if (st != HZ_OK) return st;
    if (p.cap < bytes) {
        if (p.host) (void)hipHostFree(p.host);
        p.host = nullptr;
        p.cap = 0;
        HZ_HIP(hipHostMalloc(&p.host, bytes, hipHostMallocDefault), "hipHostMalloc");
        p.cap = bytes;
    }
    std::memcpy(p.host, src, bytes);
    HZ_HIP(hipMemcpyAsync(dst, p.host, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    *slot = &p;
    return HZ_OK;
}

// Scene boards as affine side/u/v functions of the position (double on the
// host, float for the kernels).  The inner boards are those whose bounding box
// comes within one voxel of the volume, the only ones a step's chord can cross.
static hz_status make_scene(const hz_scene *scene, const hz_grid &g, TraceLaunch *L, std::vector<SceneQuad> &qs,
                            const char *fn)
{
    L->nquads = 0;
    L->ninner = 0;
    L->inner_idx = 0u;
    qs.clear();
    if (!scene || scene->nquads == 0) return HZ_OK;
    if (scene->nquads < 0 || scene->nquads > kMaxQuads)
        return fail(HZ_E_INVALID, "%s: nquads = %d outside [0, %d]", fn, scene->nquads, kMaxQuads);
    if (!scene->quads) return fail(HZ_E_INVALID, "%s: NULL quads with nquads = %d", fn, scene->nquads);
    double vox = INFINITY;
    for (int a = 0; a < 3; ++a) vox = std::min(vox, (g.hi[a] - g.lo[a]) / g.res[a]);
    qs.resize((size_t)scene->nquads);
    for (int k = 0; k < scene->nquads; ++k) {
        const hz_quad &q = scene->quads[k];
        double o[3], ea[3], eb[3];
        for (int a = 0; a < 3; ++a) {
            o[a] = q.origin[a];
            ea[a] = q.edge_u[a];
            eb[a] = q.edge_v[a];
            if (!std::isfinite(o[a]) || !std::isfinite(ea[a]) || !std::isfinite(eb[a]))
                return fail(HZ_E_INVALID, "%s: board %d has non-finite values", fn, k);
        }
        const double x[3] = {ea[1] * eb[2] - ea[2] * eb[1], ea[2] * eb[0] - ea[0] * eb[2],
                             ea[0] * eb[1] - ea[1] * eb[0]};
        const double area = std::sqrt(dot3(x, x));
        if (!(area > 1e-9 * std::sqrt(dot3(ea, ea) * dot3(eb, eb))) || !(area > 0.0))
            return fail(HZ_E_INVALID, "%s: board %d has zero or parallel edges", fn, k);
        const double n[3] = {x[0] / area, x[1] / area, x[2] / area};
        // du = (eb x n) / area, dv = (n x ea) / area: u(o + u ea + v eb) = u, v(...) = v
        const double du[3] = {(eb[1] * n[2] - eb[2] * n[1]) / area, (eb[2] * n[0] - eb[0] * n[2]) / area,
                              (eb[0] * n[1] - eb[1] * n[0]) / area};
        const double dv[3] = {(n[1] * ea[2] - n[2] * ea[1]) / area, (n[2] * ea[0] - n[0] * ea[2]) / area,
                              (n[0] * ea[1] - n[1] * ea[0]) / area};
        SceneQuad &Q = qs[(size_t)k];
        for (int a = 0; a < 3; ++a) {
            Q.n[a] = (float)n[a];
            Q.du[a] = (float)du[a];
            Q.dv[a] = (float)dv[a];
        }
        // offsets from the rounded coefficients, so side/u/v vanish at the origin
        double on = 0.0, odu = 0.0, odv = 0.0;
        for (int a = 0; a < 3; ++a) {
            on += (double)Q.n[a] * o[a];
            odu += (double)Q.du[a] * o[a];
            odv += (double)Q.dv[a] * o[a];
        }
        Q.n0 = (float)on;
        Q.du0 = (float)odu;
        Q.dv0 = (float)odv;
        bool overlap = true;
        for (int a = 0; a < 3; ++a) {
            const double c4[4] = {o[a], o[a] + ea[a], o[a] + eb[a], o[a] + ea[a] + eb[a]};
            const double lo = *std::min_element(c4, c4 + 4), hi = *std::max_element(c4, c4 + 4);
            if (hi < g.lo[a] - vox || lo > g.hi[a] + vox) overlap = false;
        }
        if (overlap) {
            if (L->ninner == kMaxInner)
                return fail(HZ_E_UNSUPPORTED, "%s: more than %d boards within a voxel of the volume", fn, kMaxInner);
            L->inner_idx |= (uint32_t)k << (8 * L->ninner);
            ++L->ninner;
        }
    }
    L->nquads = scene->nquads;
    return HZ_OK;
}

// Validation and launch description shared by the tracing entry points:
// jobs[0..nviews) get the camera frames (queue order: 8x8 pixel tiles, view
// after view) and, when all rays are traced, the per-view output pointers;
// L gets everything but the scratch pointers.
static hz_status prepare_trace(hz_ctx *c, const hz_field *fc, const hz_view *views, int32_t nviews, int32_t max_views,
                               const hz_step *step, const int64_t *ray_ids, int64_t nrays, const hz_trace_out *out,
                               uint8_t *surface, uint32_t *tri_tests, TraceJob *jobs, TraceLaunch *Lp,
                               const char *fn)
{
    if (!c || !fc || !views || !out) return fail(HZ_E_INVALID, "%s: NULL argument", fn);
    const hz_field *f = fc;
    if (f->ctx != c) return fail(HZ_E_INVALID, "%s: field belongs to another context", fn);
    if (nviews < 1) return fail(HZ_E_INVALID, "%s: nviews = %d < 1", fn, nviews);
    if (nviews > max_views)
        return fail(max_views < 4096 ? HZ_E_UNSUPPORTED : HZ_E_INVALID, "%s: nviews = %d above the limit of %d", fn,
                    nviews, max_views);
    hz_status st = check_step(step, fn);
    if (st != HZ_OK) return st;
    st = check_field_usable(c, f, fn);
    if (st != HZ_OK) return st;
    int64_t slot = 0, ray = 0;
    for (int i = 0; i < nviews; ++i) {
        st = make_job(&views[i], f->data, slot, ray, &jobs[i], fn, i);
        if (st != HZ_OK) return st;
        const int64_t tiles = (int64_t)((views[i].width + 7) / 8) * ((views[i].height + 7) / 8);
        slot += tiles * 64;
        ray += (int64_t)views[i].width * views[i].height;
    }
    if (slot > INT32_MAX || ray > INT32_MAX) return fail(HZ_E_INVALID, "%s: more than 2^31 - 1 rays", fn);
    const bool subset = ray_ids != nullptr;
    if (!subset && nrays != ray) return fail(HZ_E_INVALID, "%s: nrays = %lld but the views hold %lld rays", fn,
                                             (long long)nrays, (long long)ray);
    if (subset && (nrays < 0 || nrays > INT32_MAX)) return fail(HZ_E_INVALID, "%s: bad nrays %lld", fn,
                                                               (long long)nrays);

    TraceLaunch &L = *Lp;
    L = TraceLaunch{};
    L.njobs = nviews;
    L.subset = subset ? 1 : 0;
    L.nslots = subset ? nrays : slot;
    L.ray_ids = ray_ids;
    L.flat = TraceOutFlat{out->disp, out->exit_pos, out->exit_dir, out->steps, out->status, surface, tri_tests};
    if (!subset)
        for (int i = 0; i < nviews; ++i) {
            TraceJob &J = jobs[i];
            const int64_t base = J.ray_begin;
            J.disp = out->disp ? out->disp + 2 * base : nullptr;
            J.exit_pos = out->exit_pos ? out->exit_pos + 3 * base : nullptr;
            J.exit_dir = out->exit_dir ? out->exit_dir + 3 * base : nullptr;
            J.steps = out->steps ? out->steps + base : nullptr;
            J.status = out->status ? out->status + base : nullptr;
            J.surface = surface ? surface + base : nullptr;
            J.tri_tests = tri_tests ? tri_tests + base : nullptr;
        }
    make_trace_grid(f->grid, f->store_scale, &L.grid);
    make_trace_step(*step, f->grid, &L.step);
    L.refill_min = c->refill_min;
    L.inv_len_bin = length_bin_scale(f->grid);
    return HZ_OK;
}

// Persistent march grid: what fits on the chip at once.
static int march_grid_blocks(const hz_ctx *c, const TraceLaunch &L, int dt)
{
    const int64_t want_blocks = (L.nslots + 255) / 256;
    const int fit = L.mesh.ntris > 0 ? c->march_bpc_scene[2][dt]
                    : L.ninner > 0   ? c->march_bpc_scene[1][dt]
                    : L.nquads > 0   ? c->march_bpc_scene[0][dt]
                                     : c->march_bpc[dt];
    const int bpc = c->blocks_per_cu > 0 ? std::min(c->blocks_per_cu, fit) : fit;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want_blocks, (int64_t)bpc * c->num_cus));
}

static hz_status trace_impl(hz_ctx *c, const hz_field *fc, const hz_view *views, int32_t nviews,
                            const hz_scene *scene, const hz_mesh *mesh, const hz_step *step, const int64_t *ray_ids,
                            int64_t nrays, const hz_trace_out *out, uint8_t *surface, uint32_t *tri_tests,
                            void *hip_stream, const char *fn)
{
    std::vector<TraceJob> jobs((size_t)std::max(0, std::min(nviews, 4096)));
    TraceLaunch L;
    hz_status st = prepare_trace(c, fc, views, nviews, 4096, step, ray_ids, nrays, out, surface, tri_tests,
                                 jobs.data(), &L, fn);
    if (st != HZ_OK) return st;
    hz_field *f = const_cast<hz_field *>(fc);
    if (mesh) {
        if (mesh_ctx(mesh) != c) return fail(HZ_E_INVALID, "%s: mesh belongs to another context", fn);
        const float longest = step->uniform ? step->ds_uniform : step->ds_max;
        if (longest > mesh_reach(mesh))
            return fail(HZ_E_INVALID, "%s: steps up to %g m, but the mesh's shell serves steps up to %g m", fn,
                        (double)longest, (double)mesh_reach(mesh));
        L.mesh = mesh_launch(mesh);
    }
    std::vector<SceneQuad> quads;
    st = make_scene(scene, f->grid, &L, quads, fn);
    if (st != HZ_OK) return st;
    if (L.nslots == 0) return HZ_OK;

    HZ_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    // one upload: the view table, then the scene boards
    const size_t job_bytes = sizeof(TraceJob) * jobs.size();
    const size_t quad_bytes = sizeof(SceneQuad) * quads.size();
    std::vector<unsigned char> table(job_bytes + quad_bytes);
    std::memcpy(table.data(), jobs.data(), job_bytes);
    if (quad_bytes) std::memcpy(table.data() + job_bytes, quads.data(), quad_bytes);
    st = scratch_acquire(c, c->jobs, table.size(), s);
    if (st == HZ_OK) st = scratch_acquire(c, c->hits, 4u * (size_t)L.nslots, s);
    if (st == HZ_OK) st = scratch_acquire(c, c->bins, (size_t)L.nslots, s);
    if (st == HZ_OK) st = scratch_acquire(c, c->counters, kCounterBytes, s);
    if (st != HZ_OK) return st;
    PinnedSlot *staging = nullptr;
    st = staged_copy(c, c->jobs.ptr, table.data(), table.size(), s, &staging);
    if (st != HZ_OK) return st;
    L.jobs = (const TraceJob *)c->jobs.ptr;
    L.quads = quad_bytes ? (const SceneQuad *)((unsigned char *)c->jobs.ptr + job_bytes) : nullptr;
    L.hits = (uint32_t *)c->hits.ptr;
    L.counters = (uint32_t *)c->counters.ptr + (size_t)c->counter_set * kCounterSetWords;
    L.counters_next = (uint32_t *)c->counters.ptr + (size_t)(1 - c->counter_set) * kCounterSetWords;
    L.slot_bin = (uint8_t *)c->bins.ptr;
    const int dt = (int)f->dtype;
    const int blocks = march_grid_blocks(c, L, dt);
    // this launch's counter set was cleared by the previous launch's ray
    // generation; new memory, or a set after a failed call, needs clearing
    const bool clear = !c->counters.clean;
    c->counters.clean = false;
    const KTimer t0 = prof_timer(c, "raygen");
    HZ_HIP(launch_raygen(L, clear, s, t0), "raygen launch");
    prof_commit(c, "raygen", t0);
    // ray generation reads no field data, so only the march waits for the
    // field's construction: on another stream than the splat's, ray
    // generation runs beside it
    st = field_order_read(c, f, s);
    if (st != HZ_OK) {
        // the ray generation just launched still uses the scratch
        CallMark m;
        if (mark_issue(c, s, &m) == HZ_OK) {
            for (Scratch *b : {&c->jobs, &c->hits, &c->bins, &c->counters}) b->last = m;
            staging->last = m;
        }
        return st;
    }
    const KTimer t1 = prof_timer(c, "march");
    HZ_HIP(launch_march(dt, L, blocks, s, t1), "march launch");
    prof_commit(c, "march", t1);
    c->counter_set = 1 - c->counter_set;
    c->counters.clean = true;
    CallMark done;
    st = mark_issue(c, s, &done);
    if (st != HZ_OK) return st;
    for (Scratch *b : {&c->jobs, &c->hits, &c->bins, &c->counters}) b->last = done;
    staging->last = done;
    field_mark_used(f, done);
    if (mesh) mesh_use(const_cast<hz_mesh *>(mesh), done);
    return HZ_OK;
}

extern "C" hz_status hz_trace_views(hz_ctx *c, const hz_field *fc, const hz_view *views, int32_t nviews,
                                    const hz_step *step, const int64_t *ray_ids, int64_t nrays,
                                    const hz_trace_out *out, void *hip_stream)
{
    return trace_impl(c, fc, views, nviews, nullptr, nullptr, step, ray_ids, nrays, out, nullptr, nullptr,
                      hip_stream, "hz_trace_views");
}

extern "C" hz_status hz_trace_scene(hz_ctx *c, const hz_field *fc, const hz_view *views, int32_t nviews,
                                    const hz_scene *scene, const hz_step *step, const int64_t *ray_ids,
                                    int64_t nrays, const hz_trace_out *out, uint8_t *surface, void *hip_stream)
{
    return trace_impl(c, fc, views, nviews, scene, nullptr, step, ray_ids, nrays, out, surface, nullptr,
                      hip_stream, "hz_trace_scene");
}

extern "C" hz_status hz_trace_mesh(hz_ctx *c, const hz_field *fc, const hz_view *views, int32_t nviews,
                                   const hz_mesh *mesh, const hz_step *step, const int64_t *ray_ids, int64_t nrays,
                                   const hz_trace_out *out, uint8_t *surface, uint32_t *tri_tests, void *hip_stream)
{
    if (!mesh) return fail(HZ_E_INVALID, "hz_trace_mesh: mesh is NULL");
    return trace_impl(c, fc, views, nviews, nullptr, mesh, step, ray_ids, nrays, out, surface, tri_tests,
                      hip_stream, "hz_trace_mesh");
}

// ---------------------------------------------------------------------------
// tracing without allocation
// ---------------------------------------------------------------------------
// hz_trace_views_noalloc runs the kernels of hz_trace_views with their launch
// scratch (counter sets, view table, hit list, length bins) in one file-scope
// device array instead of context memory.  Each GPU holds its own copy of the
// array for the life of the process; host code never uses the array's name as
// an address: hz_ctx_create looks up the array's address on the context's
// device once (hipGetSymbolAddress) and every call uses that.
constexpr int32_t kNoAllocViews = 64;
constexpr int64_t kNoAllocSlots = (int64_t)1 << 23;
constexpr size_t kNoAllocTableOff = (kCounterBytes + 255) & ~(size_t)255;
constexpr size_t kNoAllocHitsOff = (kNoAllocTableOff + kNoAllocViews * sizeof(TraceJob) + 255) & ~(size_t)255;
constexpr size_t kNoAllocBinsOff = kNoAllocHitsOff + 4 * (size_t)kNoAllocSlots;
constexpr size_t kNoAllocBytes = kNoAllocBinsOff + (size_t)kNoAllocSlots;
static_assert(sizeof(TraceJob) % 4 == 0, "the view table is copied in 32-bit words");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kNoAllocMaxDevices] = {};

// Once per device, with that device current: the address of `scratch` there.
static hz_status noalloc_setup(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return HZ_OK;   // the entry point then reports it
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_addr[device]) return HZ_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(HZ_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[device] = p;
    return HZ_OK;
}

static void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_addr[device];
}

extern "C" hz_status hz_trace_views_noalloc(hz_ctx *c, const hz_field *fc, const hz_view *views, int32_t nviews,
                                            const hz_step *step, const int64_t *ray_ids, int64_t nrays,
                                            const hz_trace_out *out, void *hip_stream)
{
    const char *fn = "hz_trace_views_noalloc";
    TraceJob jobs[kNoAllocViews];
    TraceLaunch L;
    hz_status st = prepare_trace(c, fc, views, nviews, kNoAllocViews, step, ray_ids, nrays, out, nullptr, nullptr,
                                 jobs, &L, fn);
    if (st != HZ_OK) return st;
    if (L.nslots > kNoAllocSlots)
        return fail(HZ_E_UNSUPPORTED,
                    "%s: %lld queue slots (views padded to 8x8 pixel tiles, or ray ids) exceed the static scratch "
                    "of %lld", fn, (long long)L.nslots, (long long)kNoAllocSlots);
    if (L.nslots == 0) return HZ_OK;
    unsigned char *base = (unsigned char *)noalloc_scratch(c->device);
    if (!base) return fail(HZ_E_DEVICE, "%s: no static scratch address for device %d", fn, c->device);
    hz_field *f = const_cast<hz_field *>(fc);
    HZ_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    st = field_order_read(c, f, s);
    if (st != HZ_OK) return st;
    HZ_HIP(launch_put_table(base + kNoAllocTableOff, jobs, sizeof(TraceJob) * (size_t)nviews, s), "table launch");
    L.jobs = (const TraceJob *)(base + kNoAllocTableOff);
    L.hits = (uint32_t *)(base + kNoAllocHitsOff);
    L.slot_bin = base + kNoAllocBinsOff;
    // every call clears its counter set (k_trace_init); the other set only
    // receives ray generation's clearing for a next launch
    L.counters = (uint32_t *)base;
    L.counters_next = (uint32_t *)base + kCounterSetWords;
    const int dt = (int)f->dtype;
    HZ_HIP(launch_raygen(L, true, s, KTimer{}), "raygen launch");
    HZ_HIP(launch_march(dt, L, march_grid_blocks(c, L, dt), s, KTimer{}), "march launch");
    CallMark done;
    st = mark_issue(c, s, &done);
    if (st != HZ_OK) return st;
    field_mark_used(f, done);
    return HZ_OK;
}

// ---------------------------------------------------------------------------
// serving entry points (serve.hip holds the scheduler)
// ---------------------------------------------------------------------------
namespace haze {
Server *&ctx_server(hz_ctx *c) { return c->server; }
const hz_grid &field_grid(const hz_field *f) { return f->grid; }
hz_dtype field_dtype(const hz_field *f) { return f->dtype; }
float field_scale(const hz_field *f) { return f->store_scale; }
const void *field_data(const hz_field *f) { return f->data; }
hz_ctx *field_ctx(const hz_field *f) { return f->ctx; }
hz_status ctx_mark(hz_ctx *c, hipStream_t s, CallMark *out) { return mark_issue(c, s, out); }
hz_status ctx_mark_sync(hz_ctx *c, const CallMark &t) { return mark_sync(c, t); }
void field_use(hz_field *f, const CallMark &t) { field_mark_used(f, t); }
hz_status field_ready(hz_field *f, hipStream_t s) { return field_order_read(f->ctx, f, s); }
int march_blocks(hz_ctx *c, int dt, int scene_mode)
{
    return (scene_mode == 0 ? c->march_bpc[dt] : c->march_bpc_scene[scene_mode - 1][dt]) * c->num_cus;
}
hz_status build_scene(const hz_scene *scene, const hz_grid &g, TraceLaunch *L, std::vector<SceneQuad> &qs,
                      const char *fn)
{
    return make_scene(scene, g, L, qs, fn);
}
// A time measured by the caller's own events, added to a group's sums when
// profiling is on and the group selected.
void profile_add(hz_ctx *c, const char *name, double ms)
{
    std::lock_guard<std::mutex> g(c->prof_mu);
    if (!c->prof_on) return;
    if (!c->prof_only.empty() && std::find(c->prof_only.begin(), c->prof_only.end(), name) == c->prof_only.end())
        return;
    auto &acc = c->prof_acc[name];
    acc.first += ms;
    acc.second += 1;
}
hz_status set_error(hz_status s, const char *msg) { return fail(s, "%s", msg); }
hz_status field_usable(hz_ctx *c, const hz_field *f, const char *fn) { return check_field_usable(c, f, fn); }
}  // namespace haze
