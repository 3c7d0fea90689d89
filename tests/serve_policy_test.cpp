// CPU test of the serving loop's batching policy (serve_policy.h).
#include "serve_policy.h"

#include <cstdio>
#include <cstdlib>

using namespace haze;

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static PendingInfo req(int key, int64_t slots, int64_t bytes)
{
    PendingInfo p;
    p.key = zero_key();
    p.key.res[0] = key;   // requests with equal `key` share launches
    p.slots = slots;
    p.out_bytes = bytes;
    return p;
}

int main()
{
    // empty queue
    CHECK(plan_batch({}, 100, 100, 8).empty());
    // the oldest request leads; compatible followers join in order
    {
        std::vector<PendingInfo> q = {req(1, 10, 10), req(2, 10, 10), req(1, 20, 20), req(1, 30, 30)};
        auto p = plan_batch(q, 100, 1000, 8);
        CHECK(p.size() == 3 && p[0] == 0 && p[1] == 2 && p[2] == 3);
    }
    // slot capacity: a follower that would overflow is skipped, a later smaller one joins
    {
        std::vector<PendingInfo> q = {req(1, 60, 1), req(1, 50, 1), req(1, 30, 1)};
        auto p = plan_batch(q, 100, 1000, 8);
        CHECK(p.size() == 2 && p[0] == 0 && p[1] == 2);
    }
    // memory admission: the head waits when its outputs do not fit
    {
        std::vector<PendingInfo> q = {req(1, 10, 500), req(1, 10, 10)};
        CHECK(plan_batch(q, 100, 400, 8).empty());
        auto p = plan_batch(q, 100, 505, 8);
        CHECK(p.size() == 1 && p[0] == 0);
        p = plan_batch(q, 100, 510, 8);
        CHECK(p.size() == 2);
    }
    // a head larger than a launch can never run in this slot
    {
        std::vector<PendingInfo> q = {req(1, 200, 1)};
        CHECK(plan_batch(q, 100, 1000, 8).empty());
    }
    // request cap per launch
    {
        std::vector<PendingInfo> q;
        for (int i = 0; i < 20; ++i) q.push_back(req(3, 1, 1));
        CHECK(plan_batch(q, 100, 1000, 5).size() == 5);
    }
    // requests with different scene boards never share a launch
    {
        std::vector<PendingInfo> q = {req(1, 10, 10), req(1, 10, 10), req(1, 10, 10)};
        q[1].key.nquads = 1;
        q[1].key.quads[0][4] = 0.5f;
        q[2].key.nquads = 1;
        q[2].key.quads[0][4] = 0.5f;
        auto p = plan_batch(q, 100, 1000, 8);
        CHECK(p.size() == 1 && p[0] == 0);
        std::vector<PendingInfo> r(q.begin() + 1, q.end());
        auto p2 = plan_batch(r, 100, 1000, 8);
        CHECK(p2.size() == 2);
    }
    // requests with different meshes never share a launch; the same mesh does
    {
        std::vector<PendingInfo> q = {req(1, 10, 10), req(1, 10, 10), req(1, 10, 10), req(1, 10, 10)};
        q[0].key.mesh = 0x1000;
        q[1].key.mesh = 0x2000;
        q[2].key.mesh = 0x1000;
        auto p = plan_batch(q, 100, 1000, 8);
        CHECK(p.size() == 2 && p[0] == 0 && p[1] == 2);
    }
    // slot counting: 8x8 tiles of 64 slots, ragged edges padded
    CHECK(view_slots(8, 8) == 64);
    CHECK(view_slots(9, 8) == 128);
    CHECK(view_slots(1280, 720) == 1280 * 720);
    CHECK(view_slots(37, 23) == 5 * 3 * 64);
    CHECK(kOutBytesPerRay == 38);   // disp, exit_pos, exit_dir, steps, status, surface
    // output size classes: hold the request, at least 64 KiB, at most 1.25x above that, monotone, four per octave
    {
        size_t prev = 0;
        int classes_in_octave = 0;
        size_t octave = (size_t)64 << 10;
        for (int64_t b = 1; b <= ((int64_t)1 << 33); b = b < 4096 ? b + 1 : b + b / 97 + 1) {
            const size_t c = out_class(b);
            CHECK(c >= (size_t)b);
            CHECK(c >= ((size_t)64 << 10));
            if (b > ((int64_t)64 << 10)) CHECK((double)c <= 1.25 * (double)b);
            CHECK(c >= prev);
            if (c != prev) {
                while (c > 2 * octave) {
                    octave *= 2;
                    classes_in_octave = 0;
                }
                CHECK(++classes_in_octave <= 4 + 1);
            }
            prev = c;
        }
        CHECK(out_class(0) == ((size_t)64 << 10));
        CHECK(out_class((int64_t)64 << 10) == ((size_t)64 << 10));
        CHECK(out_class(((int64_t)64 << 10) + 1) == ((size_t)80 << 10));
        CHECK(out_class((int64_t)1 << 20) == ((size_t)1 << 20));
        CHECK(out_class(((int64_t)1 << 20) + 1) == ((size_t)1280 << 10));
    }
    // the output pool: blocks come back by class, the byte count follows, drain empties it
    {
        OutputPool pool;
        int a = 0, b = 0, c = 0;
        pool.put(&a, 1024);
        pool.put(&b, 2048);
        pool.put(&c, 1024);
        CHECK(pool.bytes == 4096);
        CHECK(pool.take(4096) == nullptr);
        void *x = pool.take(2048);
        CHECK(x == &b && pool.bytes == 2048);
        void *y = pool.take(1024), *z = pool.take(1024);
        CHECK(((y == &a && z == &c) || (y == &c && z == &a)) && pool.bytes == 0);
        CHECK(pool.take(1024) == nullptr);
        pool.put(&a, 1024);
        pool.put(&b, 4096);
        const std::vector<PoolBlock> all = pool.drain();
        CHECK(all.size() == 2 && pool.bytes == 0 && pool.blocks.empty());
        CHECK(pool.take(4096) == nullptr);
    }
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
    return failures ? 1 : 0;
}
