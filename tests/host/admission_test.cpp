// Host-only checks of the roll-out server's arena and admission order
// (paper_2408_00930_amd/csrc/admission.h), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py. A fake clock
// and a fake arena stand in for the GPU: no HIP call is made.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "admission.h"

#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__,    \
                         __LINE__, #c);                                    \
            std::exit(1);                                                  \
        }                                                                  \
    } while (0)

using wsx::Arena;

static void arena_first_fit_and_merging() {
    Arena a;
    a.init(4096);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(1000, &o1) && o1 == 0);        // rounded up to 1024
    CHECK(a.alloc(256, &o2) && o2 == 1024);
    CHECK(a.alloc(2000, &o3) && o3 == 1280);     // 2048 bytes
    CHECK(a.in_use() == 1024 + 256 + 2048);
    CHECK(!a.alloc(1024, &o4));                   // 768 bytes left
    CHECK(a.alloc(768, &o4) && o4 == 3328);
    CHECK(a.in_use() == 4096 && a.largest_free() == 0);
    a.release(o2, 256);                           // a hole of 256 between o1 and o3
    CHECK(!a.alloc(512, &o2));
    a.release(o1, 1000);                          // merges with the hole: 1280 at 0
    CHECK(a.free_blocks() == 1 && a.largest_free() == 1280);
    CHECK(a.alloc(1280, &o1) && o1 == 0);
    a.release(o3, 2000);
    a.release(o4, 768);                           // merges with o3's block
    CHECK(a.free_blocks() == 1 && a.largest_free() == 2048 + 768);
    a.release(o1, 1280);                          // everything free, one block
    CHECK(a.free_blocks() == 1 && a.largest_free() == 4096 && a.in_use() == 0);
    CHECK(a.peak() == 4096);
}

// Random allocations and releases against a byte map of owners: blocks never
// overlap, never leave the arena, and the free list always covers the rest.
static void arena_random_against_a_byte_map() {
    const size_t size = 1 << 20;
    Arena a;
    a.init(size);
    std::vector<int> owner(size / 256, -1);
    std::map<int, std::pair<size_t, size_t>> live;
    std::mt19937_64 rng(7);
    int next = 0;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            const size_t want = 1 + rng() % 40000;
            size_t off;
            if (a.alloc(want, &off)) {
                const size_t g = wsx::arena_align(want) / 256;
                CHECK(off % 256 == 0 && off / 256 + g <= owner.size());
                for (size_t i = 0; i < g; ++i) {
                    CHECK(owner[off / 256 + i] == -1);
                    owner[off / 256 + i] = next;
                }
                live[next++] = {off, want};
            } else {
                CHECK(a.largest_free() < wsx::arena_align(want));
            }
        } else {
            auto itl = live.begin();
            std::advance(itl, (long)(rng() % live.size()));
            const size_t g = wsx::arena_align(itl->second.second) / 256;
            for (size_t i = 0; i < g; ++i) owner[itl->second.first / 256 + i] = -1;
            a.release(itl->second.first, itl->second.second);
            live.erase(itl);
        }
        size_t used = 0;
        for (int o : owner) used += o >= 0 ? 256 : 0;
        CHECK(used == a.in_use());
    }
}

struct FakeRequest {
    double submitted_ms;
    size_t bytes;
    size_t off = 0;
    bool admitted = false;
};

// The admission pass with a fake clock: requests that fit are admitted in
// queue order, smaller later ones overtake a large one that does not fit,
// until the large one has waited past the limit at the head of the queue.
static void admission_order_with_a_fake_clock() {
    Arena a;
    a.init(10 * 256);
    std::map<int64_t, FakeRequest> reqs;
    std::deque<int64_t> queue;
    double now = 0.0;
    auto submit = [&](int64_t id, size_t bytes) {
        reqs[id] = FakeRequest{now, bytes};
        queue.push_back(id);
    };
    auto pass = [&]() {
        return wsx::admit_in_order(
            queue, 100.0,
            [&](int64_t id) {
                FakeRequest& r = reqs[id];
                if (!a.alloc(r.bytes, &r.off)) return false;
                r.admitted = true;
                return true;
            },
            [&](int64_t id) { return now - reqs[id].submitted_ms; });
    };
    auto finish = [&](int64_t id) { a.release(reqs[id].off, reqs[id].bytes); };

    submit(1, 6 * 256);
    submit(2, 6 * 256);   // does not fit beside 1
    submit(3, 2 * 256);   // fits: overtakes 2
    now = 1.0;
    CHECK(pass());
    CHECK(reqs[1].admitted && !reqs[2].admitted && reqs[3].admitted);
    CHECK(queue.size() == 1 && queue.front() == 2);
    // 2 is at the head but has waited only 40 ms: a small one may overtake
    now = 40.0;
    submit(4, 256);
    CHECK(pass());
    CHECK(reqs[4].admitted && !reqs[2].admitted);
    // past 100 ms at the head nothing behind 2 is admitted
    now = 150.0;
    submit(5, 256);
    CHECK(!pass());
    CHECK(!reqs[5].admitted && queue.size() == 2);
    // once memory frees, 2 goes first, then 5
    finish(1);
    now = 151.0;
    CHECK(pass());
    CHECK(reqs[2].admitted && reqs[5].admitted && queue.empty());
    CHECK(a.in_use() == (6 + 2 + 1 + 1) * 256);
}

int main() {
    arena_first_fit_and_merging();
    arena_random_against_a_byte_map();
    admission_order_with_a_fake_clock();
    std::printf("admission: ok\n");
    return 0;
}
