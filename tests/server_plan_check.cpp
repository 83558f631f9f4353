// CPU check of the serving loop's scheduling (paper_1605_00561_amd/csrc/server_plan.h):
// range sets and the arena free list against brute-force models, and the choice of
// each batch on hand-made request queues.  Built and run by tests/test_server_plan.py;
// prints "ok <checks>" or the first failed check and exits non-zero.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "server_plan.h"

using namespace dwt2::serve;

static int checks = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        ++checks;                                                              \
        if (!(c)) {                                                            \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

static void range_sets()
{
    RangeSet s;
    CHECK(!s.overlaps(0, 100));
    s.insert(10, 20);
    CHECK(s.overlaps(15, 16) && s.overlaps(0, 11) && s.overlaps(19, 30));
    CHECK(!s.overlaps(0, 10) && !s.overlaps(20, 30));  // half-open ranges only touch
    s.insert(20, 30);                                   // touching: merged
    CHECK(s.size() == 1 && s.overlaps(25, 26));
    s.insert(50, 60);
    s.insert(5, 55);                                    // spans both
    CHECK(s.size() == 1 && s.overlaps(58, 59) && !s.overlaps(60, 70));
    // random ranges against a bitmap over [0, 512)
    std::mt19937 rng(7);
    for (int round = 0; round < 200; round++) {
        RangeSet r;
        std::vector<bool> bits(512, false);
        for (int k = 0; k < 12; k++) {
            const unsigned lo = rng() % 500, hi = lo + 1 + rng() % 12;
            r.insert(lo, hi);
            for (unsigned i = lo; i < hi; i++) bits[i] = true;
        }
        for (int q = 0; q < 50; q++) {
            const unsigned lo = rng() % 500, hi = lo + 1 + rng() % 20;
            bool any = false;
            for (unsigned i = lo; i < hi && i < 512; i++) any |= bits[i];
            CHECK(r.overlaps(lo, hi) == any);
        }
    }
}

static void arenas()
{
    Arena a(1000);
    CHECK(a.fits(1000) && !a.fits(1001));
    const size_t x = a.alloc(300), y = a.alloc(300), z = a.alloc(400);
    CHECK(x == 0 && y == 300 && z == 600 && !a.fits(1) && a.alloc(1) == SIZE_MAX);
    a.release(y, 300);
    CHECK(a.fits(300) && !a.fits(301) && a.alloc(200) == 300);   // first fit
    a.release(300, 200);
    a.release(x, 300);                                         // coalesces with [300, 600)
    CHECK(a.blocks() == 1 && a.fits(600) && !a.fits(601));
    a.release(z, 400);
    CHECK(a.blocks() == 1 && a.fits(1000));
    // random traffic against a bitmap: allocations never overlap, everything is
    // returned, and the list ends as one block
    std::mt19937 rng(11);
    Arena b(4096);
    std::vector<int> owner(4096, -1);
    std::vector<std::pair<size_t, size_t>> live;
    for (int step = 0; step < 4000; step++) {
        if (live.empty() || rng() % 2) {
            const size_t n = 1 + rng() % 300;
            if (!b.fits(n)) continue;
            const size_t off = b.alloc(n);
            CHECK(off != SIZE_MAX && off + n <= 4096);
            for (size_t i = off; i < off + n; i++) {
                CHECK(owner[i] == -1);
                owner[i] = step;
            }
            live.push_back({off, n});
        } else {
            const size_t k = rng() % live.size();
            for (size_t i = live[k].first; i < live[k].first + live[k].second; i++) owner[i] = -1;
            b.release(live[k].first, live[k].second);
            live.erase(live.begin() + k);
        }
    }
    for (auto &l : live) b.release(l.first, l.second);
    CHECK(b.blocks() == 1 && b.fits(4096));
}

// table bytes of a batched call in this check: 256 per image plus 256 per level
static size_t table(int count, int lmax) { return 256 * (size_t)count + 256 * (size_t)lmax; }

static Item req(uintptr_t src, uintptr_t dst, size_t bytes, int inverse, int levels, size_t ll)
{
    Item it{src, src + bytes, dst, dst + bytes, inverse, levels, ll, 0};
    it.footprint = footprint_of(it);
    return it;
}

static size_t plan(const std::vector<Item> &q, int max_batch, const Arena &a, Group g[2],
                   size_t budget = SIZE_MAX, size_t *fp_out = nullptr)
{
    size_t fp = 0;
    const size_t n = next_batch([&](size_t i) { return q[i]; }, q.size(), max_batch, a, budget, table, g, &fp);
    if (fp_out) *fp_out = fp;
    return n;
}

// The footprint budget against a brute-force model: the batch is the longest
// prefix (within max_batch, no range conflicts here) whose footprints sum to
// at most the budget, and the reported footprint is that sum.
static void footprints()
{
    Arena big(1 << 30);
    Group g[2];
    std::vector<Item> q;
    for (int i = 0; i < 8; i++) q.push_back(req(0x100000 * (2 * i + 1), 0x100000 * (2 * i + 2), 1000, i % 2, 2, 100));
    CHECK(q[0].footprint == 2100);  // input + output + LL buffers
    size_t fp = 0;
    CHECK(plan(q, 256, big, g, SIZE_MAX, &fp) == 8 && fp == 8 * 2100);
    CHECK(plan(q, 256, big, g, 2099, &fp) == 0 && fp == 0);      // the head alone is over
    CHECK(plan(q, 256, big, g, 2100, &fp) == 1 && fp == 2100);
    CHECK(plan(q, 256, big, g, 3 * 2100 + 2099, &fp) == 3 && fp == 3 * 2100);
    std::mt19937 rng(13);
    for (int round = 0; round < 300; round++) {
        std::vector<Item> r;
        const int n = 1 + rng() % 12;
        for (int i = 0; i < n; i++)
            r.push_back(req(0x1000000 * (2 * i + 1), 0x1000000 * (2 * i + 2), 1 + rng() % 5000,
                            rng() % 2, 1 + rng() % 6, rng() % 3000));
        const size_t budget = rng() % 40000;
        const int max_batch = 1 + rng() % 16;
        size_t want = 0, acc = 0;
        while (want < r.size() && (int)want < max_batch && acc + r[want].footprint <= budget)
            acc += r[want++].footprint;
        CHECK(plan(r, max_batch, big, g, budget, &fp) == want && fp == acc);
        CHECK(g[0].count + g[1].count == (int)want);
    }
}

static void batches()
{
    Arena big(1 << 30);
    Group g[2];
    std::vector<Item> q;
    for (int i = 0; i < 10; i++) q.push_back(req(0x100000 * (2 * i + 1), 0x100000 * (2 * i + 2), 4096, i % 2, 1 + i % 3, 512));
    CHECK(plan(q, 256, big, g) == 10);                      // independent requests: one batch
    CHECK(g[0].count == 5 && g[1].count == 5 && g[0].lmax == 3 && g[1].lmax == 3);
    CHECK(g[0].ll == 5 * 512 && group_bytes(g[0], table) == table(5, 3) + 5 * 512);
    CHECK(plan(q, 4, big, g) == 4);                         // max_batch
    // a request reading the output of an earlier one waits for the next batch
    q[3].src_lo = q[1].dst_lo + 100;
    q[3].src_hi = q[3].src_lo + 10;
    CHECK(plan(q, 256, big, g) == 3);
    // writing what an earlier one reads, or writes, also ends the batch
    std::vector<Item> w = {req(0x1000, 0x2000, 0x100, 0, 1, 0), req(0x5000, 0x1080, 0x10, 0, 1, 0)};
    CHECK(plan(w, 256, big, g) == 1);
    w[1] = req(0x5000, 0x20f0, 0x100, 0, 1, 0);
    CHECK(plan(w, 256, big, g) == 1);
    // two requests reading the same source share a batch
    w[1] = req(0x1000, 0x9000, 0x100, 1, 2, 0);
    CHECK(plan(w, 256, big, g) == 2 && g[0].count == 1 && g[1].count == 1);
    // the arena: the prefix stops at the first request that no longer fits
    std::vector<Item> m;
    for (int i = 0; i < 6; i++) m.push_back(req(0x100000 * (2 * i + 1), 0x100000 * (2 * i + 2), 64, 0, 2, 1000));
    Arena small(3000);  // one image: 256 + 512 + 1000 = 1768; two: 512 + 512 + 2000 = 3024
    CHECK(plan(m, 256, small, g) == 1 && group_bytes(g[0], table) == 1768);
    Arena none(1000);
    CHECK(plan(m, 256, none, g) == 0);                      // the head does not fit
    CHECK(plan(m, 256, Arena(0), g) == 0);
    std::vector<Item> empty;
    CHECK(plan(empty, 256, big, g) == 0 && g[0].count == 0 && g[1].count == 0);
}

int main()
{
    range_sets();
    arenas();
    batches();
    footprints();
    printf("ok %d\n", checks);
    return 0;
}
