// Host check of the device-memory arena's bookkeeping (offsets only; segment
// memory is simulated).  Exit status 0 when every invariant holds.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "rsf_arena.hpp"

#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                                  \
        }                                                              \
    } while (0)

int main()
{
    using rsf::Arena;
    const size_t A = 256;
    // 1. budget and segment growth
    {
        Arena a(10000 * A, 4000 * A, A);
        int grows = 0;
        auto grow = [&](size_t len) { ++grows; return len % A == 0; };
        Arena::Block b1, b2, b3, b4, b5;
        CHECK(a.alloc(3000 * A, b1, grow) && grows == 1 && a.segments() == 1);
        CHECK(a.segment_bytes(0) == 4000 * A);
        CHECK(a.alloc(1000 * A, b2, grow) && grows == 1 && b2.seg == 0 && b2.off == 3000 * A);
        // larger than a segment: a segment of its own size
        CHECK(a.alloc(5000 * A, b3, grow) && grows == 2 && a.segment_bytes(1) == 5000 * A);
        // the last segment is cut to what the budget leaves
        CHECK(a.alloc(600 * A, b4, grow) && grows == 3 && a.segment_bytes(2) == 1000 * A);
        CHECK(!a.alloc(401 * A, b5, grow) && grows == 3);
        CHECK(a.alloc(400 * A, b5, grow) && b5.seg == 2 && b5.off == 600 * A);
        CHECK(a.in_use() == 10000 * A && a.peak() == 10000 * A && a.reserved() == 10000 * A);
        CHECK(!a.alloc(1, b5, grow));
        a.release(b2);
        Arena::Block b6;
        CHECK(a.alloc(999 * A + 1, b6, grow) && b6.seg == 0 && b6.off == 3000 * A &&
              b6.len == 1000 * A);
        a.release(b1);
        a.release(b6);
        a.release(b3);
        a.release(b4);
        a.release(b5);
        CHECK(a.in_use() == 0);
        CHECK(a.largest_free(0) == 4000 * A && a.largest_free(1) == 5000 * A &&
              a.largest_free(2) == 1000 * A);
    }
    // 2. a failing grow leaves the arena unchanged
    {
        Arena a(100 * A, 50 * A, A);
        Arena::Block b;
        CHECK(!a.alloc(10 * A, b, [](size_t) { return false; }));
        CHECK(a.segments() == 0 && a.reserved() == 0 && a.in_use() == 0);
    }
    // 3. random alloc/free: no overlap, in-use accounting, full coalescing
    {
        std::mt19937_64 rng(12345);
        Arena a(1 << 30, 1 << 24, A);
        std::vector<Arena::Block> live;
        for (int step = 0; step < 20000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t n = 1 + rng() % (1 << 20);
                Arena::Block b;
                if (a.alloc(n, b, [](size_t) { return true; })) {
                    CHECK(b.off % A == 0 && b.len % A == 0 && b.len >= n);
                    CHECK(b.off + b.len <= a.segment_bytes(b.seg));
                    for (const auto &o : live)
                        CHECK(o.seg != b.seg || o.off + o.len <= b.off || b.off + b.len <= o.off);
                    live.push_back(b);
                }
            } else {
                const size_t k = rng() % live.size();
                a.release(live[k]);
                live[k] = live.back();
                live.pop_back();
            }
            size_t sum = 0;
            for (const auto &o : live) sum += o.len;
            CHECK(sum == a.in_use());
            CHECK(a.reserved() <= (size_t)1 << 30);
        }
        for (const auto &o : live) a.release(o);
        CHECK(a.in_use() == 0);
        for (int s = 0; s < a.segments(); ++s) CHECK(a.largest_free(s) == a.segment_bytes(s));
    }
    std::printf("arena ok\n");
    return 0;
}
