// CPU checks of the sort server's admission control (compiled by
// tests/test_serving_host.py with g++; no GPU involved).
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "ssort_admission.h"

#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); std::exit(1); } } while (0)

int main() {
    using ssd::Admission;
    using ssd::Arena;
    {   // arena: first fit, release, coalescing
        Arena a(1024, 64);
        size_t o1, o2, o3, o4;
        CHECK(a.alloc(100, &o1) && o1 == 0);
        CHECK(a.alloc(100, &o2) && o2 == 128);
        CHECK(a.alloc(500, &o3) && o3 == 256);
        CHECK(!a.alloc(300, &o4));              // 1024 - 768 = 256 free
        a.release(o2);
        CHECK(a.alloc(64, &o4) && o4 == 128);   // first fit reuses the hole
        a.release(o4);
        a.release(o1);
        CHECK(a.free_blocks() == 2);            // [0,256) and [768,1024)
        a.release(o3);
        CHECK(a.free_blocks() == 1 && a.used() == 0);
        CHECK(a.alloc(1024, &o1) && o1 == 0);
        std::printf("arena ok\n");
    }
    {   // admission: over-budget refusal, budget exhaustion, FIFO, release
        Admission ad(1000, 1);
        CHECK(!ad.submit(99, 1001));            // larger than the whole budget
        CHECK(ad.submit(1, 600) && ad.submit(2, 300) && ad.submit(3, 200));
        auto got = ad.admit(10);
        CHECK(got.size() == 2 && got[0].first == 1 && got[1].first == 2);
        CHECK(ad.waiting() == 1 && ad.used() == 900);
        CHECK(ad.admit(10).empty());            // job 3 waits for memory
        ad.release(got[0].second);
        auto got2 = ad.admit(10);
        CHECK(got2.size() == 1 && got2[0].first == 3);
        // head of line: a big job is not overtaken by a small one behind it
        CHECK(ad.submit(4, 900) && ad.submit(5, 10));
        CHECK(ad.admit(10).empty());
        ad.release(got[1].second);
        ad.release(got2[0].second);
        auto got3 = ad.admit(10);
        CHECK(got3.size() == 2 && got3[0].first == 4 && got3[1].first == 5);
        std::printf("admission ok\n");
    }
    {   // cancellation and the per-launch job limit
        Admission ad(100, 1);
        for (uint64_t t = 1; t <= 5; ++t) CHECK(ad.submit(t, 10));
        CHECK(ad.cancel(3) && !ad.cancel(3) && !ad.cancel(42));
        auto got = ad.admit(2);
        CHECK(got.size() == 2 && got[0].first == 1 && got[1].first == 2);
        auto got2 = ad.admit(10);
        CHECK(got2.size() == 2 && got2[0].first == 4 && got2[1].first == 5);
        CHECK(ad.waiting() == 0);
        // weight limit (strings per launch): always admits at least one job
        CHECK(ad.submit(6, 10) && ad.submit(7, 10) && ad.submit(8, 10));
        auto got3 = ad.admit(10, 15, [](uint64_t t) { return (uint64_t)(t == 6 ? 20 : 5); });
        CHECK(got3.size() == 1 && got3[0].first == 6);
        auto got4 = ad.admit(10, 15, [](uint64_t) { return (uint64_t)5; });
        CHECK(got4.size() == 2);
        std::printf("cancel/limits ok\n");
    }
    {   // packed batches: one block per launch, FIFO prefix, per-launch limits
        Admission ad(1000, 1);
        for (uint64_t t = 1; t <= 4; ++t) CHECK(ad.submit(t, 100 * t));   // 100, 200, 300, 400
        size_t tot = 0;
        std::vector<uint64_t> got;
        size_t off;
        auto reset = [&] { tot = 0; };
        reset();
        // packed size: sum of the jobs plus 50 bytes of shared overhead
        CHECK(ad.admit_batch(10, [&](uint64_t t) { tot += 100 * t; }, [&] { return tot + 50; }, &got, &off));
        CHECK(got.size() == 3 && got[0] == 1 && got[2] == 3 && off == 0 && ad.used() == 650);
        reset();
        CHECK(!ad.admit_batch(10, [&](uint64_t t) { tot += 100 * t; }, [&] { return tot + 50; }, &got, &off));
        ad.release(0);
        reset();
        // a second limit (e.g. strings per launch) cuts the batch
        CHECK(ad.submit(5, 10) && ad.submit(6, 10));
        size_t cnt = 0;
        CHECK(ad.admit_batch(10, [&](uint64_t t) { tot += t == 4 ? 400 : 10; ++cnt; },
                             [&] { return cnt > 2 ? (size_t)-1 : tot; }, &got, &off));
        CHECK(got.size() == 2 && got[0] == 4 && got[1] == 5 && ad.waiting() == 1);
        std::printf("batch ok\n");
    }
    std::printf("ALL OK\n");
    return 0;
}
