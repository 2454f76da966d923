// Checks of the host worker pool (host_pool.h) on the CPU: every chunk runs
// exactly once, a loop nested in a chunk and loops from several threads at
// once complete, an exception thrown in a chunk reaches the caller, and the
// per-loop cost (printed) after the pool has started.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <stdexcept>
#include <thread>
#include <vector>

#include "host_pool.h"

using bfi::for_chunks;
using bfi::parallel_range;

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                            \
        }                                                          \
    } while (0)

static void every_chunk_once(size_t n, size_t grain)
{
    std::vector<std::atomic<int>> hits(n);
    for (auto &h : hits)
        h.store(0);
    parallel_range(n, grain, [&](size_t i) { hits[i].fetch_add(1); });
    for (size_t i = 0; i < n; ++i)
        CHECK(hits[i].load() == 1);
}

int main()
{
    for (size_t n : {0, 1, 2, 3, 17, 1000, 65537})
        for (size_t g : {1, 7, 1024})
            every_chunk_once(n, g);

    // a loop nested in a chunk (threads of its own) and the outer loop's sums
    {
        std::vector<long> outer(8, 0);
        for_chunks(8, [&](size_t c) {
            std::vector<long> inner(16, 0);
            for_chunks(16, [&](size_t k) { inner[k] = static_cast<long>(c * 100 + k); });
            long s = 0;
            for (long v : inner)
                s += v;
            outer[c] = s;
        });
        for (size_t c = 0; c < 8; ++c)
            CHECK(outer[c] == static_cast<long>(16 * c * 100 + 120));
    }

    // loops from several threads at once: one gets the pool, the others start
    // threads of their own
    {
        std::vector<std::thread> callers;
        std::atomic<int> bad{0};
        for (int t = 0; t < 4; ++t)
            callers.emplace_back([&, t]() {
                for (int rep = 0; rep < 200; ++rep) {
                    std::vector<int> out(64, -1);
                    for_chunks(64, [&](size_t c) { out[c] = static_cast<int>(c) + t; });
                    for (size_t c = 0; c < 64; ++c)
                        if (out[c] != static_cast<int>(c) + t)
                            bad.fetch_add(1);
                }
            });
        for (auto &th : callers)
            th.join();
        CHECK(bad.load() == 0);
    }

    // an exception in a chunk, on whichever thread runs it, reaches the
    // caller; the pool stays usable
    for (size_t throw_at : {0, 5, 63}) {
        bool caught = false;
        std::atomic<int> ran{0};
        try {
            for_chunks(64, [&](size_t c) {
                ran.fetch_add(1);
                if (c == throw_at)
                    throw std::runtime_error("chunk");
            });
        } catch (const std::runtime_error &) {
            caught = true;
        }
        CHECK(caught);
        CHECK(ran.load() <= 64);
        every_chunk_once(1000, 3);
    }

    // cost of one loop once the pool runs
    const int reps = 2000;
    std::vector<double> sink(64, 0.0);
    auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps; ++r)
        for_chunks(64, [&](size_t c) { sink[c] += 1.0; });
    auto t1 = std::chrono::steady_clock::now();
    for (double v : sink)
        CHECK(v == reps);
    std::printf("per loop %.1f us\n",
                std::chrono::duration<double, std::micro>(t1 - t0).count() / reps);
    if (failures)
        return 1;
    std::printf("ok\n");
    return 0;
}
