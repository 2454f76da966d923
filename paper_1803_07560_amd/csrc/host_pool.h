// Parallel loops of the host runtime over a persistent worker pool.  Plain
// C++ (no HIP): the adaptive driver's passes over the leaves, finalize and
// the ranking run their chunks here.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstddef>
#include <thread>
#include <type_traits>
#include <vector>

namespace bfi {

// Host threads one parallel loop may use: one GPU's share of the host.
constexpr size_t kMaxHostThreads = 16;

// Run fn(ctx, chunk) for chunks 0 .. nchunks-1 on the calling thread and
// nthreads - 1 threads of a pool that persists for the process (created at
// first use); returns false without running anything when the pool is taken
// (another thread's loop, or a loop nested in one) or was inherited through a
// fork.
bool pool_run(size_t nchunks, size_t nthreads, void (*fn)(void *, size_t), void *ctx);

// Run body(chunk) for chunks 0 .. nchunks-1, on up to kMaxHostThreads host
// threads when there are several; each chunk writes its own outputs, so results
// do not depend on the number of threads.  The threads come from the pool;
// when it is taken they are started for this loop alone.
template <class F>
void for_chunks(size_t nchunks, F &&body)
{
    const size_t hw = std::max<size_t>(1, std::thread::hardware_concurrency());
    const size_t nthreads = std::min<size_t>({nchunks, hw, kMaxHostThreads});
    if (nthreads <= 1) {
        for (size_t c = 0; c < nchunks; ++c)
            body(c);
        return;
    }
    using B = std::remove_reference_t<F>;
    auto call = [](void *p, size_t c) { (*static_cast<B *>(p))(c); };
    if (pool_run(nchunks, nthreads, call, const_cast<void *>(static_cast<const void *>(&body))))
        return;
    std::atomic<size_t> next{0};
    auto worker = [&]() {
        for (size_t c = next++; c < nchunks; c = next++)
            body(c);
    };
    std::vector<std::thread> pool;
    pool.reserve(nthreads - 1);
    for (size_t t = 1; t < nthreads; ++t)
        pool.emplace_back(worker);
    worker();
    for (auto &th : pool)
        th.join();
}

// Apply body(i) to i in [0, n) in parallel chunks of `grain` (serially when n
// is below two grains).
template <class F>
void parallel_range(size_t n, size_t grain, F &&body)
{
    const size_t nchunks = (n + grain - 1) / grain;
    for_chunks(nchunks, [&](size_t c) {
        const size_t i1 = std::min(n, (c + 1) * grain);
        for (size_t i = c * grain; i < i1; ++i)
            body(i);
    });
}

}  // namespace bfi
