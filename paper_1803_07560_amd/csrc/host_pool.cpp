// The host worker pool behind for_chunks (host_pool.h).
#include "host_pool.h"

#include <chrono>
#include <condition_variable>
#include <exception>
#include <mutex>

#include <unistd.h>

namespace bfi {

namespace {

// Loops come in bursts (a round of the adaptive driver runs a few dozen):
// a thread that finds no work yet polls for this long before it sleeps, so
// the next loop starts without waking anyone.
constexpr auto kSpin = std::chrono::microseconds(100);

template <class P>
void spin_until(P ready)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned i = 1; !ready(); ++i) {
        if ((i & 63) == 0 && std::chrono::steady_clock::now() - t0 > kSpin)
            return;
#if defined(__x86_64__)
        __builtin_ia32_pause();
#endif
    }
}

// Set on the pool's threads, and on a caller while it runs a loop's chunks: a
// loop nested in a chunk then starts threads of its own.
thread_local bool t_in_pool_loop = false;

// One loop at a time: the caller publishes the loop under the lock and bumps
// the generation, the first `want` workers take chunks from a shared counter
// alongside it, and the last of them to finish signals the caller.  Between
// loops the workers poll briefly, then sleep.
class ChunkPool {
public:
    ChunkPool() : pid_(getpid())
    {
        const size_t hw = std::max<size_t>(1, std::thread::hardware_concurrency());
        const size_t workers = std::min(hw, kMaxHostThreads) - 1;
        threads_.reserve(workers);
        for (size_t k = 0; k < workers; ++k)
            threads_.emplace_back([this, k]() { work(k); });
    }
    ~ChunkPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_.store(true);
        }
        wake_.notify_all();
        for (auto &t : threads_)
            t.join();
    }
    bool run(size_t nchunks, size_t nthreads, void (*fn)(void *, size_t), void *ctx)
    {
        if (t_in_pool_loop || getpid() != pid_ || threads_.empty())
            return false;  // nested, or a forked child (the object without the threads)
        std::unique_lock<std::mutex> job(job_mu_, std::try_to_lock);
        if (!job.owns_lock())
            return false;
        const size_t want = std::min(nthreads - 1, threads_.size());
        {
            std::lock_guard<std::mutex> lk(mu_);
            nchunks_ = nchunks;
            fn_ = fn;
            ctx_ = ctx;
            next_.store(0);
            want_ = want;
            active_.store(want);
            gen_.store(gen_.load() + 1);
        }
        wake_.notify_all();
        t_in_pool_loop = true;
        chunks(nchunks, fn, ctx);
        t_in_pool_loop = false;
        std::exception_ptr err;
        spin_until([this]() { return active_.load() == 0; });
        {
            std::unique_lock<std::mutex> lk(mu_);
            done_.wait(lk, [this]() { return active_.load() == 0; });
            err = err_;
            err_ = nullptr;
        }
        if (err)
            std::rethrow_exception(err);
        return true;
    }

private:
    void work(size_t index)
    {
        t_in_pool_loop = true;
        uint64_t seen = 0;
        for (;;) {
            size_t nchunks;
            void (*fn)(void *, size_t);
            void *ctx;
            spin_until([&]() { return stop_.load() || gen_.load() != seen; });
            {
                std::unique_lock<std::mutex> lk(mu_);
                wake_.wait(lk, [&]() { return stop_.load() || gen_.load() != seen; });
                if (stop_.load())
                    return;
                seen = gen_.load();
                if (index >= want_)
                    continue;
                nchunks = nchunks_;
                fn = fn_;
                ctx = ctx_;
            }
            chunks(nchunks, fn, ctx);
            if (active_.fetch_sub(1) == 1) {
                std::lock_guard<std::mutex> lk(mu_);
                done_.notify_one();
            }
        }
    }
    // Take chunks until none is left.  A chunk that throws stops the hand-out
    // and its exception (the first one) goes to the caller once every thread
    // of the loop is done with the loop's state.
    void chunks(size_t nchunks, void (*fn)(void *, size_t), void *ctx)
    {
        try {
            for (size_t c = next_++; c < nchunks; c = next_++)
                fn(ctx, c);
        } catch (...) {
            next_.store(nchunks);
            std::lock_guard<std::mutex> lk(mu_);
            if (!err_)
                err_ = std::current_exception();
        }
    }

    const pid_t pid_;
    std::mutex job_mu_;  // held by the caller for the whole loop
    std::mutex mu_;      // guards the fields below and the sleeps
    std::condition_variable wake_, done_;
    std::atomic<uint64_t> gen_{0};  // written under mu_, polled without it
    std::atomic<size_t> active_{0};  // workers of the loop not done yet
    size_t nchunks_ = 0, want_ = 0;
    void (*fn_)(void *, size_t) = nullptr;
    void *ctx_ = nullptr;
    std::atomic<bool> stop_{false};
    std::exception_ptr err_;
    std::atomic<size_t> next_{0};
    std::vector<std::thread> threads_;
};

}  // namespace

bool pool_run(size_t nchunks, size_t nthreads, void (*fn)(void *, size_t), void *ctx)
{
    static ChunkPool pool;
    return pool.run(nchunks, nthreads, fn, ctx);
}

}  // namespace bfi
