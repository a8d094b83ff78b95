// The host thread pool of the update resolution (csrc/bsim_resolve.h):
// every share of a job runs exactly once, whatever the share count against
// the pool's workers; callers on several threads at once get their jobs
// done (the pool takes one job at a time, the others start threads of
// their own); an exception in any share reaches the caller, after every
// share has ended, and the pool goes on working.  Built with the address,
// undefined-behaviour and thread sanitizers by tests/test_sanitizers.py.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <thread>
#include <vector>

#include "bsim_resolve.h"

using bsim::host_parallel;
using bsim::HostPool;

static int g_checks = 0;

#define CHECK(cond, what)                                          \
    do {                                                           \
        if (!(cond)) {                                             \
            std::printf("FAIL: %s (line %d)\n", what, __LINE__);   \
            std::exit(1);                                          \
        }                                                          \
        g_checks++;                                                \
    } while (0)

// Run a job of T shares and check that share t ran exactly once.
static void once_each(HostPool* pool, size_t T) {
    std::vector<std::atomic<int>> hits(T);
    for (auto& h : hits) h.store(0);
    host_parallel(T, [&](size_t t) { hits[t].fetch_add(1); }, pool);
    for (size_t t = 0; t < T; t++) CHECK(hits[t].load() == 1, "every share runs once");
}

int main(int argc, char** argv) {
    const unsigned seed = argc > 1 ? static_cast<unsigned>(std::atoi(argv[1])) : 1;
    std::srand(seed);
    for (size_t workers : {0u, 1u, 3u, 7u}) {
        HostPool pool(workers);
        for (size_t T = 0; T <= 12; T++) once_each(&pool, T);
        once_each(nullptr, 5);  // no pool: threads of the call's own
        // several callers at once: one job on the pool at a time
        std::vector<std::thread> callers;
        std::atomic<long> total{0};
        for (int c = 0; c < 4; c++)
            callers.emplace_back([&, c] {
                for (int r = 0; r < 60; r++) {
                    const size_t T = 1 + static_cast<size_t>((c * 7 + r * 3 + static_cast<int>(seed)) % 9);
                    std::vector<int> hits(T, 0);  // share t writes only hits[t]
                    host_parallel(T, [&](size_t t) { hits[t]++; }, &pool);
                    long sum = 0;
                    for (int h : hits) sum += h;
                    if (sum != static_cast<long>(T)) std::abort();
                    total += sum;
                }
            });
        for (auto& t : callers) t.join();
        CHECK(total.load() > 0, "concurrent callers completed");
        // an exception in a worker's share and in the caller's share
        for (size_t bad : {size_t(0), size_t(2)}) {
            std::atomic<int> ran{0};
            bool caught = false;
            try {
                host_parallel(4, [&](size_t t) {
                    ran.fetch_add(1);
                    if (t == bad) throw std::runtime_error("share failed");
                }, &pool);
            } catch (const std::runtime_error&) {
                caught = true;
            }
            CHECK(caught, "a share's exception reaches the caller");
            CHECK(ran.load() == 4, "every share ran before the call returned");
            once_each(&pool, 6);  // and the pool still works
        }
    }
    // the process-wide pool
    for (size_t T = 1; T <= 9; T++) once_each(&bsim::shared_host_pool(), T);
    std::printf("ok %d\n", g_checks);
    return 0;
}
