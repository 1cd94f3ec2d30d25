// Checks run_threads (analysis.hpp): every share runs, every thread is
// joined, and an exception thrown by a worker share (here std::bad_alloc,
// the failure an allocation inside the analysis would raise) reaches the
// calling thread instead of terminating the process.
#include <atomic>
#include <cstdio>
#include <new>
#include <stdexcept>

#include "analysis.hpp"

int main() {
    using ckkt::run_threads;
    int fails = 0;
    for (int nthreads : {1, 2, 6}) {
        std::atomic<int> ran{0};
        run_threads(nthreads, [&](int) { ran++; });
        if (ran != nthreads) { std::printf("shares ran %d of %d\n", ran.load(), nthreads); fails++; }
        for (int thrower = 0; thrower < nthreads; ++thrower) {
            std::atomic<int> done{0};
            bool caught = false;
            try {
                run_threads(nthreads, [&](int t) {
                    if (t == thrower) throw std::bad_alloc();
                    done++;
                });
            } catch (const std::bad_alloc&) {
                caught = true;
            }
            if (!caught || done != nthreads - 1) {
                std::printf("nthreads %d thrower %d: caught %d done %d\n", nthreads, thrower, (int)caught,
                            done.load());
                fails++;
            }
        }
        // every share throws: exactly one exception reaches the caller
        int caught = 0;
        try {
            run_threads(nthreads, [&](int t) { throw std::runtime_error("share " + std::to_string(t)); });
        } catch (const std::runtime_error&) {
            caught++;
        }
        if (caught != 1) { std::printf("all throw: caught %d\n", caught); fails++; }
    }
    std::printf("run_threads %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
