// fused_schedule_sim.cpp -- host threads play the workgroups of the fused X-Y
// pass (tests/test_fused_schedule.py).  The work order is the kernel's own
// (pf::fused_item, fused_schedule.h); the protocol is the kernel's: a thread
// takes the next ticket of its queue, a consumer item waits until every
// producer item of its plane has been published, a producer item publishes
// itself when done.  Checked for each configuration on the command line:
//   * statically: every (plane, kind, index) item occurs exactly once, and in
//     each queue all producer items of a plane precede its consumer items;
//   * dynamically: with fewer threads per queue than items and random delays,
//     every item is processed exactly once and no wait exceeds its bound (a
//     wait that never ends would be a deadlock).
// Usage: fused_schedule_sim nz nq lag pi ci threads_per_queue [seed]
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "fused_schedule.h"

int main(int argc, char **argv) {
    if (argc < 7) return 2;
    const int nz = atoi(argv[1]), nq = atoi(argv[2]), lag = atoi(argv[3]), pi = atoi(argv[4]), ci = atoi(argv[5]);
    const int tpq = atoi(argv[6]);
    const unsigned seed = argc > 7 ? (unsigned)atoi(argv[7]) : 1u;
    int bad = 0;
    // static checks
    std::vector<int> seen((size_t)nz * (pi + ci), 0);
    for (int q = 0; q < nq; ++q) {
        const int np = (nz - q + nq - 1) / nq;
        std::vector<int> produced(np > 0 ? np : 1, 0);
        int k = 0, kind, j, idx;
        for (; pf::fused_item(k, np, lag, pi, ci, kind, j, idx); ++k) {
            if (j < 0 || j >= np || idx < 0 || idx >= (kind ? ci : pi)) {
                ++bad;
                break;
            }
            const int plane = q + j * nq;
            seen[(size_t)plane * (pi + ci) + (kind ? pi + idx : idx)] += 1;
            if (kind == 0) produced[j] += 1;
            else if (produced[j] != pi) ++bad;  // a consumer before all of its plane's producers
        }
        if (k != np * (pi + ci)) ++bad;
    }
    for (int c : seen)
        if (c != 1) ++bad;
    if (bad) {
        printf("static check failed: %d\n", bad);
        return 1;
    }
    // dynamic: threads play workgroups; queue of thread b is b mod nq
    std::vector<std::atomic<int>> tickets(nq), done(nz);
    std::vector<std::atomic<int>> count((size_t)nz * (pi + ci));
    for (auto &t : tickets) t = 0;
    for (auto &d : done) d = 0;
    for (auto &c : count) c = 0;
    std::atomic<int> timeouts{0};
    std::vector<std::thread> th;
    for (int b = 0; b < nq * tpq; ++b)
        th.emplace_back([&, b]() {
            std::mt19937 rng(seed * 7919u + (unsigned)b);
            const int q = b % nq;
            const int np = (nz - q + nq - 1) / nq;
            while (true) {
                const int k = tickets[q].fetch_add(1);
                int kind, j, idx;
                if (!pf::fused_item(k, np, lag, pi, ci, kind, j, idx)) break;
                const int plane = q + j * nq;
                if (kind == 1) {
                    const auto t0 = std::chrono::steady_clock::now();
                    while (done[plane].load(std::memory_order_acquire) < pi) {
                        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(10)) {
                            timeouts.fetch_add(1);
                            break;
                        }
                        std::this_thread::yield();
                    }
                }
                if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
                count[(size_t)plane * (pi + ci) + (kind ? pi + idx : idx)].fetch_add(1);
                if (kind == 0) done[plane].fetch_add(1, std::memory_order_release);
            }
        });
    for (auto &t : th) t.join();
    for (auto &c : count)
        if (c.load() != 1) ++bad;
    printf("nz %d nq %d lag %d pi %d ci %d threads/queue %d: %d items, %d timeouts, %d bad\n", nz, nq, lag, pi, ci,
           tpq, nz * (pi + ci), timeouts.load(), bad);
    return bad || timeouts.load() ? 1 : 0;
}
