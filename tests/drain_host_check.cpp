// Host model of the persistent drain loop (gfq_drain.h, the same code the device kernel
// runs): workgroups are groups of threads with a barrier of their own and a shared slot, the
// queue head is an atomic, and an item's work calls the barrier a per-item number of times,
// as a tile calls it once per slab.  Checks, for several (workgroups, threads, items) and two
// launches with the head reset between them: every item is run exactly once, by every thread
// of one workgroup; every thread exits; nothing waits longer than a deadline (a watchdog
// thread fails the run instead of letting it hang).  Built with ThreadSanitizer and with
// AddressSanitizer + UndefinedBehaviorSanitizer.  Prints "ok <case>" per case and "ok all".
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "gfq_drain.h"

static void fail(const char *what, long long a = 0, long long b = 0) {
    printf("FAIL %s %lld %lld\n", what, a, b);
    fflush(stdout);
    std::_Exit(1);
}

// Reusable barrier of n threads (a generation count behind a mutex).
struct Barrier {
    std::mutex mu;
    std::condition_variable cv;
    int n, waiting = 0;
    uint64_t gen = 0;
    explicit Barrier(int count) : n(count) {}
    void wait() {
        std::unique_lock<std::mutex> lk(mu);
        const uint64_t g = gen;
        if (++waiting == n) {
            waiting = 0;
            gen++;
            cv.notify_all();
        } else {
            cv.wait(lk, [&] { return gen != g; });
        }
    }
};

struct Group {
    Barrier bar;
    uint32_t slot = 0;                 // workgroup-shared: ordered by the barriers alone
    explicit Group(int threads) : bar(threads) {}
};

struct Work {
    std::vector<int> barriers;                       // barriers inside each item
    std::unique_ptr<std::atomic<int>[]> runs;        // threads that ran each item
    std::unique_ptr<std::atomic<int>[]> owner;       // the workgroup that ran it (-1: none)
    explicit Work(size_t items) : barriers(items), runs(new std::atomic<int>[items]), owner(new std::atomic<int>[items]) {
        for (size_t i = 0; i < items; i++) {
            runs[i] = 0;
            owner[i] = -1;
        }
    }
};

struct HostCtx {
    Group &g;
    int group, t;
    std::atomic<uint32_t> &head;
    Work &w;
    bool leader() const { return t == 0; }
    void barrier() { g.bar.wait(); }
    uint32_t fetch_head() { return head.fetch_add(1u); }
    void slot_store(uint32_t v) { g.slot = v; }
    uint32_t slot_load() { return g.slot; }
    uint32_t uniform(uint32_t v) { return v; }
    void run(uint32_t it) {
        int expected = -1;
        if (!w.owner[it].compare_exchange_strong(expected, group) && expected != group)
            fail("item run by two workgroups", it, group);
        w.runs[it]++;
        for (int b = 0; b < w.barriers[it]; b++) barrier();
    }
};

static void drain_case(int groups, int threads, uint32_t items, unsigned seed) {
    std::atomic<uint32_t> head{0};
    for (int launch = 0; launch < 2; launch++) {
        head = 0;                                   // the reset that precedes every launch
        Work w(items ? items : 1);
        std::mt19937 rng(seed * 7 + launch);
        for (uint32_t i = 0; i < items; i++) w.barriers[i] = (int)(rng() % 9);
        std::vector<std::unique_ptr<Group>> gs;
        for (int gi = 0; gi < groups; gi++) gs.emplace_back(new Group(threads));
        std::atomic<int> finished{0};
        std::vector<std::thread> th;
        for (int gi = 0; gi < groups; gi++)
            for (int t = 0; t < threads; t++)
                th.emplace_back([&, gi, t] {
                    HostCtx c{*gs[gi], gi, t, head, w};
                    gfq::drain_queue(c, items);
                    finished++;
                });
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::seconds(30);
        while (finished.load() < groups * threads) {
            if (std::chrono::steady_clock::now() > deadline) fail("drain did not finish", finished.load(), groups * threads);
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
        }
        for (auto &x : th) x.join();
        for (uint32_t i = 0; i < items; i++)
            if (w.runs[i] != threads) fail("item not run by a whole workgroup once", i, w.runs[i].load());
        // every workgroup fetched until it saw an index past the end: items + groups fetches
        if (head.load() != items + (uint32_t)groups) fail("fetches", head.load(), items + groups);
    }
    printf("ok drain groups=%d threads=%d items=%u\n", groups, threads, items);
}

int main() {
    drain_case(8, 16, 1000, 1);
    drain_case(3, 64, 17, 2);
    drain_case(5, 8, 0, 3);
    drain_case(64, 4, 5, 4);
    drain_case(1, 32, 300, 5);
    printf("ok all\n");
    return 0;
}
