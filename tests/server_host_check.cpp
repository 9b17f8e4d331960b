// Host build of the product server's worker (gfq_serve_core.h) with a fake executor: device
// time is simulated, the arena hands out ranges of a fake address space, and the executor
// checks that no two batches in flight hold overlapping ranges.  Four submitter threads and
// a polling thread drive it (the test builds this file with ThreadSanitizer and with
// AddressSanitizer + UndefinedBehaviorSanitizer).  Prints "ok <name>" per scenario, or
// "FAIL ..." and exits 1.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "gfq_serve_core.h"

using namespace gfq;
typedef std::chrono::steady_clock Clock;

static void fail(const char *what, long long a = 0, long long b = 0) {
    printf("FAIL %s %lld %lld\n", what, a, b);
    fflush(stdout);
    exit(1);
}

struct FakeReq {
    double arrival = 0;
    size_t bytes = 0, items = 0;
    uint64_t tag = 0;
    double work_us = 0;              // simulated device time
};

// Fake device memory for the arena: chunks at distinct bases, checked on return.
struct FakeMemory {
    std::mutex mu;                   // the arena runs on the worker; the checker reads at the end
    std::map<uintptr_t, size_t> live;
    uintptr_t next = (uintptr_t)1 << 40;
    size_t held = 0, peak = 0;
    bool grow(size_t size, uintptr_t *out) {
        std::lock_guard<std::mutex> lk(mu);
        *out = next;
        next += (uintptr_t)1 << 40;
        live[*out] = size;
        held += size;
        peak = std::max(peak, held);
        return true;
    }
    void shrink(uintptr_t p) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = live.find(p);
        if (it == live.end()) fail("shrink of an unknown chunk");
        held -= it->second;
        live.erase(it);
    }
};

struct FakeExec {
    typedef std::vector<std::pair<FakeReq, uintptr_t>> Batch;
    struct Slot {
        Clock::time_point done_at;
        bool pending = false, hung = false, retired = false;
        std::vector<std::pair<uintptr_t, size_t>> ranges;
    };
    std::vector<Slot> sl;
    uint64_t hang_tag = ~0ull, fail_tag = ~0ull;   // a batch holding this tag hangs / fails to launch
    int launches = 0, retires = 0;
    std::set<std::pair<uintptr_t, size_t>> in_flight;

    explicit FakeExec(int n) : sl(n) {}
    int slots() const { return (int)sl.size(); }
    int launch(int i, const Batch &b) {
        Slot &s = sl[i];
        if (s.pending || s.retired) fail("launch on a busy or retired slot", i);
        double us = 5.0;
        for (auto &rp : b) {
            if (rp.first.tag == fail_tag) return -8;
            // no range of this batch overlaps a range of a batch in flight
            const uintptr_t p = rp.second;
            const size_t n = Arena::round(rp.first.bytes);
            auto it = in_flight.lower_bound(std::make_pair(p, (size_t)0));
            if (it != in_flight.end() && it->first < p + n) fail("overlapping arena ranges", (long long)p);
            if (it != in_flight.begin() && std::prev(it)->first + std::prev(it)->second > p)
                fail("overlapping arena ranges", (long long)p);
            in_flight.insert(std::make_pair(p, n));
            s.ranges.push_back(std::make_pair(p, n));
            us += rp.first.work_us;
            s.hung = s.hung || rp.first.tag == hang_tag;
        }
        s.pending = true;
        s.done_at = Clock::now() + std::chrono::microseconds((int64_t)us);
        launches++;
        return 0;
    }
    int poll(int i) {
        Slot &s = sl[i];
        if (!s.pending) fail("poll of an idle slot", i);
        if (s.hung || Clock::now() < s.done_at) return 1;
        s.pending = false;
        for (auto &r : s.ranges) in_flight.erase(r);
        s.ranges.clear();
        return 0;
    }
    void drain(int i) {
        Slot &s = sl[i];
        s.pending = false;
        for (auto &r : s.ranges) in_flight.erase(r);
        s.ranges.clear();
    }
    void retire(int i) {
        sl[i].retired = true;
        retires++;
    }
};

struct Run {
    int completed_ok = 0, completed_hip = 0, completed_nomem = 0;
    std::map<uint64_t, int> seen;
};

// Drive a core: `submitters` threads submit `per_thread` requests each in small groups with
// arrivals spread over `spread_us`; one thread polls until every accepted request has
// completed (or, once the core has failed, until nothing more arrives for a while).
static Run drive(ServeCore<FakeReq, FakeExec> &core, int submitters, int per_thread, double spread_us,
                 unsigned seed, std::atomic<int> *accepted) {
    std::vector<std::thread> th;
    std::atomic<int> finished{0};
    for (int t = 0; t < submitters; t++) {
        th.emplace_back([&, t] {
            std::mt19937_64 rng(seed * 131 + t);
            std::uniform_real_distribution<double> u(0.0, 1.0);
            for (int i = 0; i < per_thread;) {
                std::vector<FakeReq> group;
                const int g = 1 + (int)(u(rng) * 8);
                for (int j = 0; j < g && i < per_thread; j++, i++) {
                    FakeReq r;
                    r.tag = (uint64_t)t * 1000000 + i;
                    r.bytes = 256 + (size_t)(u(rng) * u(rng) * (4 << 20));
                    r.items = 1 + (size_t)(u(rng) * 300);
                    r.work_us = 20.0 + u(rng) * 200.0;
                    r.arrival = core.now() + u(rng) * spread_us;
                    group.push_back(r);
                }
                const int n = (int)group.size();
                if (core.submit(group)) *accepted += n;
                std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(u(rng) * 200)));
            }
            finished++;
        });
    }
    Run run;
    std::vector<ServeCompletion> buf(512);
    int idle_polls = 0;
    while (true) {
        const int n = core.poll(buf.data(), (int)buf.size(), 20000.0);
        for (int i = 0; i < n; i++) {
            const ServeCompletion &c = buf[i];
            if (run.seen[c.tag]++) fail("request completed twice", (long long)c.tag);
            if (c.status == kServeOk) run.completed_ok++;
            else if (c.status == kServeHip) run.completed_hip++;
            else if (c.status == kServeNoMem) run.completed_nomem++;
            else fail("unexpected status", c.status);
            if (c.done_us < c.arrival_us) fail("completed before its arrival", (long long)c.tag);
        }
        idle_polls = n ? 0 : idle_polls + 1;
        const int done = run.completed_ok + run.completed_hip + run.completed_nomem;
        if (finished == submitters && done == accepted->load()) break;
        if (idle_polls > 250) fail("no completion for 5 s", done, accepted->load());
    }
    for (auto &x : th) x.join();
    return run;
}

int main() {
    // 1. ordinary traffic: every request completes once, OK, budget respected
    for (unsigned seed : {1u, 2u}) {
        FakeMemory mem;
        FakeExec ex(3);
        Arena arena((size_t)64 << 20, (size_t)16 << 20, [&](size_t s, uintptr_t *p) { return mem.grow(s, p); },
                    [&](uintptr_t p) { mem.shrink(p); });
        ServeLimits lim;
        lim.max_batch = 64;
        lim.max_items = 4096;
        std::atomic<int> accepted{0};
        Run run;
        {
            // each core on the heap: its mutex never shares an address with an earlier one
            std::unique_ptr<ServeCore<FakeReq, FakeExec>> cp(new ServeCore<FakeReq, FakeExec>(ex, arena, lim));
            ServeCore<FakeReq, FakeExec> &core = *cp;
            core.start();
            run = drive(core, 4, 600, 20000.0, seed, &accepted);
            core.stop();
            if (core.a_peak > ((size_t)64 << 20)) fail("arena above budget", (long long)core.a_peak.load());
        }
        if (accepted != 2400 || run.completed_ok != 2400) fail("traffic: completions", run.completed_ok, accepted);
        if (mem.peak > ((size_t)64 << 20)) fail("device memory above budget", (long long)mem.peak);
        if (!ex.in_flight.empty()) fail("ranges left in flight");
        printf("ok traffic seed=%u launches=%d\n", seed, ex.launches);
    }
    // 2. a launch that fails: its batch completes with the HIP status, the core fails, and no
    //    later submission is accepted
    {
        FakeMemory mem;
        FakeExec ex(2);
        ex.fail_tag = 1000000 + 37;
        Arena arena((size_t)64 << 20, (size_t)16 << 20, [&](size_t s, uintptr_t *p) { return mem.grow(s, p); },
                    [&](uintptr_t p) { mem.shrink(p); });
        ServeLimits lim;
        std::atomic<int> accepted{0};
        std::unique_ptr<ServeCore<FakeReq, FakeExec>> cp(new ServeCore<FakeReq, FakeExec>(ex, arena, lim));
        ServeCore<FakeReq, FakeExec> &core = *cp;
        core.start();
        Run run = drive(core, 2, 300, 5000.0, 7, &accepted);
        if (run.completed_hip < 1) fail("launch failure not reported");
        if (!core.failed()) fail("core not failed after a launch failure");
        std::vector<FakeReq> late(1);
        late[0].tag = 99;
        if (core.submit(late)) fail("submission accepted after failure");
        core.stop();
        printf("ok launch_failure hip=%d ok=%d\n", run.completed_hip, run.completed_ok);
    }
    // 3. a batch that never completes: the watchdog fails its requests, retires its slot and
    //    keeps its arena ranges out of use; the other slots keep serving what was queued
    {
        FakeMemory mem;
        FakeExec ex(3);
        ex.hang_tag = 2 * 1000000 + 11;
        Arena arena((size_t)64 << 20, (size_t)16 << 20, [&](size_t s, uintptr_t *p) { return mem.grow(s, p); },
                    [&](uintptr_t p) { mem.shrink(p); });
        ServeLimits lim;
        lim.max_batch = 16;
        lim.watchdog_us = 50000.0;
        std::atomic<int> accepted{0};
        std::unique_ptr<ServeCore<FakeReq, FakeExec>> cp(new ServeCore<FakeReq, FakeExec>(ex, arena, lim));
        ServeCore<FakeReq, FakeExec> &core = *cp;
        core.start();
        Run run = drive(core, 3, 200, 5000.0, 11, &accepted);
        core.stop();
        if (ex.retires != 1) fail("watchdog retired slots", ex.retires);
        if (!ex.sl[0].retired && !ex.sl[1].retired && !ex.sl[2].retired) fail("no retired slot");
        if (run.completed_hip < 1 || run.seen.count(ex.hang_tag) == 0) fail("hung request not failed");
        if (!core.failed()) fail("core not failed after the watchdog");
        printf("ok watchdog hip=%d ok=%d\n", run.completed_hip, run.completed_ok);
    }
    printf("ok all\n");
    return 0;
}
