// Host build of the server's scheduling core (gfq_sched.h) against an independent model:
// a fake device address space, a shadow list of live ranges, and an event-driven replay
// of the server loop.  Prints one "ok <name> ..." line per check, or "FAIL ..." and exits 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "gfq_sched.h"

using namespace gfq;

static void fail(const char *what, long long a = 0, long long b = 0) {
    printf("FAIL %s %lld %lld\n", what, a, b);
    exit(1);
}

// Fake device memory: chunks at distinct 1 TiB-aligned bases, checked on return.
struct FakeDevice {
    std::map<uintptr_t, size_t> live;   // base -> size
    uintptr_t next = (uintptr_t)1 << 40;
    size_t total = 0, peak = 0, grows = 0;
    bool grow(size_t size, uintptr_t *out) {
        *out = next;
        next += (uintptr_t)1 << 40;
        live[*out] = size;
        total += size;
        peak = std::max(peak, total);
        grows++;
        return true;
    }
    void shrink(uintptr_t p) {
        auto it = live.find(p);
        if (it == live.end()) fail("shrink of unknown chunk");
        total -= it->second;
        live.erase(it);
    }
    bool inside(uintptr_t p, size_t n) const {
        auto it = live.upper_bound(p);
        if (it == live.begin()) return false;
        --it;
        return p >= it->first && p + n <= it->first + it->second;
    }
};

static Arena make_arena(FakeDevice &d, size_t budget, size_t chunk) {
    return Arena(budget, chunk, [&d](size_t s, uintptr_t *p) { return d.grow(s, p); },
                 [&d](uintptr_t p) { d.shrink(p); });
}

// Random alloc / release against a shadow set of live ranges.
static void check_arena_random(unsigned seed) {
    std::mt19937_64 rng(seed);
    FakeDevice dev;
    const size_t budget = (size_t)64 << 20, chunk = (size_t)8 << 20;
    {
        Arena a = make_arena(dev, budget, chunk);
        std::map<uintptr_t, size_t> shadow;   // start -> rounded size
        size_t shadow_bytes = 0, allocs = 0, refusals = 0;
        for (int step = 0; step < 200000; step++) {
            const bool do_alloc = shadow.empty() || (rng() % 100) < 55;
            if (do_alloc) {
                const int cls = (int)(rng() % 4);
                size_t bytes = cls == 0 ? 1 + rng() % 4096 : cls == 1 ? 1 + rng() % (1 << 20)
                             : cls == 2 ? 1 + rng() % (6 << 20) : 1 + rng() % (20 << 20);
                uintptr_t p = 0;
                if (!a.alloc(bytes, &p)) {
                    refusals++;
                    // a refusal must be justified: no single free extent fits and no room to grow
                    if (Arena::round(bytes) <= budget - a.held()) fail("refused with room to grow", bytes, a.held());
                    continue;
                }
                const size_t r = Arena::round(bytes);
                if (p % Arena::kAlign) fail("misaligned", p);
                if (!dev.inside(p, r)) fail("outside every chunk", p, r);
                auto nx = shadow.lower_bound(p);
                if (nx != shadow.end() && nx->first < p + r) fail("overlaps next", p, nx->first);
                if (nx != shadow.begin()) {
                    auto pv = std::prev(nx);
                    if (pv->first + pv->second > p) fail("overlaps previous", p, pv->first);
                }
                shadow[p] = r;
                shadow_bytes += r;
                allocs++;
            } else {
                auto it = shadow.begin();
                std::advance(it, rng() % shadow.size());
                a.release(it->first, it->second);
                shadow_bytes -= it->second;
                shadow.erase(it);
            }
            if (a.in_use() != shadow_bytes) fail("in_use mismatch", a.in_use(), shadow_bytes);
            if (a.held() > budget || dev.total != a.held()) fail("budget", a.held(), dev.total);
        }
        for (auto &kv : shadow) a.release(kv.first, kv.second);
        if (a.in_use() != 0) fail("in_use after release", a.in_use());
        // every chunk coalesced back to one extent: a chunk-sized request fits without growing
        const size_t grows = dev.grows;
        uintptr_t p;
        if (a.chunks() > 0 && !a.alloc(chunk, &p)) fail("no whole-chunk extent after release");
        if (dev.grows != grows) fail("grew although a coalesced chunk was free");
        printf("ok arena_random seed=%u allocs=%zu refusals=%zu chunks=%zu peak_held=%zu\n", seed, allocs,
               refusals, a.chunks(), dev.peak);
    }
    if (!dev.live.empty()) fail("chunks not returned by the destructor");
}

// A request larger than every chunk but within the budget is placed after an idle reset.
static void check_arena_reset() {
    FakeDevice dev;
    Arena a = make_arena(dev, 100 << 20, 30 << 20);
    std::vector<uintptr_t> ps;
    for (int i = 0; i < 3; i++) {
        uintptr_t p;
        if (!a.alloc(30 << 20, &p)) fail("reset: fill");
        ps.push_back(p);
    }
    uintptr_t p;
    if (a.alloc(60 << 20, &p)) fail("reset: should not fit while held");
    for (uintptr_t x : ps) a.release(x, 30 << 20);
    if (a.alloc(60 << 20, &p)) fail("reset: should not fit in 30 MiB chunks");
    a.reset();
    if (!dev.live.empty()) fail("reset: chunks still live");
    if (!a.alloc(60 << 20, &p)) fail("reset: does not fit after reset");
    if (a.alloc(101 << 20, &p)) fail("reset: over budget accepted");
    a.release(p, 60 << 20);
    printf("ok arena_reset\n");
}

// Earliest arrival first; equal arrivals in submission order; eligibility by time.
static void check_queue() {
    ArrivalQueue<int> q;
    std::mt19937_64 rng(7);
    std::vector<std::pair<double, int>> ref;
    for (int i = 0; i < 5000; i++) {
        const double t = (double)(rng() % 300);
        q.push(t, i);
        ref.push_back({t, i});
    }
    std::stable_sort(ref.begin(), ref.end(), [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
        return x.first < y.first;
    });
    if (q.ready(-1.0)) fail("queue: ready before any arrival");
    size_t i = 0;
    for (double now = 0; now < 300; now += 1.0) {
        while (q.ready(now)) {
            if (q.front() != ref[i].second || q.front_arrival() != ref[i].first) fail("queue order", i, q.front());
            if (ref[i].first > now) fail("queue: early release");
            q.pop();
            i++;
        }
        if (i < ref.size() && ref[i].first <= now) fail("queue: eligible request held back", i);
    }
    if (!q.empty() || i != ref.size()) fail("queue: leftovers");
    printf("ok queue\n");
}

// Event-driven replay of the server loop: Poisson arrivals, a slot limit, batches formed by
// admit_batch, service time proportional to a batch's work.  Checks that every request
// completes exactly once, admission follows arrival order, batch limits hold, the arena
// never exceeds its budget and is empty at the end.
struct Req {
    int id;
    double arrival;
    size_t bytes, items;
    double work;
};

static void check_server_replay(unsigned seed, size_t budget, int slots, int max_batch, size_t max_items) {
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(1.0);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    FakeDevice dev;
    int done_count = 0;
    {
        Arena arena = make_arena(dev, budget, budget / 8);
        ArrivalQueue<Req> queue;
        const int N = 20000;
        std::vector<Req> reqs(N);
        double t = 0;
        for (int i = 0; i < N; i++) {
            t += gap(rng);
            const double n = std::exp(std::log(128.0) + u(rng) * (std::log(4096.0) - std::log(128.0)));
            reqs[i] = Req{i, t, (size_t)(n * n * 0.9), (size_t)std::ceil(n / 256) * (size_t)std::ceil(n / 512),
                          n * n * n * 1e-9};
        }
        // requests are submitted at their arrival time; the loop reacts to arrivals and completions
        struct Flight { double end; std::vector<std::pair<Req, uintptr_t>> reqs; };
        std::vector<Flight> flights;
        std::vector<int> done(N, 0);
        int next_submit = 0, last_admitted = -1, batches = 0;
        double now = 0, peak_batch = 0;
        while (done_count < N) {
            // next event: an arrival or a completion
            double t_next = next_submit < N ? reqs[next_submit].arrival : 1e300;
            for (auto &f : flights) t_next = std::min(t_next, f.end);
            now = std::max(now, t_next);
            while (next_submit < N && reqs[next_submit].arrival <= now) {
                queue.push(reqs[next_submit].arrival, reqs[next_submit]);
                next_submit++;
            }
            for (size_t j = 0; j < flights.size();) {
                if (flights[j].end <= now) {
                    for (auto &rp : flights[j].reqs) {
                        if (done[rp.first.id]++) fail("completed twice", rp.first.id);
                        arena.release(rp.second, rp.first.bytes);
                        done_count++;
                    }
                    flights.erase(flights.begin() + j);
                } else {
                    j++;
                }
            }
            while ((int)flights.size() < slots && queue.ready(now)) {
                std::vector<std::pair<Req, uintptr_t>> batch;
                const bool idle = flights.empty();
                const bool ok = admit_batch(queue, arena, now, max_batch, max_items,
                                            [](const Req &r) { return r.items; },
                                            [](const Req &r) { return r.bytes; }, &batch, idle);
                if (!ok) {
                    if (arena.in_use() != 0) fail("idle reset with memory in use");
                    arena.reset();
                    continue;
                }
                if (batch.empty()) break;
                if ((int)batch.size() > max_batch) fail("batch too large", batch.size());
                size_t items = 0;
                double work = 0;
                for (auto &rp : batch) {
                    if (rp.first.id != last_admitted + 1) fail("admission out of arrival order", rp.first.id, last_admitted);
                    last_admitted = rp.first.id;
                    if (rp.first.arrival > now) fail("admitted before arrival", rp.first.id);
                    items += rp.first.items;
                    work += rp.first.work;
                }
                if (batch.size() > 1 && items > max_items) fail("batch items over limit", items);
                if (arena.held() > budget) fail("arena over budget", arena.held());
                peak_batch = std::max(peak_batch, (double)batch.size());
                flights.push_back(Flight{now + 0.02 + work, batch});
                batches++;
            }
        }
        if (arena.in_use() != 0) fail("arena not empty at the end", arena.in_use());
        printf("ok server_replay seed=%u budget=%zu slots=%d batches=%d peak_batch=%.0f peak_held=%zu\n", seed,
               budget, slots, batches, peak_batch, dev.peak);
    }
    if (done_count != 20000) fail("not every request completed", done_count);
}

int main() {
    check_arena_random(1);
    check_arena_random(2);
    check_arena_reset();
    check_queue();
    check_server_replay(11, (size_t)1 << 40, 3, 256, 65536);   // budget never binds
    check_server_replay(12, (size_t)48 << 20, 3, 256, 65536);   // budget binds (about 3 large requests)
    check_server_replay(13, (size_t)16 << 20, 1, 4, 64);        // budget barely above the largest request
    printf("ok all\n");
    return 0;
}
