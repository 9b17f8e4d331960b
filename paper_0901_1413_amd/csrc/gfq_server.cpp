// gfq_server.cpp -- the product server: continuous batching of requests as they arrive.
//
// A worker thread owns the device side.  Requests wait in an arrival-ordered queue; while a
// slot (a stream with its own descriptor buffers) is free, the worker admits the eligible
// requests that fit the memory budget and the batch limits, stages their descriptors in the
// slot's pinned host buffer, and enqueues on the slot's stream: one copy of the
// descriptors, one conversion launch packing every uint8 operand, one work-list launch per
// (field, tile height) for the products, one conversion launch unpacking every uint8
// product, and an event.  Completed slots release their arena ranges and report their
// requests.  Slots overlap on the device, so a batch formed while others run fills the
// compute units they leave idle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "gfq.h"
#include "gfq_batch.h"
#include "gfq_host.h"
#include "gfq_internal.h"
#include "gfq_sched.h"

using namespace gfq;

namespace {

typedef std::chrono::steady_clock Clock;

constexpr int64_t kMaxSide = 65535;   // keeps every tile index of a request in 16 bits
constexpr size_t kNone = ~(size_t)0;

size_t rup(size_t x) { return (x + 255) & ~(size_t)255; }

struct Req {
    gfq_request r;
    double arrival = 0;
    size_t bytes = 0;                  // arena bytes (packed forms the server makes)
    size_t items = 0;                  // tile bound
    size_t offA = kNone, offB = kNone, offC = kNone;   // within the arena range
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    char *dev = nullptr;               // descriptors (staged part, then counts and times)
    char *host = nullptr;              // pinned staging mirror of the staged part
    u32 *done = nullptr;               // per-product tile counts (zero between launches)
    unsigned long long *times = nullptr;
    bool busy = false;
    double launch_us = 0;
    std::vector<std::pair<Req, uintptr_t>> reqs;
};

bool overlaps(uintptr_t a, size_t na, uintptr_t b, size_t nb) { return na && nb && a < b + nb && b < a + na; }

// Bytes spanned by an operand: packed size, or rows x ld uint8 (last row cols long).
size_t span(int q, int64_t rows, int64_t cols, int64_t ld, bool packed) {
    if (rows <= 0 || cols <= 0) return 0;
    return packed ? gfq_packed_bytes(q, rows, cols) : (size_t)((rows - 1) * ld + cols);
}

}  // namespace

struct gfq_server {
    gfq_server_opts o{};
    int device = 0;
    size_t staged_cap = 0;             // bytes of the staged part of a slot buffer
    size_t off_done = 0, off_times = 0, slot_bytes = 0;
    Clock::time_point t0;
    std::vector<Slot> slots;
    Arena *arena = nullptr;
    ArrivalQueue<Req> queue;           // worker only

    std::mutex mu;                     // guards incoming, completions, stop, failed
    std::condition_variable cv_work, cv_done;
    std::vector<Req> incoming;
    std::deque<gfq_completion> completions;
    bool stop = false;
    bool failed = false;
    std::thread worker;

    std::atomic<int64_t> submitted{0}, completed{0}, batches{0}, admitted{0}, max_batch_seen{0};
    std::atomic<size_t> a_in_use{0}, a_held{0}, a_peak{0};

    double now() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

namespace {

void complete(gfq_server *s, Slot &sl, int status) {
    const double t = s->now();
    std::vector<gfq_completion> out;
    out.reserve(sl.reqs.size());
    for (auto &rp : sl.reqs) {
        s->arena->release(rp.second, rp.first.bytes);
        gfq_completion c;
        c.tag = rp.first.r.tag;
        c.status = status;
        c.batch_size = (int)sl.reqs.size();
        c.arrival_us = rp.first.arrival;
        c.launch_us = sl.launch_us;
        c.done_us = t;
        out.push_back(c);
    }
    s->a_in_use = s->arena->in_use();
    sl.reqs.clear();
    sl.busy = false;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &c : out) s->completions.push_back(c);
        if (status != GFQ_OK) s->failed = true;
    }
    s->completed += (int64_t)out.size();
    s->cv_done.notify_all();
}

// Batched mode: stage descriptors and enqueue the launches of one batch on slot sl.
hipError_t launch_batch(gfq_server *s, Slot &sl) {
    const int nreq = (int)sl.reqs.size();
    std::vector<gfq_problem> probs(nreq);
    std::vector<ConvJob> pack, unpack;
    u32 pack_blocks = 0, unpack_blocks = 0;
    auto add_job = [](std::vector<ConvJob> &v, u32 &blocks, const void *src, void *dst, int64_t ld, int64_t rows,
                      int64_t cols, int q, int is_pack) {
        if (rows <= 0 || cols <= 0) return;
        ConvJob j;
        std::memset(&j, 0, sizeof j);
        j.src = src;
        j.dst = dst;
        j.ld = ld;
        j.rows = (int)rows;
        j.cols = (int)cols;
        j.W = words_of(cols);
        j.q = q;
        j.pack = is_pack;
        const uintptr_t u8p = (uintptr_t)(is_pack ? src : dst);
        j.aligned = (u8p % 16 == 0) && (ld % 16 == 0);
        j.first_block = blocks;
        blocks += conv_job_blocks(j);
        v.push_back(j);
    };
    for (int i = 0; i < nreq; i++) {
        const Req &rq = sl.reqs[i].first;
        const gfq_request &r = rq.r;
        char *base = (char *)sl.reqs[i].second;
        const void *A = rq.offA != kNone ? base + rq.offA : r.A;
        const void *B = rq.offB != kNone ? base + rq.offB : r.B;
        void *C = rq.offC != kNone ? base + rq.offC : r.C;
        if (rq.offA != kNone) add_job(pack, pack_blocks, r.A, (void *)A, r.lda, r.m, r.l, r.q, 1);
        if (rq.offB != kNone) add_job(pack, pack_blocks, r.B, (void *)B, r.ldb, r.l, r.n, r.q, 1);
        if (rq.offC != kNone) add_job(unpack, unpack_blocks, C, r.C, r.ldc, r.m, r.n, r.q, 0);
        probs[i] = gfq_problem{r.q, r.m, r.l, r.n, A, B, C};
    }
    std::vector<BatchProd> prods(std::max(nreq, 1));
    std::vector<BatchGroup> groups;
    size_t nitems = 0;
    plan_batch(nreq, probs.data(), nullptr, prods.data(), &groups, &nitems);

    // staged layout: pack jobs | unpack jobs | products | items
    const size_t o_unpack = rup(sizeof(ConvJob) * pack.size());
    const size_t o_prods = o_unpack + rup(sizeof(ConvJob) * unpack.size());
    const size_t o_items = o_prods + rup(sizeof(BatchProd) * nreq);
    const size_t used = o_items + sizeof(BatchItem) * nitems;
    if (used > s->staged_cap) return hipErrorInvalidValue;   // bounded by the batch limits
    char *h = sl.host;
    std::memcpy(h, pack.data(), sizeof(ConvJob) * pack.size());
    std::memcpy(h + o_unpack, unpack.data(), sizeof(ConvJob) * unpack.size());
    std::memcpy(h + o_prods, prods.data(), sizeof(BatchProd) * nreq);
    for (const BatchGroup &g : groups)
        std::memcpy(h + o_items + sizeof(BatchItem) * g.item_off, g.items.data(), sizeof(BatchItem) * g.items.size());
    hipError_t e = hipMemcpyAsync(sl.dev, h, used, hipMemcpyHostToDevice, sl.st);
    if (e == hipSuccess)
        e = launch_conv_list((const ConvJob *)sl.dev, (int)pack.size(), pack_blocks, sl.st);
    // the lists run one after another on the slot's stream: the slots already overlap one
    // another's batches, and forking each slot's lists onto side streams (as gfq_batch_launch
    // does) measured slower here (served p99 10.9 -> 13.8 ms)
    for (size_t j = 0; e == hipSuccess && j < groups.size(); j++) {
        BatchList bl;
        bl.prods = (const BatchProd *)(sl.dev + o_prods);
        bl.items = (const BatchItem *)(sl.dev + o_items) + groups[j].item_off;
        bl.prod_done = sl.done;
        bl.prod_time = sl.times + 1;
        e = launch_batched(groups[j].q, groups[j].R, groups[j].twd, bl, (int)groups[j].items.size(), groups[j].lds,
                           sl.st);
    }
    if (e == hipSuccess)
        e = launch_conv_list((const ConvJob *)(sl.dev + o_unpack), (int)unpack.size(), unpack_blocks, sl.st);
    return e;
}

// Serial mode: the single-product calls for the slot's one request.
hipError_t launch_serial(gfq_server *s, Slot &sl) {
    (void)s;
    gfq_set_stream(sl.st);
    const Req &rq = sl.reqs[0].first;
    const gfq_request &r = rq.r;
    char *base = (char *)sl.reqs[0].second;
    const void *A = rq.offA != kNone ? base + rq.offA : r.A;
    const void *B = rq.offB != kNone ? base + rq.offB : r.B;
    void *C = rq.offC != kNone ? base + rq.offC : r.C;
    int st = GFQ_OK;
    if (rq.offA != kNone) st = gfq_pack(r.q, r.m, r.l, (const uint8_t *)r.A, r.lda, (void *)A);
    if (st == GFQ_OK && rq.offB != kNone) st = gfq_pack(r.q, r.l, r.n, (const uint8_t *)r.B, r.ldb, (void *)B);
    if (st == GFQ_OK) st = gfq_matmul(r.q, r.m, r.l, r.n, A, B, C);
    if (st == GFQ_OK && rq.offC != kNone) st = gfq_unpack(r.q, r.m, r.n, C, (uint8_t *)r.C, r.ldc);
    return st == GFQ_OK ? hipSuccess : hipErrorLaunchFailure;
}

// Poll the busy slots; returns true if any finished.
bool reap(gfq_server *s) {
    bool any = false;
    for (Slot &sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t e = hipEventQuery(sl.ev);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) hip_fail(e, "server batch");
        complete(s, sl, e == hipSuccess ? GFQ_OK : GFQ_EHIP);
        any = true;
    }
    return any;
}

// Admit and launch batches while a slot is free; returns true if anything was launched.
bool admit(gfq_server *s) {
    bool any = false;
    int retries = 0;
    for (Slot &sl : s->slots) {
        if (sl.busy) continue;
        while (true) {
            const double t = s->now();
            bool idle = true;
            for (const Slot &x : s->slots) idle = idle && !x.busy;
            sl.reqs.clear();
            const bool ok = admit_batch(s->queue, *s->arena, t, s->o.max_batch, (size_t)s->o.max_items,
                                        [](const Req &r) { return r.items; }, [](const Req &r) { return r.bytes; },
                                        &sl.reqs, idle);
            if (!ok) {
                // nothing in flight and the head request fits no free extent: start the arena
                // afresh once; if even that fails, the device has no memory for it
                if (retries++ == 0) {
                    s->arena->reset();
                    s->a_held = 0;
                    continue;
                }
                Req head = s->queue.front();
                s->queue.pop();
                s->admitted++;
                gfq_completion c{head.r.tag, GFQ_ENOMEM, 0, head.arrival, t, t};
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->completions.push_back(c);
                }
                s->completed++;
                s->cv_done.notify_all();
                retries = 0;
                continue;
            }
            break;
        }
        if (sl.reqs.empty()) break;
        s->admitted += (int64_t)sl.reqs.size();
        s->a_in_use = s->arena->in_use();
        s->a_held = s->arena->held();
        if (s->a_in_use > s->a_peak) s->a_peak = s->a_in_use.load();
        if ((int64_t)sl.reqs.size() > s->max_batch_seen) s->max_batch_seen = (int64_t)sl.reqs.size();
        sl.launch_us = s->now();
        hipError_t e = s->o.mode == GFQ_SERVE_SERIAL ? launch_serial(s, sl) : launch_batch(s, sl);
        if (e == hipSuccess) e = hipEventRecord(sl.ev, sl.st);
        s->batches++;
        sl.busy = true;
        if (e != hipSuccess) {
            hip_fail(e, "server launch");
            (void)hipStreamSynchronize(sl.st);
            complete(s, sl, GFQ_EHIP);
        }
        any = true;
    }
    return any;
}

void worker_main(gfq_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        for (Req &r : s->incoming) s->queue.push(r.arrival, r);
        s->incoming.clear();
        const bool stopping = s->stop;
        lk.unlock();
        bool busy = false;
        reap(s);
        if (!stopping) admit(s);
        for (const Slot &sl : s->slots) busy = busy || sl.busy;
        const double next = s->queue.next_arrival();
        lk.lock();
        if (stopping && !busy) break;
        if (!s->incoming.empty()) continue;
        if (busy) {
            // batches in flight: poll their events closely (completion latency matters)
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else if (!s->queue.empty() && !stopping) {
            const double wait = next - s->now();
            if (wait > 300.0) {
                s->cv_work.wait_for(lk, std::chrono::microseconds((int64_t)(wait - 150.0)));
            } else if (wait > 0) {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        } else if (!stopping) {
            s->cv_work.wait(lk, [s] { return s->stop || !s->incoming.empty(); });
        }
    }
}

void server_free(gfq_server *s) {
    if (!s) return;
    delete s->arena;
    for (Slot &sl : s->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    delete s;
}

}  // namespace

extern "C" {

int gfq_server_create(const gfq_server_opts *opts, gfq_server **out) {
    if (!out) return GFQ_ENULL;
    *out = nullptr;
    gfq_server_opts o{};
    if (opts) o = *opts;
    if (o.mode != GFQ_SERVE_BATCHED && o.mode != GFQ_SERVE_SERIAL) return GFQ_EINVAL;
    if (o.budget_bytes == 0) o.budget_bytes = (size_t)1 << 30;
    if (o.slots == 0) o.slots = 3;
    if (o.max_batch == 0) o.max_batch = 256;
    if (o.max_items == 0) o.max_items = 65536;
    if (o.slots < 1 || o.slots > 8 || o.max_batch < 1 || o.max_batch > 4096 || o.max_items < 32768 ||
        o.max_items > (1 << 20))
        return GFQ_EINVAL;
    if (o.mode == GFQ_SERVE_SERIAL) {
        o.slots = 1;
        o.max_batch = 1;
    }
    gfq_server *s = new gfq_server();
    s->o = o;
    s->t0 = Clock::now();
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = set_batched_lds_limits();
    if (e != hipSuccess) { server_free(s); return hip_fail(e, "server setup"); }
    const size_t mb = (size_t)o.max_batch;
    s->staged_cap = rup(sizeof(ConvJob) * 2 * mb) + rup(sizeof(ConvJob) * mb) + rup(sizeof(BatchProd) * mb) +
                    rup(sizeof(BatchItem) * (size_t)o.max_items);
    s->off_done = s->staged_cap;
    s->off_times = s->off_done + rup(sizeof(u32) * mb);
    s->slot_bytes = s->off_times + rup(sizeof(unsigned long long) * (mb + 1));
    s->slots.resize(o.slots);
    for (Slot &sl : s->slots) {
        e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.dev, s->slot_bytes);
        if (e == hipSuccess) e = hipHostMalloc(&sl.host, s->staged_cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMemset(sl.dev, 0, s->slot_bytes);
        if (e != hipSuccess) { server_free(s); return hip_fail(e, "server slots"); }
        sl.done = (u32 *)(sl.dev + s->off_done);
        sl.times = (unsigned long long *)(sl.dev + s->off_times);
    }
    const int dev = s->device;
    s->arena = new Arena(
        o.budget_bytes, std::min(o.budget_bytes, (size_t)1 << 30),
        [dev](size_t bytes, uintptr_t *p) {
            void *v = nullptr;
            (void)hipSetDevice(dev);
            if (hipMalloc(&v, bytes) != hipSuccess) { (void)hipGetLastError(); return false; }
            *p = (uintptr_t)v;
            return true;
        },
        [](uintptr_t p) { (void)hipFree((void *)p); });
    s->worker = std::thread(worker_main, s);
    *out = s;
    return GFQ_OK;
}

int gfq_server_submit(gfq_server *s, const gfq_request *reqs, int count) {
    if (!s) return GFQ_ENULL;
    if (count < 0) return GFQ_EINVAL;
    if (count == 0) return GFQ_OK;
    if (!reqs) return GFQ_ENULL;
    std::vector<Req> v(count);
    const double t = s->now();
    for (int i = 0; i < count; i++) {
        const gfq_request &r = reqs[i];
        if (!valid_field(r.q)) return GFQ_EFIELD;
        if (r.m < 0 || r.l < 0 || r.n < 0 || r.m > kMaxSide || r.l > kMaxSide || r.n > kMaxSide) return GFQ_EDIM;
        if (r.flags & ~(GFQ_REQ_A_PACKED | GFQ_REQ_B_PACKED | GFQ_REQ_C_PACKED)) return GFQ_EINVAL;
        const bool pa = r.flags & GFQ_REQ_A_PACKED, pb = r.flags & GFQ_REQ_B_PACKED, pc = r.flags & GFQ_REQ_C_PACKED;
        const bool work = r.m > 0 && r.n > 0, inner = work && r.l > 0;
        if (work && !r.C) return GFQ_ENULL;
        if (inner && (!r.A || !r.B)) return GFQ_ENULL;
        if (inner && ((!pa && r.lda < r.l) || (!pb && r.ldb < r.n))) return GFQ_EDIM;
        if (work && !pc && r.ldc < r.n) return GFQ_EDIM;
        if ((inner && pa && ((uintptr_t)r.A & 15)) || (inner && pb && ((uintptr_t)r.B & 15)) ||
            (work && pc && ((uintptr_t)r.C & 15)))
            return GFQ_EALIGN;
        const size_t sc = work ? span(r.q, r.m, r.n, r.ldc, pc) : 0;
        if (inner && (overlaps((uintptr_t)r.C, sc, (uintptr_t)r.A, span(r.q, r.m, r.l, r.lda, pa)) ||
                      overlaps((uintptr_t)r.C, sc, (uintptr_t)r.B, span(r.q, r.l, r.n, r.ldb, pb))))
            return GFQ_EALIAS;
        Req &q = v[i];
        q.r = r;
        q.arrival = std::max(t, r.not_before_us);
        size_t off = 0;
        if (inner && !pa) { q.offA = off; off += rup(gfq_packed_bytes(r.q, r.m, r.l)); }
        if (inner && !pb) { q.offB = off; off += rup(gfq_packed_bytes(r.q, r.l, r.n)); }
        if (work && !pc) { q.offC = off; off += rup(gfq_packed_bytes(r.q, r.m, r.n)); }
        q.bytes = off;
        q.items = batch_tiles_bound(r.m, r.n);
        if (Arena::round(q.bytes) > s->o.budget_bytes) return GFQ_EBUDGET;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->failed) return GFQ_EHIP;
        for (Req &r : v) s->incoming.push_back(r);
    }
    s->submitted += count;
    s->cv_work.notify_one();
    return GFQ_OK;
}

int gfq_server_poll(gfq_server *s, gfq_completion *out, int max, int *got, double timeout_us) {
    if (!s || !got || (max > 0 && !out)) return GFQ_ENULL;
    *got = 0;
    if (max < 0) return GFQ_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completions.empty() && timeout_us != 0) {
        auto ready = [s] { return !s->completions.empty(); };
        if (timeout_us < 0) s->cv_done.wait(lk, ready);
        else s->cv_done.wait_for(lk, std::chrono::microseconds((int64_t)timeout_us), ready);
    }
    int n = 0;
    while (n < max && !s->completions.empty()) {
        out[n++] = s->completions.front();
        s->completions.pop_front();
    }
    *got = n;
    return GFQ_OK;
}

double gfq_server_now_us(const gfq_server *s) { return s ? s->now() : 0.0; }

int gfq_server_stats_read(const gfq_server *s, gfq_server_stats *out) {
    if (!s || !out) return GFQ_ENULL;
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->batches = s->batches;
    out->queued = s->submitted - s->admitted;
    out->max_batch_seen = s->max_batch_seen;
    out->arena_in_use = s->a_in_use;
    out->arena_held = s->a_held;
    out->arena_peak_in_use = s->a_peak;
    return GFQ_OK;
}

int gfq_server_destroy(gfq_server *s) {
    if (!s) return GFQ_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    hipError_t e = hipSetDevice(s->device);
    for (Slot &sl : s->slots)
        if (e == hipSuccess && sl.st) e = hipStreamSynchronize(sl.st);
    server_free(s);
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "server destroy");
}

}  // extern "C"
