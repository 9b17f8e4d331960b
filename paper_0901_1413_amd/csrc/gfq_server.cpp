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
#include "gfq_serve_core.h"

using namespace gfq;

namespace {

constexpr int64_t kMaxSide = 65535;   // keeps every tile index of a request in 16 bits
constexpr size_t kNone = ~(size_t)0;

size_t rup(size_t x) { return (x + 255) & ~(size_t)255; }

struct Req {
    gfq_request r;
    double arrival = 0;
    size_t bytes = 0;                  // arena bytes (packed forms the server makes)
    size_t items = 0;                  // tile bound
    uint64_t tag = 0;
    size_t offA = kNone, offB = kNone, offC = kNone;   // within the arena range
};

bool overlaps(uintptr_t a, size_t na, uintptr_t b, size_t nb) { return na && nb && a < b + nb && b < a + na; }

// Bytes spanned by an operand: packed size, or rows x ld uint8 (last row cols long).
size_t span(int q, int64_t rows, int64_t cols, int64_t ld, bool packed) {
    if (rows <= 0 || cols <= 0) return 0;
    return packed ? gfq_packed_bytes(q, rows, cols) : (size_t)((rows - 1) * ld + cols);
}

// The device side of the server: one stream, completion event and descriptor buffer (with
// its pinned staging mirror) per slot.
struct HipExec {
    typedef std::vector<std::pair<Req, uintptr_t>> Batch;
    struct Slot {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        char *dev = nullptr;               // descriptors (staged part, then counts and times)
        char *host = nullptr;              // pinned staging mirror of the staged part
        u32 *done = nullptr;               // per-product tile counts (zero between launches)
        unsigned long long *times = nullptr;
        bool retired = false;              // given up by the watchdog: never waited for or freed
    };
    int mode = GFQ_SERVE_BATCHED;
    size_t staged_cap = 0;
    std::vector<Slot> sl;

    int slots() const { return (int)sl.size(); }
    int launch(int i, const Batch &b);
    int poll(int i) {
        const hipError_t e = hipEventQuery(sl[i].ev);
        if (e == hipErrorNotReady) return 1;
        return e == hipSuccess ? 0 : hip_fail(e, "server batch");
    }
    void drain(int i) { (void)hipStreamSynchronize(sl[i].st); }
    void retire(int i) { sl[i].retired = true; }
    hipError_t copy_to_host(const Req &rq, const void *C, hipStream_t st) const;
    hipError_t launch_batch(Slot &s, const Batch &b);
    hipError_t launch_serial(Slot &s, const Batch &b);
};

// The request's product to its host destination, if it has one: the span of C (uint8 with
// leading dimension ldc, or packed), after the product is complete on the stream.
hipError_t HipExec::copy_to_host(const Req &rq, const void *C, hipStream_t st) const {
    const gfq_request &r = rq.r;
    if (!r.C_host || r.m <= 0 || r.n <= 0) return hipSuccess;
    const bool pc = r.flags & GFQ_REQ_C_PACKED;
    return hipMemcpyAsync(r.C_host, C, span(r.q, r.m, r.n, r.ldc, pc), hipMemcpyDeviceToHost, st);
}

// Batched mode: stage descriptors and enqueue the launches of one batch on slot s.
hipError_t HipExec::launch_batch(Slot &s, const Batch &b) {
    const int nreq = (int)b.size();
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
        const Req &rq = b[i].first;
        const gfq_request &r = rq.r;
        char *base = (char *)b[i].second;
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
    if (used > staged_cap) return hipErrorInvalidValue;   // bounded by the batch limits
    char *h = s.host;
    std::memcpy(h, pack.data(), sizeof(ConvJob) * pack.size());
    std::memcpy(h + o_unpack, unpack.data(), sizeof(ConvJob) * unpack.size());
    std::memcpy(h + o_prods, prods.data(), sizeof(BatchProd) * nreq);
    for (const BatchGroup &g : groups)
        std::memcpy(h + o_items + sizeof(BatchItem) * g.item_off, g.items.data(), sizeof(BatchItem) * g.items.size());
    hipError_t e = hipMemcpyAsync(s.dev, h, used, hipMemcpyHostToDevice, s.st);
    if (e == hipSuccess)
        e = launch_conv_list((const ConvJob *)s.dev, (int)pack.size(), pack_blocks, s.st);
    // the lists run one after another on the slot's stream: the slots already overlap one
    // another's batches, and forking each slot's lists onto side streams (as gfq_batch_launch
    // does) measured slower here (served p99 10.9 -> 13.8 ms)
    for (size_t j = 0; e == hipSuccess && j < groups.size(); j++) {
        BatchList bl;
        bl.prods = (const BatchProd *)(s.dev + o_prods);
        bl.items = (const BatchItem *)(s.dev + o_items) + groups[j].item_off;
        bl.prod_done = s.done;
        bl.prod_time = s.times + 1;
        e = launch_batched(groups[j].q, groups[j].R, groups[j].twd, bl, (int)groups[j].items.size(), groups[j].lds,
                           s.st);
    }
    if (e == hipSuccess)
        e = launch_conv_list((const ConvJob *)(s.dev + o_unpack), (int)unpack.size(), unpack_blocks, s.st);
    for (int i = 0; e == hipSuccess && i < nreq; i++) {
        const Req &rq = b[i].first;
        e = copy_to_host(rq, rq.offC != kNone ? rq.r.C : probs[i].C, s.st);
    }
    return e;
}

// Serial mode: the single-product calls for the slot's one request.
hipError_t HipExec::launch_serial(Slot &s, const Batch &b) {
    gfq_set_stream(s.st);
    const Req &rq = b[0].first;
    const gfq_request &r = rq.r;
    char *base = (char *)b[0].second;
    const void *A = rq.offA != kNone ? base + rq.offA : r.A;
    const void *B = rq.offB != kNone ? base + rq.offB : r.B;
    void *C = rq.offC != kNone ? base + rq.offC : r.C;
    int st = GFQ_OK;
    if (rq.offA != kNone) st = gfq_pack(r.q, r.m, r.l, (const uint8_t *)r.A, r.lda, (void *)A);
    if (st == GFQ_OK && rq.offB != kNone) st = gfq_pack(r.q, r.l, r.n, (const uint8_t *)r.B, r.ldb, (void *)B);
    if (st == GFQ_OK) st = gfq_matmul(r.q, r.m, r.l, r.n, A, B, C);
    if (st == GFQ_OK && rq.offC != kNone) st = gfq_unpack(r.q, r.m, r.n, C, (uint8_t *)r.C, r.ldc);
    if (st != GFQ_OK) return hipErrorLaunchFailure;
    return copy_to_host(rq, r.C, s.st);
}

int HipExec::launch(int i, const Batch &b) {
    Slot &s = sl[i];
    hipError_t e = mode == GFQ_SERVE_SERIAL ? launch_serial(s, b) : launch_batch(s, b);
    if (e == hipSuccess) e = hipEventRecord(s.ev, s.st);
    return e == hipSuccess ? 0 : hip_fail(e, "server launch");
}

}  // namespace

struct gfq_server {
    gfq_server_opts o{};
    int device = 0;
    HipExec exec;
    Arena *arena = nullptr;
    ServeCore<Req, HipExec> *core = nullptr;
};

namespace {

void server_free(gfq_server *s) {
    if (!s) return;
    delete s->core;                    // stops the worker
    // ranges handed out to a retired slot may still be written by the device: the arena's
    // memory is kept then
    bool retired = false;
    for (const HipExec::Slot &x : s->exec.sl) retired = retired || x.retired;
    if (retired) s->arena = nullptr;
    delete s->arena;
    for (HipExec::Slot &sl : s->exec.sl) {
        if (sl.retired) continue;
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
        o.max_items > (1 << 20) || !(o.watchdog_s >= 0.0))
        return GFQ_EINVAL;
    if (o.mode == GFQ_SERVE_SERIAL) {
        o.slots = 1;
        o.max_batch = 1;
    }
    gfq_server *s = new gfq_server();
    s->o = o;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = set_batched_lds_limits();
    if (e != hipSuccess) { server_free(s); return hip_fail(e, "server setup"); }
    const size_t mb = (size_t)o.max_batch;
    HipExec &x = s->exec;
    x.mode = o.mode;
    x.staged_cap = rup(sizeof(ConvJob) * 2 * mb) + rup(sizeof(ConvJob) * mb) + rup(sizeof(BatchProd) * mb) +
                   rup(sizeof(BatchItem) * (size_t)o.max_items);
    const size_t off_done = x.staged_cap;
    const size_t off_times = off_done + rup(sizeof(u32) * mb);
    const size_t slot_bytes = off_times + rup(sizeof(unsigned long long) * (mb + 1));
    x.sl.resize(o.slots);
    for (HipExec::Slot &sl : x.sl) {
        e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.dev, slot_bytes);
        if (e == hipSuccess) e = hipHostMalloc(&sl.host, x.staged_cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMemset(sl.dev, 0, slot_bytes);
        if (e != hipSuccess) { server_free(s); return hip_fail(e, "server slots"); }
        sl.done = (u32 *)(sl.dev + off_done);
        sl.times = (unsigned long long *)(sl.dev + off_times);
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
    ServeLimits lim;
    lim.max_batch = o.max_batch;
    lim.max_items = (size_t)o.max_items;
    lim.watchdog_us = o.watchdog_s * 1e6;
    s->core = new ServeCore<Req, HipExec>(s->exec, *s->arena, lim);
    s->core->start_on([dev] { (void)hipSetDevice(dev); });
    *out = s;
    return GFQ_OK;
}

int gfq_server_submit(gfq_server *s, const gfq_request *reqs, int count) {
    if (!s) return GFQ_ENULL;
    if (count < 0) return GFQ_EINVAL;
    if (count == 0) return GFQ_OK;
    if (!reqs) return GFQ_ENULL;
    std::vector<Req> v(count);
    const double t = s->core->now();
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
        q.tag = r.tag;
        q.arrival = std::max(t, r.not_before_us);
        size_t off = 0;
        if (inner && !pa) { q.offA = off; off += rup(gfq_packed_bytes(r.q, r.m, r.l)); }
        if (inner && !pb) { q.offB = off; off += rup(gfq_packed_bytes(r.q, r.l, r.n)); }
        if (work && !pc) { q.offC = off; off += rup(gfq_packed_bytes(r.q, r.m, r.n)); }
        q.bytes = off;
        q.items = batch_tiles_bound(r.m, r.n);
        if (Arena::round(q.bytes) > s->o.budget_bytes) return GFQ_EBUDGET;
    }
    return s->core->submit(v) ? GFQ_OK : GFQ_EHIP;
}

int gfq_server_poll(gfq_server *s, gfq_completion *out, int max, int *got, double timeout_us) {
    if (!s || !got || (max > 0 && !out)) return GFQ_ENULL;
    *got = 0;
    if (max < 0) return GFQ_EINVAL;
    std::vector<ServeCompletion> c(std::max(max, 1));
    const int n = s->core->poll(c.data(), max, timeout_us);
    for (int i = 0; i < n; i++)
        out[i] = gfq_completion{c[i].tag, c[i].status, c[i].batch_size, c[i].arrival_us, c[i].launch_us, c[i].done_us};
    *got = n;
    return GFQ_OK;
}

double gfq_server_now_us(const gfq_server *s) { return s ? s->core->now() : 0.0; }

int gfq_server_stats_read(const gfq_server *s, gfq_server_stats *out) {
    if (!s || !out) return GFQ_ENULL;
    const ServeCore<Req, HipExec> &c = *s->core;
    out->submitted = c.submitted;
    out->completed = c.completed;
    out->batches = c.batches;
    out->queued = c.submitted - c.admitted;
    out->max_batch_seen = c.max_batch_seen;
    out->arena_in_use = c.a_in_use;
    out->arena_held = c.a_held;
    out->arena_peak_in_use = c.a_peak;
    return GFQ_OK;
}

int gfq_server_destroy(gfq_server *s) {
    if (!s) return GFQ_OK;
    s->core->stop();
    hipError_t e = hipSetDevice(s->device);
    for (HipExec::Slot &sl : s->exec.sl)
        if (e == hipSuccess && sl.st && !sl.retired) e = hipStreamSynchronize(sl.st);
    server_free(s);
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "server destroy");
}

}  // extern "C"
