// gfq_batch_host.cpp -- building, launching and timing batches of products (the host side
// of gfq_batch.hip): per-product launch parameters, work lists ordered longest first, slab
// slices for products whose tiles are too long for the batch, and one device allocation for
// all descriptors and partial products.  A launch is a start stamp, one work-list kernel per
// (field, tile height) -- the first on the caller's stream, the others forked onto side
// streams and joined back, so that one group's last workgroups overlap the others' -- and,
// when products are sliced, one partial-sum launch; it allocates nothing, so a caller may
// capture it into a graph (the fork becomes parallel branches of the graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "gfq.h"
#include "gfq_batch.h"
#include "gfq_host.h"

using namespace gfq;

namespace {

// Side streams (default priority) and their events for the batch launches made on one
// caller stream, created on first need and kept until the process ends.  They are never
// created while the caller's stream is being captured: a capture without them launches the
// groups one after another on the caller's stream.
struct SidePool {
    hipEvent_t fork = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
};
std::mutex g_side_mu;
std::map<std::pair<int, hipStream_t>, SidePool> g_side;

SidePool *side_pool(hipStream_t st, size_t n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_side_mu);
    SidePool &p = g_side[std::make_pair(dev, st)];
    if (p.fork && p.streams.size() >= n) return &p;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    if (!p.fork && hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) != hipSuccess) {
        p.fork = nullptr;
        return nullptr;
    }
    while (p.streams.size() < n) {
        hipStream_t s = nullptr;
        hipEvent_t d = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&d, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(s);
            return nullptr;
        }
        p.streams.push_back(s);
        p.done.push_back(d);
    }
    return &p;
}

int group_index(int q, int R, int twd) {
    const int qi = q == 3 ? 0 : (q == 4 ? 1 : (q == 5 ? 2 : (q == 7 ? 3 : (q == 8 ? 4 : 5))));
    return qi * 4 + (twd == 8 ? 2 : (twd == 4 ? 3 : (R == 2 ? 0 : 1)));
}

}  // namespace

// Launch parameters of every product and its tiles, grouped by (field, rows per lane) and
// ordered longest first within a group.
void gfq::plan_batch(int count, const gfq_problem *problems, const gfq_config *cfgs, BatchProd *prods,
                     std::vector<BatchGroup> *groups, size_t *nitems, BatchSlicing *slicing) {
    std::vector<BatchGroup> g(24);
    struct Shape { int gi = -1, tx = 0, ty = 0, TM = 0, twd = 16; double tile_cost = 0; };
    std::vector<Shape> sh(count);
    double total = 0;
    for (int i = 0; i < count; i++) {
        const gfq_problem &p = problems[i];
        BatchProd &bp = prods[i];
        std::memset(&bp, 0, sizeof bp);
        gfq_config c;
        if (cfgs) c = cfgs[i];
        else if (gfq_tune_lookup(p.q, p.m, p.l, p.n, GFQ_TUNE_BATCH, &c) != GFQ_OK)
            gfq_choose_config(p.q, p.m, p.l, p.n, &c);
        const int P = planes_of(p.q);
        // Tile shape: 16-word tiles with the configured rows per lane; a product taller than
        // 256 rows and at most 256 (128) columns wide is one narrow tile column of 8 (4) words
        // and 512 (1024) rows per tile instead, which pads it less.  The super-rows of the
        // kernel bound the slab width.
        int R = c.rows <= 256 ? 2 : max_rows_per_lane_batch(p.q);
        int twd = 16;
        if (p.m > 256 && p.n <= 128) twd = 4, R = 2;
        else if (p.m > 256 && p.n <= 256) twd = 8, R = 2;
        const int srb = twd == 16 ? batch_srb(p.q, R) : 256;
        int k = std::min(c.k, batch_kmax(p.q, twd == 16 ? R : 2));
        if (p.l > 0 && p.l < k) k = (int)p.l;
        if (k < 1) k = 1;
        const int TM = NT_MM / (twd / 4) * R;
        MMArgs &a = bp.a;
        a.A = (const u32 *)p.A;
        a.B = (const u32 *)p.B;
        a.out = (u32 *)p.C;
        a.m = (int)p.m;
        a.l = (int)p.l;
        a.n = (int)p.n;
        a.Wl = words_of(p.l);
        a.Wn = words_of(p.n);
        a.k = k;
        a.S = p.l > 0 ? (int)((p.l + k - 1) / k) : 0;
        a.slabs_per_split = std::max(a.S, 1);
        a.split_stride = (size_t)p.m * P * a.Wn;
        mm_lds_bytes(p.q, k, srb, TM, &a.tb1);
        bp.slices = 1;
        bp.C = (u32 *)p.C;
        bp.q = p.q;
        if (p.m == 0 || p.n == 0) continue;
        Shape &s = sh[i];
        s.tx = (a.Wn + twd - 1) / twd;
        s.ty = (a.m + TM - 1) / TM;
        s.TM = TM;
        s.twd = twd;
        s.gi = group_index(p.q, R, twd);
        // relative tile cost: rows x words x slabs (plus the tables it builds); the first tile
        // is a whole one, the costliest
        const double rows = std::min<int64_t>(TM, p.m), words = std::min(twd, a.Wn);
        s.tile_cost = (rows + (double)(1 << k)) * words * std::max(a.S, 1) * (P == 2 ? 1.0 : 3.0);
        for (int y = 0; y < s.ty; y++)
            for (int x = 0; x < s.tx; x++)
                total += (std::min<int64_t>(TM, p.m - (int64_t)y * TM) + (double)(1 << k)) *
                         std::min(twd, a.Wn - x * twd) * std::max(a.S, 1) * (P == 2 ? 1.0 : 3.0);
        BatchGroup &gr = g[s.gi];
        gr.q = p.q;
        gr.R = R;
        gr.twd = twd;
        gr.kmax = std::max(gr.kmax, k);
    }
    if (slicing) {
        slicing->partial_words = 0;
        slicing->part_off.assign(count, 0);
        slicing->reduce.clear();
    }
    const double share = total / std::max(1, slicing ? slicing->cus : 1);
    for (int i = 0; i < count; i++) {
        const Shape &s = sh[i];
        if (s.gi < 0) continue;
        BatchProd &bp = prods[i];
        MMArgs &a = bp.a;
        int slices = 1;
        if (slicing && a.S >= 16 && s.tile_cost > 0.5 * share) {
            // slices of at least 8 slabs, at most 64, and at most 256 MiB of partial products
            const size_t part_bytes = a.split_stride * 4;
            int64_t want = (int64_t)std::ceil(2.0 * s.tile_cost / share);
            want = std::min<int64_t>(want, std::min<int64_t>(a.S / 8, 64));
            want = std::min<int64_t>(want, (int64_t)(((size_t)256 << 20) / std::max<size_t>(part_bytes, 1)));
            if (want >= 2) {
                a.slabs_per_split = (a.S + (int)want - 1) / (int)want;
                slices = (a.S + a.slabs_per_split - 1) / a.slabs_per_split;
            }
        }
        bp.slices = (u32)slices;
        bp.units = (u32)(s.tx * s.ty * slices);
        if (slices > 1) {
            slicing->part_off[i] = slicing->partial_words;
            slicing->partial_words += (size_t)slices * a.split_stride;
            const u32 ngroups = (u32)a.m * (u32)(a.Wn / 4), chunk = 1024;
            for (u32 f = 0; f < ngroups; f += chunk) {
                slicing->reduce.push_back(ReduceItem{(u32)i, f, std::min(chunk, ngroups - f)});
                bp.units++;
            }
        }
        BatchGroup &gr = g[s.gi];
        const int P = planes_of(problems[i].q);
        for (int y = 0; y < s.ty; y++)
            for (int x = 0; x < s.tx; x++)
                for (int z = 0; z < slices; z++) {
                    const double rows = std::min<int64_t>(s.TM, a.m - (int64_t)y * s.TM);
                    const double words = std::min(s.twd, a.Wn - x * s.twd);
                    const int slabs = std::max(1, std::min(a.slabs_per_split, a.S - z * a.slabs_per_split));
                    gr.items.push_back(BatchItem{(u32)i, (uint16_t)x, (uint16_t)y, (u32)z});
                    // relative item cost: rows x words x slabs (plus the tables it builds)
                    gr.cost.push_back((rows + (double)(1 << a.k)) * words * slabs * (P == 2 ? 1.0 : 3.0));
                }
    }
    groups->clear();
    size_t n = 0;
    for (BatchGroup &gr : g) {
        if (gr.items.empty()) continue;
        std::vector<size_t> idx(gr.items.size());
        for (size_t j = 0; j < idx.size(); j++) idx[j] = j;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return gr.cost[x] > gr.cost[y]; });
        std::vector<BatchItem> sorted(idx.size());
        for (size_t j = 0; j < idx.size(); j++) sorted[j] = gr.items[idx[j]];
        gr.items.swap(sorted);
        gr.cost.clear();
        gr.item_off = n;
        n += gr.items.size();
        gr.lds = mm_lds_bytes(gr.q, gr.kmax, gr.twd == 16 ? batch_srb(gr.q, gr.R) : 256,
                              NT_MM / (gr.twd / 4) * gr.R, nullptr);
        groups->push_back(std::move(gr));
    }
    *nitems = n;
}

hipError_t gfq::launch_group_lists(const std::vector<BatchGroup> &groups, const BatchList &base, hipStream_t st,
                                   u32 *queue_heads) {
    const size_t ng = groups.size();
    SidePool *sp = ng > 1 ? side_pool(st, ng - 1) : nullptr;
    hipError_t e = sp ? hipEventRecord(sp->fork, st) : hipSuccess;
    for (size_t j = 0; e == hipSuccess && j < ng; j++) {
        const BatchGroup &gr = groups[j];
        const bool side = sp && j > 0;
        hipStream_t s = side ? sp->streams[j - 1] : st;
        if (side) e = hipStreamWaitEvent(s, sp->fork, 0);
        BatchList l = base;
        l.items = base.items + gr.item_off;
        if (e == hipSuccess)
            e = queue_heads ? launch_queue(gr.q, gr.R, gr.twd, l, (int)gr.items.size(), gr.lds, queue_heads + j,
                                           gr.queue_wgs, s)
                            : launch_batched(gr.q, gr.R, gr.twd, l, (int)gr.items.size(), gr.lds, s);
        if (e == hipSuccess && side) e = hipEventRecord(sp->done[j - 1], s);
    }
    for (size_t j = 1; e == hipSuccess && sp && j < ng; j++) e = hipStreamWaitEvent(st, sp->done[j - 1], 0);
    return e;
}

size_t gfq::batch_tiles_bound(int64_t m, int64_t n) {
    if (m <= 0 || n <= 0) return 0;
    return (size_t)((m + 255) / 256) * (size_t)((words_of(n) + 15) / 16);
}

hipError_t gfq::set_batched_lds_limits() {
    for (int q : {3, 4, 5, 7, 8, 9}) {
        for (int R : {2, max_rows_per_lane_batch(q)}) {
            const size_t lds = mm_lds_bytes(q, batch_kmax(q, R), batch_srb(q, R), NT_MM / 4 * R, nullptr);
            hipError_t e = hipFuncSetAttribute(batched_kernel(q, R, 16), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(queue_kernel(q, R, 16), hipFuncAttributeMaxDynamicSharedMemorySize, (int)queue_lds(lds));
            if (e != hipSuccess) return e;
        }
        for (int twd : {8, 4}) {
            const void *k = batched_kernel(q, 2, twd);
            if (!k) continue;
            const size_t lds = mm_lds_bytes(q, batch_kmax(q, 2), 256, NT_MM / (twd / 4) * 2, nullptr);
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(queue_kernel(q, 2, twd), hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)queue_lds(lds));
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

struct gfq_batch {
    int count = 0;
    int device = 0;
    std::vector<BatchGroup> groups;
    void *mem = nullptr;
    BatchProd *prods = nullptr;
    BatchItem *items = nullptr;
    u32 *prod_done = nullptr;
    unsigned long long *times = nullptr;   // [0] start, [1 + p] completion of product p
    ReduceItem *ritems = nullptr;          // partial-sum items of the sliced products
    int nritems = 0;
    u32 *heads = nullptr;                  // queue head of each list (persistent launches)
    std::vector<int> k;                    // slab width of each product
    std::vector<int> slices;               // slab slices of each product
};

static void batch_release(gfq_batch *b) {
    if (!b) return;
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

// Build a batch; cfgs (optional, one per product) overrides the per-product choice of slab
// width and tile height (the tuner uses it to time candidates).
int gfq::batch_create_with(int count, const gfq_problem *problems, const gfq_config *cfgs, gfq_batch **out) {
    if (!out) return GFQ_ENULL;
    *out = nullptr;
    if (count < 0) return GFQ_EINVAL;
    if (count > 0 && !problems) return GFQ_ENULL;
    for (int i = 0; i < count; i++) {
        const gfq_problem &p = problems[i];
        int st = validate_mm(p.q, p.m, p.l, p.n, p.A, p.B, p.C);
        if (st != GFQ_OK) return st;
        if (p.m >= (1 << 16) * 256 || p.n >= (int64_t)(1 << 16) * 512) return GFQ_EDIM;   // tile index fits 16 bits
    }
    gfq_batch *b = new gfq_batch();
    b->count = count;
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) { batch_release(b); return hip_fail(e, "hipGetDevice"); }

    std::vector<BatchProd> prods(std::max(count, 1));
    size_t nitems = 0;
    BatchSlicing sl;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
        sl.cus = cus;
    plan_batch(count, problems, cfgs, prods.data(), &b->groups, &nitems, &sl);
    b->k.resize(count);
    b->slices.resize(count);
    for (int i = 0; i < count; i++) {
        b->k[i] = prods[i].a.k;
        b->slices[i] = (int)prods[i].slices;
    }

    // one allocation: products | items | partial-sum items | unit counts | times | partials
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t nr = sl.reduce.size();
    const size_t off_items = align(sizeof(BatchProd) * std::max(count, 1));
    const size_t off_ritems = off_items + align(sizeof(BatchItem) * std::max<size_t>(nitems, 1));
    const size_t off_heads = off_ritems + align(sizeof(ReduceItem) * std::max<size_t>(nr, 1));
    const size_t off_done = off_heads + align(sizeof(u32) * 64);
    const size_t off_time = off_done + align(sizeof(u32) * std::max(count, 1));
    const size_t off_part = off_time + align(sizeof(unsigned long long) * (count + 1));
    const size_t total = off_part + align(sl.partial_words * sizeof(u32));
    e = hipMalloc(&b->mem, total);
    if (e != hipSuccess) { batch_release(b); hip_fail(e, "hipMalloc(batch)"); return GFQ_ENOMEM; }
    char *base = (char *)b->mem;
    for (int i = 0; i < count; i++)
        if (prods[i].slices > 1) prods[i].a.out = (u32 *)(base + off_part) + sl.part_off[i];
    std::vector<BatchItem> all(std::max<size_t>(nitems, 1));
    for (const BatchGroup &gr : b->groups) std::copy(gr.items.begin(), gr.items.end(), all.begin() + gr.item_off);
    e = hipMemset(b->mem, 0, off_part);
    if (e == hipSuccess && count > 0) e = hipMemcpy(base, prods.data(), sizeof(BatchProd) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess && nitems > 0) e = hipMemcpy(base + off_items, all.data(), sizeof(BatchItem) * nitems, hipMemcpyHostToDevice);
    if (e == hipSuccess && nr > 0)
        e = hipMemcpy(base + off_ritems, sl.reduce.data(), sizeof(ReduceItem) * nr, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = set_batched_lds_limits();
    // persistent workgroups per list: as many as the device holds at once, at most one per item
    for (BatchGroup &gr : b->groups) {
        if (e != hipSuccess) break;
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, queue_kernel(gr.q, gr.R, gr.twd), NT_MM,
                                                         queue_lds(gr.lds));
        gr.queue_wgs = (int)std::min<size_t>((size_t)std::max(per_cu, 1) * sl.cus, gr.items.size());
    }
    if (e != hipSuccess) { batch_release(b); return hip_fail(e, "batch upload"); }
    b->prods = (BatchProd *)base;
    b->items = (BatchItem *)(base + off_items);
    b->ritems = (ReduceItem *)(base + off_ritems);
    b->heads = (u32 *)(base + off_heads);
    b->nritems = (int)nr;
    b->prod_done = (u32 *)(base + off_done);
    b->times = (unsigned long long *)(base + off_time);
    *out = b;
    return GFQ_OK;
}

extern "C" {

int gfq_batch_create(int count, const gfq_problem *problems, gfq_batch **out) {
    return batch_create_with(count, problems, nullptr, out);
}

int gfq_batch_launch(gfq_batch *b) {
    if (!b) return GFQ_ENULL;
    hipStream_t st = current_stream();
    hipError_t e = launch_batch_stamp(b->times, st);
    BatchList base;
    base.prods = b->prods;
    base.items = b->items;
    base.prod_done = b->prod_done;
    base.prod_time = b->times + 1;
    if (e == hipSuccess) e = launch_group_lists(b->groups, base, st);
    if (e == hipSuccess && b->nritems > 0) {
        ReduceList rl;
        rl.prods = b->prods;
        rl.items = b->ritems;
        rl.prod_done = b->prod_done;
        rl.prod_time = b->times + 1;
        e = launch_reduce_list(rl, b->nritems, st);
    }
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "batch launch");
}

int gfq_batch_launch_persistent(gfq_batch *b) {
    if (!b) return GFQ_ENULL;
    if (b->groups.size() > 64) return GFQ_EINVAL;
    hipStream_t st = current_stream();
    hipError_t e = launch_batch_stamp(b->times, st);
    if (e == hipSuccess) e = launch_queue_reset(b->heads, (int)b->groups.size(), st);
    BatchList base;
    base.prods = b->prods;
    base.items = b->items;
    base.prod_done = b->prod_done;
    base.prod_time = b->times + 1;
    if (e == hipSuccess) e = launch_group_lists(b->groups, base, st, b->heads);
    if (e == hipSuccess && b->nritems > 0) {
        ReduceList rl;
        rl.prods = b->prods;
        rl.items = b->ritems;
        rl.prod_done = b->prod_done;
        rl.prod_time = b->times + 1;
        e = launch_reduce_list(rl, b->nritems, st);
    }
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "persistent batch launch");
}

int gfq_batch_times(gfq_batch *b, double *completion_us) {
    if (!b || !completion_us) return GFQ_ENULL;
    std::vector<unsigned long long> t(b->count + 1);
    hipError_t e = hipStreamSynchronize(current_stream());
    if (e == hipSuccess) e = hipMemcpy(t.data(), b->times, sizeof(unsigned long long) * t.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "batch times");
    for (int p = 0; p < b->count; p++)
        completion_us[p] = t[1 + p] >= t[0] ? (double)(t[1 + p] - t[0]) * 0.01 : 0.0;   // 100 MHz ticks
    return GFQ_OK;
}

int gfq_batch_slab_widths(const gfq_batch *b, int *k) {
    if (!b || !k) return GFQ_ENULL;
    std::copy(b->k.begin(), b->k.end(), k);
    return GFQ_OK;
}

int gfq_batch_slices(const gfq_batch *b, int *slices) {
    if (!b || !slices) return GFQ_ENULL;
    std::copy(b->slices.begin(), b->slices.end(), slices);
    return GFQ_OK;
}

int gfq_batch_destroy(gfq_batch *b) {
    if (!b) return GFQ_OK;
    hipError_t e = hipSetDevice(b->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    batch_release(b);
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "batch destroy");
}

}  // extern "C"
