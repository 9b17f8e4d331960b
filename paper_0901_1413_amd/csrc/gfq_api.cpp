// gfq_api.cpp -- the C ABI declared in include/gfq.h: argument validation, launch
// configuration, workspace and stream handling around the kernel launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "gfq.h"
#include "gfq_host.h"
#include "gfq_sw.h"
#include "gfq_internal.h"

using namespace gfq;

namespace {

thread_local hipStream_t t_stream = nullptr;
thread_local char t_hip_error[256] = "";


// Optional per-launch timing (gfq_set_timing).
struct TimedLaunch { hipEvent_t e0, e1; int kind; };   // kind 0: product, 1: partial sum
thread_local bool t_timing = false;
thread_local std::vector<TimedLaunch> t_timed;

hipEvent_t timing_mark() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    if (hipEventRecord(e, t_stream) != hipSuccess) { (void)hipEventDestroy(e); return nullptr; }
    return e;
}

// Launch f() and, when timing is on, bracket it with events.
template <typename Fn> hipError_t timed(int kind, Fn f) {
    if (!t_timing) return f();
    hipEvent_t e0 = timing_mark();
    hipError_t e = f();
    hipEvent_t e1 = timing_mark();
    if (e0 && e1) t_timed.push_back({e0, e1, kind});
    else {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    return e;
}

// Device workspace for split-l partial products: one growing buffer per (device, stream),
// so products in flight on different streams never share partial sums.  A buffer is only
// replaced after its stream has finished the work queued on it; buffers live until the
// process ends (the library cannot tell when a caller destroys a stream).
struct Workspace {
    std::mutex mu;
    std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> buf;
};
Workspace g_ws;

int workspace(size_t need, hipStream_t st, void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    std::pair<void *, size_t> &b = g_ws.buf[std::make_pair(dev, st)];
    if (b.second < need) {
        if (b.first) {
            // kernels queued on this stream may still read the old buffer
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(b.first);
            b = std::make_pair(nullptr, (size_t)0);
        }
        size_t sz = std::max(need, (size_t)64 << 20);
        void *p = nullptr;
        e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            hip_fail(e, "hipMalloc(workspace)");
            return GFQ_ENOMEM;
        }
        b = std::make_pair(p, sz);
    }
    *out = b.first;
    return GFQ_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return na && nb && pa < pb + nb && pb < pa + na;
}

// Kernel field of a product over API field q in configuration c.
int kernel_field(int q, const gfq_config &c) {
    return route_field(q, c.variant);
}

}  // namespace

// Tile height and inner-dimension slices for slab width c->k (kernel field of c) on an
// m x l x n product: the fewest slab steps on the busiest compute unit, i.e. ceil(workgroups
// / 256) rounds of (slabs per slice + 2) steps of a TM-row tile (the 2 stand for a slice's
// prologue and store), each step weighted by the table it builds; among near-equal choices
// the tallest tile and the fewest slices (least partial-sum traffic) win; a slice holds at
// least min_slabs slabs.  keep_rows: the tile height c->rows stays and only the slices are
// chosen.
void gfq::fit_tiles(int q, int64_t m, int64_t l, int64_t n, gfq_config *c, bool keep_rows, int min_slabs) {
    const int kq = kernel_field(q, *c), kk = c->k;
    const int twd = twd_of(srb_for(kq, kk));
    const int64_t ctiles = (words_of(n) + twd - 1) / twd;
    const int64_t S = l > 0 ? (l + kk - 1) / kk : 1;
    const int64_t max_split = std::max<int64_t>(1, std::min<int64_t>(S / std::max(1, min_slabs), 64));
    double best_cost = 0.0;
    const int rows_hi = keep_rows ? c->rows : 2048, rows_lo = keep_rows ? c->rows : 256;
    c->rows = rows_lo;
    c->split = 1;
    for (int rows = rows_hi; rows >= rows_lo && rows > 0; rows >>= 1) {
        const MMPlan p = mm_plan(kq, kk, rows);
        if (!p.srb) continue;
        const int64_t tiles = ctiles * ((m + p.TM - 1) / p.TM);
        for (int64_t split = 1; split <= max_split; split *= 2) {
            if (tiles == 0 && split > 1) break;          // m or n = 0: no tiles
            const int64_t rounds = (tiles * split + 255) / 256;
            const double steps = (double)((S + split - 1) / split + 2);
            const double cost = (double)rounds * p.TM * steps * (1.0 + (double)(1 << kk) / p.TM);
            if (best_cost == 0.0 || cost < best_cost * 0.98) {
                best_cost = cost;
                c->rows = rows;
                c->split = (int)split;
            }
        }
    }
}

namespace {

// Batches launched by gfq_matmul_batched stay alive until their launch has completed;
// each call (and gfq_sync) releases the ones whose completion event has fired.
struct PendingBatch { gfq_batch *b; hipEvent_t done; };
thread_local std::vector<PendingBatch> t_pending;

void release_finished(bool wait) {
    std::vector<PendingBatch> keep;
    for (PendingBatch &p : t_pending) {
        hipError_t q = wait ? hipEventSynchronize(p.done) : hipEventQuery(p.done);
        if (q == hipSuccess) {
            (void)hipEventDestroy(p.done);
            gfq_batch_destroy(p.b);
        } else {
            keep.push_back(p);
        }
    }
    t_pending.swap(keep);
}
}  // namespace

int gfq::hip_fail(hipError_t e, const char *what) {
    snprintf(t_hip_error, sizeof t_hip_error, "%s: %s", what, hipGetErrorString(e));
    return GFQ_EHIP;
}

hipStream_t gfq::current_stream() { return t_stream; }

int gfq::validate_mm(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C) {
    if (!valid_field(q)) return GFQ_EFIELD;
    if (m < 0 || l < 0 || n < 0 || l >= GFQ_MAX_DIM || m >= ((int64_t)1 << 28) || n >= ((int64_t)1 << 28))
        return GFQ_EDIM;
    if (m == 0 || n == 0) return GFQ_OK;
    if (!C || (l > 0 && (!A || !B))) return GFQ_ENULL;
    if (((uintptr_t)C & 15) || (l > 0 && (((uintptr_t)A & 15) || ((uintptr_t)B & 15)))) return GFQ_EALIGN;
    const size_t bc = gfq_packed_bytes(q, m, n);
    if (l > 0 && (overlaps(C, bc, A, gfq_packed_bytes(q, m, l)) || overlaps(C, bc, B, gfq_packed_bytes(q, l, n))))
        return GFQ_EALIAS;
    return GFQ_OK;
}


int gfq::check_config(int q, const gfq_config &c) {
    if (c.k < 1 || c.k > KMAX) return GFQ_EINVAL;
    if (c.rows != 256 && c.rows != 512 && c.rows != 1024 && c.rows != 2048) return GFQ_EINVAL;
    if (c.split < 1 || c.split > 64) return GFQ_EINVAL;
    if (c.variant != GFQ_VARIANT_ROWWISE && !(c.variant == GFQ_VARIANT_KARATSUBA && has_matrix_route(q)))
        return GFQ_EINVAL;
    if (mm_plan(kernel_field(q, c), c.k, c.rows).srb == 0) return GFQ_EINVAL;
    return GFQ_OK;
}

int gfq::matmul_into(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C,
                     const gfq_config *cfg, void *fixed_ws, size_t fixed_bytes) {
    int st = validate_mm(q, m, l, n, A, B, C);
    if (st != GFQ_OK) return st;
    if (m == 0 || n == 0) return GFQ_OK;
    gfq_config c;
    if (cfg) {
        c = *cfg;
        st = check_config(q, c);
        if (st != GFQ_OK) return st;
    } else {
        gfq_choose_config(q, m, l, n, &c);
    }
    const int P = planes_of(q);
    const int Wn = words_of(n);
    if (l == 0) {
        hipError_t e = launch_fill_zero(C, gfq_packed_bytes(q, m, n), t_stream);
        return e == hipSuccess ? GFQ_OK : hip_fail(e, "zero fill");
    }
    MMArgs a;
    a.A = (const u32 *)A;
    a.B = (const u32 *)B;
    a.m = (int)m;
    a.l = (int)l;
    a.n = (int)n;
    a.Wl = words_of(l);
    a.Wn = Wn;
    a.k = c.k;
    a.S = (int)((l + c.k - 1) / c.k);
    a.split_stride = (size_t)m * P * Wn;
    int split = std::min(c.split, a.S);
    if (fixed_ws) {
        // the slices' partial products must fit the fixed region: a chosen split is capped,
        // an explicit one that does not fit is refused
        const size_t fit = fixed_bytes / (a.split_stride * 4);
        if (split > 1 && (size_t)split > fit) {
            if (cfg) return GFQ_EBUDGET;
            split = (int)std::max<size_t>(1, std::min<size_t>(fit, (size_t)split));
        }
    }
    a.slabs_per_split = (a.S + split - 1) / split;
    split = (a.S + a.slabs_per_split - 1) / a.slabs_per_split;
    const int kq = kernel_field(q, c);
    const MMPlan plan = mm_plan(kq, c.k, c.rows);
    // launches are timed only on the allocating path (events are created per launch)
    const bool may_time = fixed_ws == nullptr;
    if (split == 1) {
        a.out = (u32 *)C;
        hipError_t e = may_time ? timed(0, [&] { return launch_matmul(kq, a, plan, t_stream); })
                                : launch_matmul(kq, a, plan, t_stream);
        return e == hipSuccess ? GFQ_OK : hip_fail(e, "matmul launch");
    }
    void *ws = fixed_ws;
    if (!ws) {
        st = workspace(a.split_stride * 4 * split, t_stream, &ws);
        if (st != GFQ_OK) return st;
    }
    a.out = (u32 *)ws;
    auto product = [&] { return launch_matmul(kq, a, plan, t_stream); };
    auto partial_sum = [&] {
        return launch_reduce(q, (const u32 *)ws, (u32 *)C, (int)m, (int)n, Wn, split, a.split_stride, t_stream);
    };
    hipError_t e = may_time ? timed(0, product) : product();
    if (e != hipSuccess) return hip_fail(e, "matmul launch");
    e = may_time ? timed(1, partial_sum) : partial_sum();
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "reduce launch");
}

extern "C" {

size_t gfq_packed_bytes(int q, int64_t rows, int64_t cols) {
    if (!valid_field(q) || rows < 0 || cols < 0) return 0;
    return (size_t)rows * planes_of(q) * words_of(cols) * 4;
}

int gfq_set_stream(void *s) {
    t_stream = (hipStream_t)s;
    return GFQ_OK;
}

int gfq_sync(void) {
    hipError_t e = hipStreamSynchronize(t_stream);
    release_finished(false);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "asynchronous error");
    return GFQ_OK;
}

const char *gfq_last_hip_error(void) { return t_hip_error; }

int gfq_set_timing(int on) {
    t_timing = on != 0;
    return GFQ_OK;
}

int gfq_timing_read(double *product_ms, int *product_launches, double *reduce_ms, int *reduce_launches) {
    double ms[2] = {0.0, 0.0};
    int cnt[2] = {0, 0};
    int status = GFQ_OK;
    for (TimedLaunch &t : t_timed) {
        float x = 0.f;
        hipError_t e = hipEventSynchronize(t.e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&x, t.e0, t.e1);
        if (e != hipSuccess) status = hip_fail(e, "timing events");
        ms[t.kind] += x;
        cnt[t.kind] += 1;
        (void)hipEventDestroy(t.e0);
        (void)hipEventDestroy(t.e1);
    }
    t_timed.clear();
    if (product_ms) *product_ms = ms[0];
    if (product_launches) *product_launches = cnt[0];
    if (reduce_ms) *reduce_ms = ms[1];
    if (reduce_launches) *reduce_launches = cnt[1];
    return status;
}

const char *gfq_strerror(int s) {
    switch (s) {
    case GFQ_OK: return "ok";
    case GFQ_EINVAL: return "invalid argument";
    case GFQ_EFIELD: return "unsupported field (q must be 3, 4, 5 or 7)";
    case GFQ_EDIM: return "invalid dimension or leading dimension";
    case GFQ_ENULL: return "null pointer";
    case GFQ_EALIGN: return "packed buffer not 16-byte aligned";
    case GFQ_EALIAS: return "output overlaps an input";
    case GFQ_ENOMEM: return "workspace allocation failed";
    case GFQ_EHIP: return "HIP runtime error";
    case GFQ_EBUDGET: return "request exceeds the memory budget";
    case GFQ_EAGAIN: return "not ready, try again";
    default: return "unknown status";
    }
}

int gfq_pack(int q, int64_t rows, int64_t cols, const uint8_t *src, int64_t ld_src, void *dst) {
    if (!valid_field(q)) return GFQ_EFIELD;
    if (rows < 0 || cols < 0 || rows >= ((int64_t)1 << 28) || cols >= ((int64_t)1 << 28)) return GFQ_EDIM;
    if (rows == 0 || cols == 0) return GFQ_OK;
    if (ld_src < cols) return GFQ_EDIM;
    if (!src || !dst) return GFQ_ENULL;
    if ((uintptr_t)dst & 15) return GFQ_EALIGN;
    if (overlaps(src, (size_t)((rows - 1) * ld_src + cols), dst, gfq_packed_bytes(q, rows, cols))) return GFQ_EALIAS;
    hipError_t e = launch_pack(q, src, ld_src, (u32 *)dst, (int)rows, (int)cols, words_of(cols), t_stream);
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "pack launch");
}

int gfq_unpack(int q, int64_t rows, int64_t cols, const void *src, uint8_t *dst, int64_t ld_dst) {
    if (!valid_field(q)) return GFQ_EFIELD;
    if (rows < 0 || cols < 0 || rows >= ((int64_t)1 << 28) || cols >= ((int64_t)1 << 28)) return GFQ_EDIM;
    if (rows == 0 || cols == 0) return GFQ_OK;
    if (ld_dst < cols) return GFQ_EDIM;
    if (!src || !dst) return GFQ_ENULL;
    if ((uintptr_t)src & 15) return GFQ_EALIGN;
    if (overlaps(dst, (size_t)((rows - 1) * ld_dst + cols), src, gfq_packed_bytes(q, rows, cols))) return GFQ_EALIAS;
    hipError_t e = launch_unpack(q, (const u32 *)src, dst, ld_dst, (int)rows, (int)cols, words_of(cols), t_stream);
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "unpack launch");
}

int gfq_choose_config(int q, int64_t m, int64_t l, int64_t n, gfq_config *out) {
    if (!valid_field(q)) return GFQ_EFIELD;
    if (!out) return GFQ_ENULL;
    if (m < 0 || l < 0 || n < 0) return GFQ_EDIM;
    if (m > 0 && n > 0 && l > 0 && gfq_tune_lookup(q, m, l, n, 0, out) == GFQ_OK) return GFQ_OK;
    // k = 7: the widest slab whose two tables fit LDS with 128-bit reads that conflict at
    // most two ways (measured best or near-best for every field on the large products).
    gfq_config best = {};
    best.k = (l > 0 && l < 7) ? (int)l : 7;
    best.variant = GFQ_VARIANT_ROWWISE;
    // where k = 7 means 32-word tiles (three- and four-plane tables), a product at most 16
    // words wide would leave half of every tile idle: k = 6 keeps 16-word tiles
    if (best.k == 7 && twd_of(srb_for(kernel_field(q, best), 7)) == 32 && words_of(n) <= 16) best.k = 6;
    fit_tiles(q, m, l, n, &best);
    *out = best;
    return GFQ_OK;
}

int gfq_matmul_config(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C,
                      const gfq_config *cfg) {
    return matmul_into(q, m, l, n, A, B, C, cfg, nullptr, 0);
}

int gfq_matmul(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C) {
    return gfq_matmul_config(q, m, l, n, A, B, C, nullptr);
}

int gfq_matmul_sw(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C, int levels,
                  const gfq_config *leaf) {
    int st = validate_mm(q, m, l, n, A, B, C);
    if (st != GFQ_OK) return st;
    if (levels == GFQ_SW_AUTO) {
        gfq_config t;
        levels = (m > 0 && l > 0 && n > 0 && gfq_tune_lookup(q, m, l, n, GFQ_TUNE_SW, &t) == GFQ_OK) ? t.k : 0;
    }
    if (levels < 0 || levels > GFQ_SW_MAX_LEVELS) return GFQ_EINVAL;
    if (leaf) {
        st = check_config(q, *leaf);
        if (st != GFQ_OK) return st;
    }
    if (levels == 0) return gfq_matmul_config(q, m, l, n, A, B, C, leaf);
    if (m == 0 || n == 0) return GFQ_OK;
    if (l == 0) {
        hipError_t e = launch_fill_zero(C, gfq_packed_bytes(q, m, n), t_stream);
        return e == hipSuccess ? GFQ_OK : hip_fail(e, "zero fill");
    }
    // dimensions per level (level 0 is the product itself) and the workspace of levels
    // 1..L: 7^i left operands, right operands and products of level i's shape
    int64_t dm[GFQ_SW_MAX_LEVELS + 1], dl[GFQ_SW_MAX_LEVELS + 1], dn[GFQ_SW_MAX_LEVELS + 1];
    size_t offA[GFQ_SW_MAX_LEVELS + 1] = {}, offB[GFQ_SW_MAX_LEVELS + 1] = {}, offC[GFQ_SW_MAX_LEVELS + 1] = {};
    size_t szA[GFQ_SW_MAX_LEVELS + 1] = {}, szB[GFQ_SW_MAX_LEVELS + 1] = {}, szC[GFQ_SW_MAX_LEVELS + 1] = {};
    dm[0] = m, dl[0] = l, dn[0] = n;
    size_t total = 0, count = 1;
    for (int i = 1; i <= levels; i++) {
        dm[i] = sw_half_rows(dm[i - 1]);
        dl[i] = sw_half_cols(dl[i - 1]);
        dn[i] = sw_half_cols(dn[i - 1]);
        count *= 7;
        szA[i] = gfq_packed_bytes(q, dm[i], dl[i]);
        szB[i] = gfq_packed_bytes(q, dl[i], dn[i]);
        szC[i] = gfq_packed_bytes(q, dm[i], dn[i]);
        offA[i] = total, total += count * szA[i];
        offB[i] = total, total += count * szB[i];
        offC[i] = total, total += count * szC[i];
    }
    // the leaves: one strided launch of count products.  Without a given configuration the
    // slab width and route are those chosen for one leaf, and the tile height and slices
    // are fitted to all the leaves' tiles together (count leaves stacked as one tall
    // product).
    gfq_config c;
    if (leaf) {
        c = *leaf;
    } else {
        gfq_choose_config(q, dm[levels], dl[levels], dn[levels], &c);
        fit_tiles(q, (int64_t)count * dm[levels], dl[levels], dn[levels], &c);
    }
    const int kq = kernel_field(q, c);
    const MMPlan plan = mm_plan(kq, c.k, c.rows);
    if (!plan.srb) return GFQ_EINVAL;
    MMArgs a;
    a.m = (int)dm[levels];
    a.l = (int)dl[levels];
    a.n = (int)dn[levels];
    a.Wl = words_of(a.l);
    a.Wn = words_of(a.n);
    a.k = c.k;
    a.S = (a.l + a.k - 1) / a.k;
    int split = std::min(c.split, a.S);
    split = std::min<int64_t>(split, 65535 / (int64_t)count);      // grid.z = leaves x slices <= 65535
    if ((int64_t)count * a.m >= ((int64_t)1 << 31)) split = 1;   // the partial sums run as one tall matrix
    a.slabs_per_split = (a.S + split - 1) / split;
    split = (a.S + a.slabs_per_split - 1) / a.slabs_per_split;
    // slice s of every leaf goes to a region of its own: the leaves' partial products of a
    // slice form one tall (count * m) x n matrix, summed by one partial-sum launch
    const size_t part_off = total;
    a.split_stride = count * szC[levels] / 4;
    if (split > 1) total += split * count * szC[levels];
    void *wsv = nullptr;
    st = workspace(total, t_stream, &wsv);
    if (st != GFQ_OK) return st;
    char *ws = (char *)wsv;
    hipError_t e = hipSuccess;
    size_t parents = 1;
    for (int i = 0; i < levels && e == hipSuccess; i++, parents *= 7) {
        const u32 *inA = i == 0 ? (const u32 *)A : (const u32 *)(ws + offA[i]);
        const u32 *inB = i == 0 ? (const u32 *)B : (const u32 *)(ws + offB[i]);
        e = timed(1, [&] {
            return launch_sw_split(q, true, inA, szA[i] / 4, (u32 *)(ws + offA[i + 1]), szA[i + 1] / 4, (int)parents,
                                   (int)dm[i], (int)dl[i], (int)dm[i + 1], (int)dl[i + 1], t_stream);
        });
        if (e == hipSuccess)
            e = timed(1, [&] {
                return launch_sw_split(q, false, inB, szB[i] / 4, (u32 *)(ws + offB[i + 1]), szB[i + 1] / 4,
                                       (int)parents, (int)dl[i], (int)dn[i], (int)dl[i + 1], (int)dn[i + 1], t_stream);
            });
    }
    if (e != hipSuccess) return hip_fail(e, "Strassen-Winograd split");
    a.A = (const u32 *)(ws + offA[levels]);
    a.B = (const u32 *)(ws + offB[levels]);
    a.out = (u32 *)(ws + (split > 1 ? part_off : offC[levels]));
    const MMStrides sd = {(int)count, szA[levels] / 4, szB[levels] / 4, szC[levels] / 4};
    e = timed(0, [&] { return launch_matmul_strided(kq, a, plan, sd, t_stream); });
    if (e != hipSuccess) return hip_fail(e, "matmul launch");
    if (split > 1) {
        e = timed(1, [&] {
            return launch_reduce(q, (const u32 *)(ws + part_off), (u32 *)(ws + offC[levels]), (int)(count * a.m), a.n,
                                 a.Wn, split, a.split_stride, t_stream);
        });
        if (e != hipSuccess) return hip_fail(e, "reduce launch");
    }
    parents = count / 7;
    for (int i = levels - 1; i >= 0 && e == hipSuccess; i--, parents /= 7) {
        u32 *out = i == 0 ? (u32 *)C : (u32 *)(ws + offC[i]);
        e = timed(1, [&] {
            return launch_sw_merge(q, (const u32 *)(ws + offC[i + 1]), szC[i + 1] / 4, out, szC[i] / 4, (int)parents,
                                   (int)dm[i], (int)dn[i], (int)dm[i + 1], (int)dn[i + 1], t_stream);
        });
    }
    return e == hipSuccess ? GFQ_OK : hip_fail(e, "Strassen-Winograd merge");
}


int gfq_matmul_batched(int count, const gfq_problem *problems) {
    if (count < 0) return GFQ_EINVAL;
    if (count == 0) return GFQ_OK;
    if (!problems) return GFQ_ENULL;
    release_finished(false);
    gfq_batch *b = nullptr;
    int st = gfq_batch_create(count, problems, &b);
    if (st != GFQ_OK) return st;
    st = gfq_batch_launch_persistent(b);
    hipEvent_t done = nullptr;
    hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(done, t_stream);
    if (e != hipSuccess) {
        if (done) (void)hipEventDestroy(done);
        (void)hipStreamSynchronize(t_stream);
        gfq_batch_destroy(b);
        return st != GFQ_OK ? st : hip_fail(e, "batch completion event");
    }
    t_pending.push_back({b, done});
    return st;
}

}  // extern "C"
