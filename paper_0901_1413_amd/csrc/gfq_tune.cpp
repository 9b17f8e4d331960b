// gfq_tune.cpp -- the autotuner: times candidate launch configurations on scratch operands
// and keeps the fastest per (device architecture, mode, field, size class).
//
// Single products (mode 0) are tuned on their own shape over slab width k, tile height and
// inner-dimension split; products inside batches (GFQ_TUNE_BATCH) over k and tile height,
// timed as a batch of identical products of the class's shape, since a batch supplies the
// parallelism that split supplies to a single product; Strassen-Winograd products
// (GFQ_TUNE_SW) over the number of levels (its entry keeps the levels in the k field).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gfq.h"
#include "gfq_host.h"
#include "gfq_internal.h"

using namespace gfq;

namespace {

typedef std::tuple<std::string, int, int, int, int, int> Key;   // arch, mode, q, bm, bl, bn

// A cached configuration; a single-product entry also keeps the rows and columns of the
// shape it was timed on (0 = the class's largest, 2^bucket).
struct Entry {
    gfq_config c;
    int64_t m = 0, n = 0;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;

int bucket(int64_t x) {
    int b = 6;
    while (b < 14 && ((int64_t)1 << b) < x) b++;
    return b;
}

// Architecture name of the current device (e.g. "gfx950"), looked up once per device.
bool arch_name(std::string *out) {
    static std::mutex mu;
    static std::vector<std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return false;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)names.size() <= dev) names.resize(dev + 1);
    if (names[dev].empty()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
        std::string a = prop.gcnArchName;
        names[dev] = a.substr(0, a.find(':'));
    }
    *out = names[dev];
    return true;
}

Key make_key(const std::string &arch, int mode, int q, int64_t m, int64_t l, int64_t n) {
    return Key(arch, mode, q, bucket(m), bucket(l), mode == GFQ_TUNE_BATCH ? 0 : bucket(n));
}

// Scratch device buffer for the tuner's operands (grown as needed, kept for the process).
struct Scratch { void *p = nullptr; size_t bytes = 0; };
Scratch g_scratch;

int scratch(size_t bytes, void **out, hipStream_t st) {
    if (g_scratch.bytes < bytes) {
        if (g_scratch.p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(g_scratch.p);
            g_scratch = Scratch();
        }
        if (hipMalloc(&g_scratch.p, bytes) != hipSuccess) return GFQ_ENOMEM;
        g_scratch.bytes = bytes;
        hipError_t e = launch_fill_random((u32 *)g_scratch.p, bytes / 4, 0x9e3779b9u, st);
        if (e != hipSuccess) return hip_fail(e, "tuner fill");
    }
    *out = g_scratch.p;
    return GFQ_OK;
}

size_t rup(size_t x) { return (x + 255) & ~(size_t)255; }

// Time one single-product configuration: the median of a few launches, in milliseconds.
double time_plain(int q, int64_t m, int64_t l, int64_t n, void *A, void *B, void *C, const gfq_config &c,
                  hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps) {
    if (gfq_matmul_config(q, m, l, n, A, B, C, &c) != GFQ_OK) return -1.0;
    std::vector<double> t;
    for (int r = 0; r < reps; r++) {
        (void)hipEventRecord(e0, st);
        if (gfq_matmul_config(q, m, l, n, A, B, C, &c) != GFQ_OK) return -1.0;
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

extern "C" {

int gfq_tune_lookup(int q, int64_t m, int64_t l, int64_t n, int mode, gfq_config *out) {
    if (!out) return GFQ_ENULL;
    std::string arch;
    if (!arch_name(&arch)) return GFQ_EAGAIN;
    std::lock_guard<std::mutex> lk(g_mu);
    const int md = (mode == GFQ_TUNE_BATCH || mode == GFQ_TUNE_SW) ? mode : 0;
    auto it = g_cache.find(make_key(arch, md, q, m, l, n));
    if (it == g_cache.end()) return GFQ_EAGAIN;
    *out = it->second.c;
    if (md == GFQ_TUNE_SW) return GFQ_OK;             // k holds the number of levels
    // the cached split belongs to the class; never split further than the slabs allow
    if (l > 0) {
        const int64_t S = (l + out->k - 1) / out->k;
        if (out->k > l) out->k = (int)l;
        out->split = (int)std::max<int64_t>(1, std::min<int64_t>(out->split, S));
    }
    // A product of the class with fewer tiles than the shape the entry was timed on would
    // leave compute units idle at that shape's split: its split is chosen again by the cost
    // model, for the tuned k and tile height, with slices down to 16 slabs, and never below
    // the tuned split (the model alone chose fewer slices than measured best in some fields).
    if (md == 0 && m > 0 && n > 0 && l >= out->k) {
        const int64_t tm = it->second.m ? it->second.m : (int64_t)1 << bucket(m);
        const int64_t tn = it->second.n ? it->second.n : (int64_t)1 << bucket(n);
        const MMPlan p = mm_plan(route_field(q, out->variant), out->k, out->rows);
        if (p.srb) {
            auto tiles = [&](int64_t mm, int64_t nn) {
                return ((int64_t)words_of(nn) + p.twd - 1) / p.twd * ((mm + p.TM - 1) / p.TM);
            };
            if (tiles(m, n) < tiles(tm, tn)) {
                const int tuned = out->split;
                fit_tiles(q, m, l, n, out, true, 16);
                const int64_t S = (l + out->k - 1) / out->k;
                out->split = (int)std::min<int64_t>(std::max(out->split, tuned), S);
            }
        }
    }
    return GFQ_OK;
}

int gfq_tune(int q, int64_t m, int64_t l, int64_t n, int mode, gfq_config *out) {
    if (!out) return GFQ_ENULL;
    if (!valid_field(q)) return GFQ_EFIELD;
    if (m <= 0 || l <= 0 || n <= 0 || m > (1 << 16) || l > (1 << 16) || n > (1 << 16)) return GFQ_EDIM;
    if (mode != 0 && mode != GFQ_TUNE_BATCH && mode != GFQ_TUNE_SW) return GFQ_EINVAL;
    std::string arch;
    if (!arch_name(&arch)) return GFQ_EHIP;
    hipStream_t st = current_stream();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GFQ_EHIP;
    gfq_config best = {};
    double best_rate = 0.0;
    int status = GFQ_OK;
    const double ops = 2.0 * (double)m * (double)l * (double)n;

    if (mode == GFQ_TUNE_SW) {
        // levels 0 .. GFQ_SW_MAX_LEVELS - 1 with the default leaf choice, median of 3
        const size_t ba = rup(gfq_packed_bytes(q, m, l)), bb = rup(gfq_packed_bytes(q, l, n));
        const size_t bc = rup(gfq_packed_bytes(q, m, n));
        void *base = nullptr;
        status = scratch(ba + bb + bc, &base, st);
        if (status == GFQ_OK) {
            char *A = (char *)base, *B = A + ba, *C = B + bb;
            for (int lev = 0; lev < GFQ_SW_MAX_LEVELS; lev++) {
                if (gfq_matmul_sw(q, m, l, n, A, B, C, lev, nullptr) != GFQ_OK) continue;
                std::vector<double> t;
                bool ok = true;
                for (int r = 0; ok && r < 3; r++) {
                    (void)hipEventRecord(e0, st);
                    ok = gfq_matmul_sw(q, m, l, n, A, B, C, lev, nullptr) == GFQ_OK;
                    (void)hipEventRecord(e1, st);
                    ok = ok && hipEventSynchronize(e1) == hipSuccess;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    t.push_back(ms);
                }
                if (!ok) continue;
                std::sort(t.begin(), t.end());
                const double ms = t[t.size() / 2];
                if (ms > 0 && ops / ms > best_rate * 1.02) {      // a level must win by 2%
                    best_rate = ops / ms;
                    best = gfq_config{lev, 0, 0, 0};
                }
            }
        }
    } else if (mode == 0) {
        const size_t ba = rup(gfq_packed_bytes(q, m, l)), bb = rup(gfq_packed_bytes(q, l, n));
        const size_t bc = rup(gfq_packed_bytes(q, m, n));
        void *base = nullptr;
        status = scratch(ba + bb + bc, &base, st);
        if (status == GFQ_OK) {
            char *A = (char *)base, *B = A + ba, *C = B + bb;
            const int reps = ops < 1e10 ? 7 : 3;
            // GF(4) also tries its Karatsuba form
            const int nvar = has_matrix_route(q) ? 2 : 1;
            for (int var = 0; var < nvar; var++)
            for (int k = 3; k <= KMAX; k++) {
                if (k > l) break;
                const int kq = route_field(q, var);
                for (int rows = 256; rows <= 2048; rows *= 2) {
                    const MMPlan pl = mm_plan(kq, k, rows);
                    if (!pl.srb) continue;
                    if (rows > 256 && pl.TM == mm_plan(kq, k, rows / 2).TM) continue;   // same tile
                    const int64_t S = (l + k - 1) / k;
                    const int64_t tiles = ((words_of(n) + pl.twd - 1) / pl.twd) * ((m + pl.TM - 1) / pl.TM);
                    for (int split = 1; split <= 16; split *= 2) {
                        if (split > 1 && (S / split < 8 || tiles * split > 2048)) break;
                        gfq_config c = {k, rows, split, var};
                        const double ms = time_plain(q, m, l, n, A, B, C, c, st, e0, e1, reps);
                        if (ms > 0 && ops / ms > best_rate) { best_rate = ops / ms; best = c; }
                    }
                }
            }
        }
    } else {
        // a batch of identical products of the class's shape, enough of them for ~1024 tiles
        const int64_t nb = 512;
        const int kcap = std::max(batch_kmax(q, 2), batch_kmax(q, max_rows_per_lane_batch(q)));
        const int64_t items_per = std::max<int64_t>(1, (m + 255) / 256);
        const int count = (int)std::max<int64_t>(16, std::min<int64_t>(2048, 1024 / items_per));
        const size_t ba = rup(gfq_packed_bytes(q, m, l)), bb = rup(gfq_packed_bytes(q, l, nb));
        const size_t bc = rup(gfq_packed_bytes(q, m, nb));
        void *base = nullptr;
        status = scratch(ba + bb + bc * count, &base, st);
        if (status == GFQ_OK) {
            char *A = (char *)base, *B = A + ba, *C0 = B + bb;
            std::vector<gfq_problem> probs(count);
            for (int i = 0; i < count; i++) probs[i] = gfq_problem{q, m, l, nb, A, B, C0 + bc * i};
            const double bops = ops / (double)n * (double)nb * count;
            for (int k = 3; k <= std::min<int64_t>(kcap, l); k++) {
                for (int rows : {256, 2048}) {
                    if (k > batch_kmax(q, rows <= 256 ? 2 : max_rows_per_lane_batch(q))) continue;
                    std::vector<gfq_config> cfg(count, gfq_config{k, rows, 1, 0});
                    gfq_batch *b = nullptr;
                    if (batch_create_with(count, probs.data(), cfg.data(), &b) != GFQ_OK) continue;
                    std::vector<double> t;
                    bool ok = gfq_batch_launch(b) == GFQ_OK;
                    for (int r = 0; ok && r < 3; r++) {
                        (void)hipEventRecord(e0, st);
                        ok = gfq_batch_launch(b) == GFQ_OK;
                        (void)hipEventRecord(e1, st);
                        ok = ok && hipEventSynchronize(e1) == hipSuccess;
                        float ms = 0.f;
                        (void)hipEventElapsedTime(&ms, e0, e1);
                        t.push_back(ms);
                    }
                    gfq_batch_destroy(b);
                    if (!ok || t.empty()) continue;
                    std::sort(t.begin(), t.end());
                    const double ms = t[t.size() / 2];
                    if (ms > 0 && bops / ms > best_rate) { best_rate = bops / ms; best = gfq_config{k, rows, 1, 0}; }
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != GFQ_OK) return status;
    if (best_rate <= 0.0) return GFQ_EHIP;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[make_key(arch, mode, q, m, l, n)] = mode == 0 ? Entry{best, m, n} : Entry{best, 0, 0};
    }
    *out = best;
    return GFQ_OK;
}

int gfq_tune_save(const char *path) {
    if (!path) return GFQ_ENULL;
    FILE *f = fopen(path, "w");
    if (!f) return GFQ_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    fprintf(f, "# arch mode q m_class l_class n_class k rows split variant [m n: shape timed, mode 0]\n");
    for (const auto &kv : g_cache) {
        const Key &k = kv.first;
        const gfq_config &c = kv.second.c;
        fprintf(f, "%s %d %d %d %d %d %d %d %d %d", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k),
                std::get<3>(k), std::get<4>(k), std::get<5>(k), c.k, c.rows, c.split, c.variant);
        if (std::get<1>(k) == 0)
            fprintf(f, " %lld %lld", (long long)(kv.second.m ? kv.second.m : (int64_t)1 << std::get<3>(k)),
                    (long long)(kv.second.n ? kv.second.n : (int64_t)1 << std::get<5>(k)));
        fprintf(f, "\n");
    }
    fclose(f);
    return GFQ_OK;
}

int gfq_tune_load(const char *path) {
    if (!path) return GFQ_ENULL;
    FILE *f = fopen(path, "r");
    if (!f) return GFQ_EINVAL;
    char line[256];
    int status = GFQ_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[64];
        int mode, q, bm, bl, bn, k, rows, split, variant = GFQ_VARIANT_ROWWISE;
        long long tm = 0, tn = 0;
        const int got = sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %lld %lld", arch, &mode, &q, &bm, &bl, &bn, &k,
                               &rows, &split, &variant, &tm, &tn);
        // the variant column may be absent; the shape columns (mode 0 only) too
        if ((got != 9 && got != 10 && got != 12) || (got == 12 && (mode != 0 || tm < 1 || tn < 1 ||
                                                                   tm > (1 << 16) || tn > (1 << 16)))) {
            status = GFQ_EINVAL;
            continue;
        }
        gfq_config c = {k, rows, split, variant};
        if (mode == GFQ_TUNE_SW) {                     // k holds the number of levels
            if (k < 0 || k > GFQ_SW_MAX_LEVELS) {
                status = GFQ_EINVAL;
                continue;
            }
            g_cache[Key(arch, mode, q, bm, bl, bn)] = Entry{gfq_config{k, 0, 0, 0}, 0, 0};
            continue;
        }
        const bool var_ok = variant == GFQ_VARIANT_ROWWISE || (variant == GFQ_VARIANT_KARATSUBA && has_matrix_route(q));
        // tile heights as gfq_matmul_config accepts them (mm_plan alone would clamp any
        // count, zero and negative ones included, to a valid tile)
        const bool rows_ok = rows == 256 || rows == 512 || rows == 1024 || rows == 2048;
        if (k < 1 || k > KMAX || !var_ok || !rows_ok ||
            mm_plan(route_field(q, variant), k, rows).srb == 0 || split < 1 ||
            split > 64) {
            status = GFQ_EINVAL;
            continue;
        }
        g_cache[Key(arch, mode, q, bm, bl, bn)] = Entry{c, tm, tn};
    }
    fclose(f);
    return status;
}

int gfq_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
    return GFQ_OK;
}

}  // extern "C"
