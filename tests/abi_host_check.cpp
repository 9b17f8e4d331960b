// Host-side paths of the C ABI, run without a GPU (built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library): the tuning-cache text parser
// and writer, configuration choice, every argument check that rejects a call before
// anything is launched, and batch planning (every tile and slab slice exactly once, the
// partial-sum items covering each sliced product, disjoint partial products).  Prints
// "ok <name>" per group, or "FAIL ..." and exits 1.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "gfq.h"
#include "gfq_host.h"

static void expect(bool ok, const char *what, long long a = 0) {
    if (!ok) {
        printf("FAIL %s %lld\n", what, a);
        fflush(stdout);
        exit(1);
    }
}

static std::string tmp_file(const char *name, const char *text) {
    const char *dir = getenv("ABI_CHECK_TMP");
    std::string path = std::string(dir ? dir : "/tmp") + "/" + name;
    FILE *f = fopen(path.c_str(), "w");
    expect(f != nullptr, "tmp file");
    fputs(text, f);
    fclose(f);
    return path;
}

int main() {
    // ---- tuning cache: good lines load and save; each bad line is refused ----
    gfq_tune_clear();
    const std::string good = tmp_file("good.txt",
                                      "# comment\n"
                                      "gfx950 0 3 13 13 13 8 1024 4 0 8192 8192\n"
                                      "gfx950 1 5 9 10 0 6 256 1 0\n"
                                      "gfx950 0 4 12 11 12 6 2048 1 1\n"
                                      "gfx950 2 5 13 13 13 3 0 0 0\n"
                                      "\n");
    expect(gfq_tune_load(good.c_str()) == GFQ_OK, "good tuning file");
    const std::string saved = std::string(getenv("ABI_CHECK_TMP") ? getenv("ABI_CHECK_TMP") : "/tmp") + "/saved.txt";
    expect(gfq_tune_save(saved.c_str()) == GFQ_OK, "save");
    gfq_tune_clear();
    expect(gfq_tune_load(saved.c_str()) == GFQ_OK, "reload of the saved file");
    const char *bad[] = {
        "gfx950 0 3 13 13 13 11 2048 2\n",             // k out of range
        "gfx950 0 3 13 13 13 7 2048 2 1\n",            // no matrix route for F_3
        "gfx950 0 3 13 13 13 7 0 2 0 8192 8192\n",     // a tile of 0 rows
        "gfx950 0 3 13 13 13 7 -512 2 0 8192 8192\n",  // negative rows
        "gfx950 0 3 13 13 13 7 2048 0 0\n",            // split 0
        "gfx950 0 3 13 13 13 7 2048 65 0\n",           // split 65
        "gfx950 0 3 13 13 13 7 2048 2 0 0 8192\n",     // a timed shape of 0 rows
        "gfx950 0 3 13 13 13 7 2048 2 0 8192\n",       // half a shape
        "gfx950 2 5 13 13 13 5 0 0 0\n",               // more levels than the maximum
        "gfx950 0 3\n",                                // truncated
        "gfx950 0 3 13 13 13 7 2048 2 0 99999999999 1\n",
        "xxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxx 0 3 13 13 "
        "13 7 2048 2\n",                               // an overlong architecture name
    };
    for (size_t i = 0; i < sizeof bad / sizeof bad[0]; i++) {
        const std::string p = tmp_file("bad.txt", bad[i]);
        expect(gfq_tune_load(p.c_str()) == GFQ_EINVAL, "bad tuning line refused", (long long)i);
    }
    expect(gfq_tune_load(nullptr) == GFQ_ENULL, "null path");
    expect(gfq_tune_load("/nonexistent/dir/file") == GFQ_EINVAL, "missing file");
    gfq_tune_clear();
    printf("ok tune_cache\n");

    // ---- configuration choice over many shapes (no device: the cache lookup declines) ----
    const int fields[] = {3, 4, 5, 7, 8, 9};
    const int64_t dims[] = {0, 1, 7, 31, 32, 33, 100, 511, 512, 513, 2500, 8192, 16384, 65535};
    for (int q : fields)
        for (int64_t m : dims)
            for (int64_t l : dims)
                for (int64_t n : {0, 1, 33, 1000, 16384}) {
                    gfq_config c;
                    expect(gfq_choose_config(q, m, l, n, &c) == GFQ_OK, "choose_config", q);
                    expect(c.k >= 1 && c.k <= 10 && c.split >= 1 && c.split <= 64, "config ranges", c.k);
                }
    gfq_config c;
    expect(gfq_choose_config(6, 8, 8, 8, &c) == GFQ_EFIELD, "field 6");
    expect(gfq_choose_config(3, -1, 8, 8, &c) == GFQ_EDIM, "negative m");
    expect(gfq_choose_config(3, 8, 8, 8, nullptr) == GFQ_ENULL, "null config");
    printf("ok choose_config\n");

    // ---- argument checks before any launch ----
    alignas(16) static unsigned char buf[1 << 16];
    void *A = buf, *B = buf + 16384, *C = buf + 32768;
    expect(gfq_packed_bytes(3, 10, 100) == 10 * 2 * 16, "packed bytes");
    expect(gfq_packed_bytes(2, 10, 100) == 0 && gfq_packed_bytes(3, -1, 10) == 0, "packed bytes invalid");
    expect(gfq_matmul(2, 4, 4, 4, A, B, C) == GFQ_EFIELD, "matmul field");
    expect(gfq_matmul(3, -1, 4, 4, A, B, C) == GFQ_EDIM, "matmul m < 0");
    expect(gfq_matmul(3, 4, (int64_t)1 << 24, 4, A, B, C) == GFQ_EDIM, "matmul l too large");
    expect(gfq_matmul(3, 4, 4, 4, nullptr, B, C) == GFQ_ENULL, "matmul null A");
    expect(gfq_matmul(3, 4, 4, 4, A, B, nullptr) == GFQ_ENULL, "matmul null C");
    expect(gfq_matmul(3, 4, 4, 4, buf + 8, B, C) == GFQ_EALIGN, "matmul misaligned A");
    expect(gfq_matmul(3, 4, 4, 4, A, B, A) == GFQ_EALIAS, "matmul C over A");
    expect(gfq_matmul(3, 0, 4, 4, nullptr, nullptr, nullptr) == GFQ_OK, "matmul m = 0 no-op");
    gfq_config bc = {11, 512, 1, 0};
    expect(gfq_matmul_config(3, 4, 4, 4, A, B, C, &bc) == GFQ_EINVAL, "config k 11");
    bc = {7, 300, 1, 0};
    expect(gfq_matmul_config(3, 4, 4, 4, A, B, C, &bc) == GFQ_EINVAL, "config rows 300");
    bc = {7, 512, 1, 1};
    expect(gfq_matmul_config(5, 4, 4, 4, A, B, C, &bc) == GFQ_EINVAL, "config matrix route for F_5");
    expect(gfq_matmul_noalloc(3, 4, 4, 4, A, B, A, nullptr) == GFQ_EALIAS, "noalloc alias");
    expect(gfq_matmul_noalloc(3, 4, 4, 4, A, B, C, &bc) == GFQ_EINVAL, "noalloc bad config");
    expect(gfq_matmul_sw(3, 4, 4, 4, A, B, C, 5, nullptr) == GFQ_EINVAL, "sw levels 5");
    expect(gfq_matmul_sw(3, 4, 4, 4, A, B, C, -2, nullptr) == GFQ_EINVAL, "sw levels -2");
    expect(gfq_pack(3, 4, 4, nullptr, 4, C) == GFQ_ENULL, "pack null src");
    expect(gfq_pack(3, 4, 8, (const uint8_t *)A, 4, C) == GFQ_EDIM, "pack ld < cols");
    expect(gfq_pack(3, 4, 4, (const uint8_t *)A, 4, buf + 4) == GFQ_EALIGN, "pack misaligned dst");
    expect(gfq_pack(3, 4, 4, (const uint8_t *)A, 4, A) == GFQ_EALIAS, "pack dst over src");
    expect(gfq_unpack(3, 4, 4, buf + 4, (uint8_t *)C, 4) == GFQ_EALIGN, "unpack misaligned src");
    expect(gfq_unpack(9, 4, 4, A, (uint8_t *)C, 2) == GFQ_EDIM, "unpack ld < cols");
    gfq_problem probs[2] = {{3, 4, 4, 4, A, B, C}, {3, 4, 4, 4, A, B, A}};
    expect(gfq_matmul_batched(2, probs) == GFQ_EALIAS, "batch rejects one bad product");
    expect(gfq_matmul_batched(-1, probs) == GFQ_EINVAL, "batch count < 0");
    expect(gfq_matmul_batched(1, nullptr) == GFQ_ENULL, "batch null");
    gfq_batch *bt = nullptr;
    expect(gfq_batch_create(2, probs, &bt) == GFQ_EALIAS && bt == nullptr, "batch create rejects");
    expect(gfq_batch_launch(nullptr) == GFQ_ENULL, "batch launch null");
    expect(gfq_batch_launch_persistent(nullptr) == GFQ_ENULL, "persistent batch launch null");
    expect(gfq_batch_slab_widths(nullptr, nullptr) == GFQ_ENULL, "batch widths null");
    expect(gfq_batch_slices(nullptr, nullptr) == GFQ_ENULL, "batch slices null");
    expect(gfq_server_submit(nullptr, nullptr, 1) == GFQ_ENULL, "server null");
    int got = 0;
    expect(gfq_server_poll(nullptr, nullptr, 1, &got, 0) == GFQ_ENULL, "server poll null");
    gfq_server_opts so = {};
    so.slots = 9;
    gfq_server *srv = nullptr;
    expect(gfq_server_create(&so, &srv) == GFQ_EINVAL && srv == nullptr, "server slots 9");
    so = {};
    so.watchdog_s = -1.0;
    expect(gfq_server_create(&so, &srv) == GFQ_EINVAL, "server negative watchdog");
    expect(gfq_server_destroy(nullptr) == GFQ_OK, "server destroy null");
    float ms = 0.f;
    double amount = 0.0;
    expect(gfq_probe_copy(A, C, 7, &ms) == GFQ_EINVAL, "probe copy size");
    expect(gfq_probe_valu(0, 1, (uint32_t *)A, &amount, &ms) == GFQ_EINVAL, "probe blocks");
    for (int s = -12; s <= 1; s++) expect(gfq_strerror(s) != nullptr && gfq_strerror(s)[0] != 0, "strerror", s);
    printf("ok validation\n");
    // ---- batch planning: items, slab slices, partial-sum items (no device: default configs) ----
    {
        static unsigned char mem[1 << 12];
        auto plan_check = [&](const std::vector<gfq_problem> &probs, bool slice, int *sliced) {
            const int count = (int)probs.size();
            std::vector<gfq::BatchProd> prods(count);
            std::vector<gfq::BatchGroup> groups;
            size_t nitems = 0;
            gfq::BatchSlicing sl;
            gfq::plan_batch(count, probs.data(), nullptr, prods.data(), &groups, &nitems, slice ? &sl : nullptr);
            // every (product, tile, slice) exactly once, each list's items contiguous
            std::map<std::tuple<unsigned, int, int, unsigned>, int> seen;
            size_t off = 0;
            for (const gfq::BatchGroup &g : groups) {
                expect(g.item_off == off, "group offsets consecutive", (long long)off);
                off += g.items.size();
                for (const gfq::BatchItem &it : g.items) {
                    expect(it.prod < (unsigned)count && it.slice < prods[it.prod].slices, "item in range", it.prod);
                    expect(seen[std::make_tuple(it.prod, (int)it.tx, (int)it.ty, it.slice)]++ == 0, "item once", it.prod);
                }
            }
            expect(off == nitems, "item count", (long long)nitems);
            *sliced = 0;
            std::vector<long long> reduce_units(count, 0), covered(count, 0);
            for (const gfq::ReduceItem &r : sl.reduce) {
                expect(r.prod < (unsigned)count && prods[r.prod].slices > 1, "reduce item of a sliced product", r.prod);
                expect(r.first == (unsigned)covered[r.prod], "reduce items contiguous", r.prod);
                covered[r.prod] += r.count;
                reduce_units[r.prod]++;
            }
            std::vector<std::pair<size_t, size_t>> spans;
            for (int i = 0; i < count; i++) {
                const gfq::BatchProd &bp = prods[i];
                const gfq::MMArgs &a = bp.a;
                long long tiles = 0;
                for (auto &kv : seen)
                    if (std::get<0>(kv.first) == (unsigned)i && std::get<3>(kv.first) == 0) tiles++;
                expect(bp.units == tiles * bp.slices + reduce_units[i], "units", i);
                if (bp.slices > 1) {
                    ++*sliced;
                    expect(slice, "sliced only when asked", i);
                    expect(a.slabs_per_split >= 8 && bp.slices <= 64, "slice bounds", a.slabs_per_split);
                    expect((long long)a.slabs_per_split * (bp.slices - 1) < a.S && (long long)a.slabs_per_split * bp.slices >= a.S,
                           "slices cover the slabs", i);
                    expect(covered[i] == (long long)a.m * (a.Wn / 4), "partial sums cover C", i);
                    expect(a.split_stride == (size_t)a.m * gfq::planes_of(bp.q) * a.Wn, "partial stride", i);
                    spans.push_back(std::make_pair(sl.part_off[i], sl.part_off[i] + bp.slices * a.split_stride));
                } else {
                    expect(a.slabs_per_split >= a.S, "a whole product has one slice", i);
                }
            }
            std::sort(spans.begin(), spans.end());
            for (size_t j = 0; j < spans.size(); j++) {
                expect(spans[j].second <= sl.partial_words, "partials inside the workspace", (long long)j);
                if (j) expect(spans[j - 1].second <= spans[j].first, "partials disjoint", (long long)j);
            }
        };
        std::vector<gfq_problem> probs;
        // long inner dimensions, few tiles each: sliced
        for (int q : {3, 4, 5, 7, 8, 9}) probs.push_back(gfq_problem{q, 300, 20000, 700, mem, mem, mem});
        // and some small products beside them
        for (int i = 0; i < 40; i++) probs.push_back(gfq_problem{3 + (i % 2) * 2, 64 + i, 100 + 7 * i, 33 + 5 * i, mem, mem, mem});
        int sliced = 0;
        plan_check(probs, true, &sliced);
        expect(sliced == 6, "the six long products sliced", sliced);
        plan_check(probs, false, &sliced);
        expect(sliced == 0, "no slices without slicing", sliced);
        // many products of similar size: none sliced
        std::vector<gfq_problem> even;
        for (int i = 0; i < 512; i++) even.push_back(gfq_problem{7, 512, 512, 512, mem, mem, mem});
        plan_check(even, true, &sliced);
        expect(sliced == 0, "an even batch is not sliced", sliced);
        // degenerate products beside a sliced one
        std::vector<gfq_problem> degen = {{5, 0, 9000, 64, mem, mem, mem}, {5, 64, 0, 64, mem, mem, mem},
                                          {5, 64, 9000, 0, mem, mem, mem}, {5, 64, 9000, 64, mem, mem, mem}};
        plan_check(degen, true, &sliced);
        expect(sliced == 1, "one of four sliced", sliced);
        printf("ok plan_batch\n");
    }
    printf("ok all\n");
    return 0;
}
