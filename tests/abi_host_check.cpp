// Host-side paths of the C ABI, run without a GPU (built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library): the tuning-cache text parser
// and writer, configuration choice, and every argument check that rejects a call before
// anything is launched.  Prints "ok <name>" per group, or "FAIL ..." and exits 1.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "gfq.h"

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
    expect(gfq_batch_slab_widths(nullptr, nullptr) == GFQ_ENULL, "batch widths null");
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
    printf("ok all\n");
    return 0;
}
