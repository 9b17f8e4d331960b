/* The oracle's C entry point under AddressSanitizer and UndefinedBehaviorSanitizer: every
 * field on ragged shapes with leading dimensions larger than the rows, the degenerate
 * shapes and the rejected arguments; products are checked against the identity and zero
 * laws and against the same product on one thread.  Prints "ok all" or "FAIL ..." and
 * exits 1. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int gfq_oracle_matmul(int q, int64_t m, int64_t l, int64_t n, const uint8_t *A, int64_t lda, const uint8_t *B,
                      int64_t ldb, uint8_t *C, int64_t ldc, int nthreads);

static void fail(const char *what, long long a) {
    printf("FAIL %s %lld\n", what, a);
    exit(1);
}

static uint32_t rnd_state = 12345u;
static uint32_t rnd(void) {
    rnd_state = rnd_state * 1664525u + 1013904223u;
    return rnd_state >> 8;
}

int main(void) {
    const int fields[] = {3, 4, 5, 7, 8, 9};
    const int64_t shapes[][3] = {{1, 1, 1}, {3, 5, 7}, {17, 33, 65}, {64, 1, 64}, {1, 200, 1}, {40, 129, 31}};
    for (int fi = 0; fi < 6; fi++) {
        const int q = fields[fi];
        for (int si = 0; si < 6; si++) {
            const int64_t m = shapes[si][0], l = shapes[si][1], n = shapes[si][2];
            const int64_t lda = l + 3, ldb = n + 5, ldc = n + 7;
            uint8_t *A = malloc((size_t)(m * lda)), *B = malloc((size_t)(l * ldb));
            uint8_t *C = malloc((size_t)(m * ldc)), *C1 = malloc((size_t)(m * ldc));
            uint8_t *I = calloc((size_t)(l * l), 1), *AI = malloc((size_t)(m * l));
            for (int64_t i = 0; i < m * lda; i++) A[i] = (uint8_t)(rnd() % q);
            for (int64_t i = 0; i < l * ldb; i++) B[i] = (uint8_t)(rnd() % q);
            memset(C, 0xEE, (size_t)(m * ldc));
            memcpy(C1, C, (size_t)(m * ldc));
            if (gfq_oracle_matmul(q, m, l, n, A, lda, B, ldb, C, ldc, 0)) fail("product", q);
            if (gfq_oracle_matmul(q, m, l, n, A, lda, B, ldb, C1, ldc, 1)) fail("one-thread product", q);
            if (memcmp(C, C1, (size_t)(m * ldc))) fail("threads change the product", q);
            for (int64_t i = 0; i < m; i++)
                for (int64_t j = n; j < ldc; j++)
                    if (C[i * ldc + j] != 0xEE) fail("write beyond the row", q);
            for (int64_t i = 0; i < l; i++) I[i * l + i] = 1;
            if (gfq_oracle_matmul(q, m, l, l, A, lda, I, l, AI, l, 0)) fail("identity product", q);
            for (int64_t i = 0; i < m; i++)
                if (memcmp(AI + i * l, A + i * lda, (size_t)l)) fail("A I != A", q);
            free(A); free(B); free(C); free(C1); free(I); free(AI);
        }
        uint8_t z[4] = {0, 0, 0, 0};
        if (gfq_oracle_matmul(q, 0, 4, 4, NULL, 4, NULL, 4, NULL, 4, 0)) fail("m = 0", q);
        if (gfq_oracle_matmul(q, 2, 0, 2, NULL, 0, NULL, 2, z, 2, 0) || z[0] || z[3]) fail("l = 0", q);
    }
    uint8_t x[16] = {0};
    if (gfq_oracle_matmul(6, 1, 1, 1, x, 1, x, 1, x, 1, 0) != -1) fail("field 6", 0);
    if (gfq_oracle_matmul(3, -1, 1, 1, x, 1, x, 1, x, 1, 0) != -2) fail("m < 0", 0);
    if (gfq_oracle_matmul(3, 2, 2, 2, x, 1, x, 2, x, 2, 0) != -2) fail("lda < l", 0);
    if (gfq_oracle_matmul(3, 2, 2, 2, NULL, 2, x, 2, x, 2, 0) != -3) fail("null A", 0);
    printf("ok all\n");
    return 0;
}
