/*
 * gfq_oracle.c -- CPU oracle for dense matrix products over F_3, F_5, F_7, GF(4), GF(8)
 * and F_9.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that tests, the smoke check and the
 * CPU-baseline leg of the benchmark can check the GPU library against an obviously
 * correct product.  No product code may include, link or call it, and it shares no
 * code, header, table or helper with the GPU library.
 *
 * What it computes (paper, Section 2, the equation writing row i of C as the sum over j
 * of a_ij times row j of B): C = A B with A of size m x l and B of size l x n, every
 * element an unsigned byte holding the canonical representative of a field element.
 *
 *   - F_p, p in {3, 5, 7}: element e in [0, p) stands for e mod p.  C[i][j] is
 *     (sum over t of A[i][t] * B[t][j]) mod p, summed exactly in 32-bit integers and
 *     reduced once at the end.  The largest sum is l (p-1)^2, below 2^31 for every l
 *     this library accepts (l < 2^24).
 *   - GF(4) = F_2[x]/(x^2 + x + 1) (paper, Section 4.3, the Karatsuba identity modulo
 *     x^2 + x + 1): element e = c0 + 2 c1 stands for c0 + c1 x.  Addition is XOR of the
 *     coefficient bits; the product of (a0 + a1 x)(b0 + b1 x) is
 *     a0 b0 + (a0 b1 + a1 b0) x + a1 b1 x^2 with x^2 replaced by x + 1.
 *   - GF(8) = F_2[x]/(x^3 + x + 1) (paper, Section 4.3, extension fields viewed as
 *     polynomials over the base field, reduced by the defining polynomial): element
 *     e = c0 + 2 c1 + 4 c2 stands for c0 + c1 x + c2 x^2.  The product is the schoolbook
 *     polynomial product over F_2 (degree up to 4), then x^4 -> x^2 + x and x^3 -> x + 1.
 *   - F_9 = F_3[i]/(i^2 + 1) (paper, Section 4.3, the same polynomial view over F_3; i^2 + 1
 *     has no root mod 3): element e = a0 + 3 a1 with a0, a1 in [0, 3) stands for a0 + a1 i.
 *     (a0 + a1 i)(b0 + b1 i) = (a0 b0 - a1 b1) + (a0 b1 + a1 b0) i; the real and imaginary
 *     sums are taken exactly in 32-bit integers (|sum| <= 2 l (p-1)^2) and reduced mod 3
 *     at the end.
 *
 * Loop order is i, t, j with no blocking: a row of C is built as a linear combination of
 * the rows of B, exactly as the equation reads.  OpenMP splits the rows of C.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Return codes: 0 ok, -1 bad field, -2 bad dimension, -3 null pointer, -4 no memory. */

static uint8_t gf4_mul(uint8_t a, uint8_t b)
{
    /* (a0 + a1 x)(b0 + b1 x) = a0b0 + (a0b1 + a1b0) x + a1b1 x^2,  x^2 = x + 1 over F_2 */
    unsigned a0 = a & 1u, a1 = (a >> 1) & 1u, b0 = b & 1u, b1 = (b >> 1) & 1u;
    unsigned x2 = a1 & b1;                    /* coefficient of x^2 */
    unsigned c0 = (a0 & b0) ^ x2;             /* x^2 contributes 1 ... */
    unsigned c1 = (a0 & b1) ^ (a1 & b0) ^ x2; /* ... and x */
    return (uint8_t)(c0 | (c1 << 1));
}

static uint8_t gf8_mul(uint8_t a, uint8_t b)
{
    /* schoolbook product over F_2: coefficient k collects a_i b_j with i + j = k */
    unsigned p[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) p[i + j] ^= ((a >> i) & 1u) & ((b >> j) & 1u);
    /* reduce by x^3 + x + 1, highest degree first: x^4 = x^2 + x, x^3 = x + 1 */
    p[2] ^= p[4]; p[1] ^= p[4];
    p[1] ^= p[3]; p[0] ^= p[3];
    return (uint8_t)(p[0] | (p[1] << 1) | (p[2] << 2));
}

int gfq_oracle_matmul(int q, int64_t m, int64_t l, int64_t n,
                      const uint8_t *A, int64_t lda,
                      const uint8_t *B, int64_t ldb,
                      uint8_t *C, int64_t ldc, int nthreads)
{
    if (q != 3 && q != 4 && q != 5 && q != 7 && q != 8 && q != 9) return -1;
    if (m < 0 || l < 0 || n < 0 || l >= (1 << 24)) return -2;
    if (m == 0 || n == 0) return 0;
    if (C == NULL || (l > 0 && (A == NULL || B == NULL))) return -3;
    if (lda < l || ldb < n || ldc < n) return -2;
    /* a thread count for this call only (the process default is never changed) */
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
        int32_t *acc = (int32_t *)malloc((size_t)n * 2 * sizeof(int32_t));
        if (acc == NULL) {
#pragma omp atomic write
            err = -4;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; i++) {
            if (acc == NULL) continue;
            memset(acc, 0, (size_t)n * 2 * sizeof(int32_t));
            const uint8_t *arow = A + i * lda;
            if (q == 9) {
                int32_t *re = acc, *im = acc + n;
                for (int64_t t = 0; t < l; t++) {
                    int32_t a0 = arow[t] % 3, a1 = arow[t] / 3;
                    if (a0 == 0 && a1 == 0) continue;
                    const uint8_t *brow = B + t * ldb;
                    for (int64_t j = 0; j < n; j++) {
                        int32_t b0 = brow[j] % 3, b1 = brow[j] / 3;
                        re[j] += a0 * b0 - a1 * b1;
                        im[j] += a0 * b1 + a1 * b0;
                    }
                }
                for (int64_t j = 0; j < n; j++) {
                    int32_t r = ((re[j] % 3) + 3) % 3, m = ((im[j] % 3) + 3) % 3;
                    C[i * ldc + j] = (uint8_t)(r + 3 * m);
                }
            } else if (q == 4 || q == 8) {
                /* the two fields in loops of their own, so that each calls its
                 * multiplication directly */
                for (int64_t t = 0; t < l; t++) {
                    uint8_t a = arow[t];
                    if (a == 0) continue;
                    const uint8_t *brow = B + t * ldb;
                    if (q == 4)
                        for (int64_t j = 0; j < n; j++) acc[j] ^= gf4_mul(a, brow[j]);
                    else
                        for (int64_t j = 0; j < n; j++) acc[j] ^= gf8_mul(a, brow[j]);
                }
                for (int64_t j = 0; j < n; j++) C[i * ldc + j] = (uint8_t)acc[j];
            } else {
                for (int64_t t = 0; t < l; t++) {
                    int32_t a = arow[t];
                    if (a == 0) continue;
                    const uint8_t *brow = B + t * ldb;
                    for (int64_t j = 0; j < n; j++) acc[j] += a * (int32_t)brow[j];
                }
                for (int64_t j = 0; j < n; j++) C[i * ldc + j] = (uint8_t)(acc[j] % q);
            }
        }
        free(acc);
    }
    return err;
}

int gfq_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
