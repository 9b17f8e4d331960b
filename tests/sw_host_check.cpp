// Host print of the Strassen-Winograd schedule tables and level shapes (gfq_sw.h), for the
// CPU test that checks them against the definition of the matrix product.
#include <cstdio>
#include "gfq_sw.h"
using namespace gfq;
int main() {
    for (int c = 0; c < 7; c++) {
        printf("A %d", c);
        for (int j = 0; j < 4; j++) printf(" %d", SW_A[c][j]);
        printf("\n");
        printf("B %d", c);
        for (int j = 0; j < 4; j++) printf(" %d", SW_B[c][j]);
        printf("\n");
    }
    for (int j = 0; j < 4; j++) {
        printf("C %d", j);
        for (int c = 0; c < 7; c++) printf(" %d", SW_C[j][c]);
        printf("\n");
    }
    for (long long d = 1; d <= 300; d++) printf("half %lld %lld %lld\n", d, sw_half_rows(d), sw_half_cols(d));
    return 0;
}
