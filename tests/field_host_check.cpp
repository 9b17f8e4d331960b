// Host build of the library's bitsliced field formulas: prints every formula's output on
// every input representative, one line per case, for the truth-table test to check.
#include <cstdio>
#include "gfq_field.h"
using namespace gfq;
static unsigned bit(u32 w) { return w & 1u; }
static P3v p3(unsigned v) { P3v a; a.b0 = v & 1; a.b1 = (v >> 1) & 1; a.b2 = (v >> 2) & 1; return a; }
static unsigned v3(P3v a) { return bit(a.b0) | bit(a.b1) << 1 | bit(a.b2) << 2; }
static F3v f3(unsigned u, unsigned s) { F3v a; a.u = u; a.s = s; return a; }
int main() {
    // F_3 on the three valid codes (u, s): (0,0) (1,0) (1,1)
    const unsigned codes[3][2] = {{0, 0}, {1, 0}, {1, 1}};
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) {
        F3v x = f3(codes[i][0], codes[i][1]), y = f3(codes[j][0], codes[j][1]);
        F3v a = f3_add(x, y), s = f3_sub(x, y);
        printf("f3 %u %u %u %u add %u %u sub %u %u\n", x.u, x.s, y.u, y.s, bit(a.u), bit(a.s), bit(s.u), bit(s.s));
    }
    for (int i = 0; i < 3; i++) { F3v n = f3_neg(f3(codes[i][0], codes[i][1])); printf("f3neg %u %u %u %u\n", codes[i][0], codes[i][1], bit(n.u), bit(n.s)); }
    for (unsigned a = 0; a < 8; a++) for (unsigned b = 0; b < 8; b++)
        printf("p3 %u %u f7add %u f5add %u\n", a, b, v3(f7_add(p3(a), p3(b))), v3(f5_add(p3(a), p3(b))));
    for (unsigned a = 0; a < 8; a++)
        printf("p1 %u f7dbl %u f7neg %u f7red %u f5dbl %u f5neg %u f5red %u\n", a, v3(f7_dbl(p3(a))), v3(f7_neg(p3(a))) & 7,
               v3(f7_reduce(p3(a))), v3(f5_dbl(p3(a))), v3(f5_neg(p3(a))), v3(f5_reduce(p3(a))));
    for (unsigned s = 0; s < 16; s++)
        printf("fold5 %u %u\n", s, v3(fold5(s & 1, (s >> 1) & 1, (s >> 2) & 1, (s >> 3) & 1)));
    for (unsigned a = 0; a < 4; a++) for (unsigned b = 0; b < 4; b++) {
        G4v x; x.c0 = a & 1; x.c1 = a >> 1; G4v y; y.c0 = b & 1; y.c1 = b >> 1;
        G4v s = g4_add(x, y), mx = g4_mulx(x);
        printf("g4 %u %u add %u mulx %u\n", a, b, bit(s.c0) | bit(s.c1) << 1, bit(mx.c0) | bit(mx.c1) << 1);
    }
    return 0;
}
