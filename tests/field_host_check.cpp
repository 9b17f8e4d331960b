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
        F3v a = f3_add(x, y);
        printf("f3 %u %u %u %u add %u %u\n", x.u, x.s, y.u, y.s, bit(a.u), bit(a.s));
    }
    for (int i = 0; i < 3; i++) { F3v n = f3_neg(f3(codes[i][0], codes[i][1])); printf("f3neg %u %u %u %u\n", codes[i][0], codes[i][1], bit(n.u), bit(n.s)); }
    for (unsigned a = 0; a < 8; a++) for (unsigned b = 0; b < 8; b++)
        printf("p3 %u %u f7add %u f7sub %u\n", a, b, v3(f7_add(p3(a), p3(b))), v3(f7_sub(p3(a), p3(b))));
    for (unsigned a = 0; a < 8; a++)
        printf("p1 %u f7dbl %u f7neg %u f7red %u f5neg %u f5red %u\n", a, v3(f7_dbl(p3(a))), v3(f7_neg(p3(a))) & 7,
               v3(f7_reduce(p3(a))), v3(f5_neg(p3(a))), v3(f5_reduce(p3(a))));
    for (unsigned a = 0; a < 4; a++) for (unsigned b = 0; b < 4; b++) {
        G4v x; x.c0 = a & 1; x.c1 = a >> 1; G4v y; y.c0 = b & 1; y.c1 = b >> 1;
        G4v s = g4_add(x, y), mx = g4_mulx(x);
        printf("g4 %u %u add %u mulx %u\n", a, b, bit(s.c0) | bit(s.c1) << 1, bit(mx.c0) | bit(mx.c1) << 1);
    }
    // GF(8): add, multiply by x and x^2, and the accumulate step c + t + x u + x^2 v
    for (unsigned a = 0; a < 8; a++) for (unsigned b = 0; b < 8; b++) {
        G8v x; x.c0 = a & 1; x.c1 = (a >> 1) & 1; x.c2 = a >> 2;
        G8v y; y.c0 = b & 1; y.c1 = (b >> 1) & 1; y.c2 = b >> 2;
        G8v s = g8_add(x, y), m1 = g8_mulx(x), m2 = g8_mulx2(x);
        printf("g8 %u %u add %u mulx %u mulx2 %u\n", a, b, bit(s.c0) | bit(s.c1) << 1 | bit(s.c2) << 2,
               bit(m1.c0) | bit(m1.c1) << 1 | bit(m1.c2) << 2, bit(m2.c0) | bit(m2.c1) << 1 | bit(m2.c2) << 2);
    }
    for (unsigned c = 0; c < 8; c++) for (unsigned t = 0; t < 8; t++)
        for (unsigned u = 0; u < 8; u++) for (unsigned v = 0; v < 8; v++) {
            u32 cc[3], tt[3], uu[3], vv[3];
            for (int i = 0; i < 3; i++) { cc[i] = (c >> i) & 1; tt[i] = (t >> i) & 1; uu[i] = (u >> i) & 1; vv[i] = (v >> i) & 1; }
            g8_acc(cc, tt, uu, vv);
            printf("g8acc %u %u %u %u %u\n", c, t, u, v, bit(cc[0]) | bit(cc[1]) << 1 | bit(cc[2]) << 2);
        }
    // binary mod 3 working form
    for (unsigned a = 0; a < 4; a++) for (unsigned b = 0; b < 4; b++) {
        u32 x[2] = {a & 1, a >> 1}, y[2] = {b & 1, b >> 1}, r[2], d[2];
        f3b_add(x, y, r); f3b_sub(x, y, d);
        u32 c0, c1; f3_from_bin(x, &c0, &c1);
        printf("f3b %u %u add %u sub %u tocode %u %u\n", a, b, bit(r[0]) | bit(r[1]) << 1, bit(d[0]) | bit(d[1]) << 1, bit(c0), bit(c1));
    }
    for (int i = 0; i < 3; i++) { u32 b[2]; f3_to_bin(codes[i][0], codes[i][1], b); printf("f3tobin %u %u %u\n", codes[i][0], codes[i][1], bit(b[0]) | bit(b[1]) << 1); }
    // carry-save steps: every (S, K, X) for NB = 2, 3, 4
    for (unsigned S = 0; S < 16; S++) for (unsigned K = 0; K < 16; K++) for (unsigned X = 0; X < 16; X++) {
        u32 s4[4], k4[4], x4[4];
        for (int i = 0; i < 4; i++) { s4[i] = (S >> i) & 1; k4[i] = (K >> i) & 1; x4[i] = (X >> i) & 1; }
        u32 s3[3] = {s4[0], s4[1], s4[2]}, k3[3] = {k4[0], k4[1], k4[2]}, x3[3] = {x4[0], x4[1], x4[2]};
        u32 s2[2] = {s4[0], s4[1]}, k2[2] = {k4[0], k4[1]}, x2[2] = {x4[0], x4[1]};
        u32 n2s[2] = {s2[0], s2[1]}, n2k[2] = {k2[0], k2[1]};
        csa_step<4>(s4, k4, x4); csa_step<3>(s3, k3, x3); csa_step<2>(s2, k2, x2);
        csa_step_neg<2>(n2s, n2k, x2);
        unsigned v4s = 0, v4k = 0, v3s = 0, v3k = 0, v2s = 0, v2k = 0;
        for (int i = 0; i < 4; i++) { v4s |= bit(s4[i]) << i; v4k |= bit(k4[i]) << i; }
        for (int i = 0; i < 3; i++) { v3s |= bit(s3[i]) << i; v3k |= bit(k3[i]) << i; }
        for (int i = 0; i < 2; i++) { v2s |= bit(s2[i]) << i; v2k |= bit(k2[i]) << i; }
        unsigned vns = bit(n2s[0]) | bit(n2s[1]) << 1, vnk = bit(n2k[0]) | bit(n2k[1]) << 1;
        printf("csa %u %u %u  %u %u  %u %u  %u %u  %u %u\n", S, K, X, v4s, v4k, v3s, v3k, v2s, v2k, vns, vnk);
    }
    // F_3 slab step as the product kernel takes it: acc + t, then - v (binary residues mod 3)
    for (unsigned a = 0; a < 4; a++)
        for (unsigned t = 0; t < 4; t++) for (unsigned v = 0; v < 4; v++) {
            u32 c[2] = {a & 1, a >> 1}, t2[2] = {t & 1, t >> 1}, v2[2] = {v & 1, v >> 1}, x[2], r[2];
            f3b_add(c, t2, x);
            f3b_sub(x, v2, r);
            printf("f3acc %u %u %u %u\n", a, t, v, bit(r[0]) | bit(r[1]) << 1);
        }
    // F_5 eight-instruction addition and subtraction on every pair of 3-bit representatives
    for (unsigned a = 0; a < 8; a++) for (unsigned b = 0; b < 8; b++) {
        u32 x[3], y[3], r[3], d[3];
        for (int i = 0; i < 3; i++) { x[i] = (a >> i) & 1; y[i] = (b >> i) & 1; }
        f5_add8(x, y, r); f5_sub8(x, y, d);
        printf("f5add8 %u %u %u %u\n", a, b, bit(r[0]) | bit(r[1]) << 1 | bit(r[2]) << 2,
               bit(d[0]) | bit(d[1]) << 1 | bit(d[2]) << 2);
    }
    // F_5 slab step of the three-plane carry-save accumulator modulo 5: every (a, b, c, t, v, w)
    for (unsigned st = 0; st < 8; st++)
        for (unsigned t = 0; t < 8; t++) for (unsigned v = 0; v < 8; v++) for (unsigned w = 0; w < 8; w++) {
            u32 s3[3], t3[3], v3[3], w3[3];
            for (int i = 0; i < 3; i++) { s3[i] = (st >> i) & 1; t3[i] = (t >> i) & 1; v3[i] = (v >> i) & 1; w3[i] = (w >> i) & 1; }
            f5_nc_slab(s3, t3, v3, w3);
            printf("f5slab %u %u %u %u %u %u %u %u\n", st & 1, (st >> 1) & 1, st >> 2, t, v, w,
                   bit(s3[0]) | bit(s3[1]) << 1 | bit(s3[2]) << 2, 0u);
        }
    for (int slabs = 0; slabs < 40; slabs++) {
        u32 s3[3];
        f5_nc_init(s3, slabs);
        bool full = true;
        for (int i = 0; i < 3; i++) full = full && (s3[i] == 0u || s3[i] == 0xffffffffu);
        printf("f5init %d %u %u %u %d\n", slabs, bit(s3[0]), bit(s3[1]), bit(s3[2]), full ? 1 : 0);
    }
    for (unsigned st = 0; st < 8; st++) {
        u32 s3[3] = {st & 1, (st >> 1) & 1, st >> 2};
        printf("f5val %u %u\n", st, v3(f5_nc_value(s3)));
    }
    return 0;
}
