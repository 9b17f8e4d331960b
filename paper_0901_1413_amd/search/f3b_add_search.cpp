// f3b_add_search.cpp -- exhaustive search behind the F_3 table addition of gfq_field.h
// (f3b_add): the fewest three-input instructions that add two residues modulo 3 held as
// 2-bit binary numbers, 0 and 3 both standing for 0.  The paper searches minimal programs
// of two-input operations for its 2-bit fields (Section 4); gfx950 executes any
// three-input Boolean function in one instruction (v_bitop3_b32), so the gates here are
// all 256 functions of three signals.
//
// Signals are truth tables over the 16 input combinations (a0, a1, b0, b1).  A program is
// a sequence of gates; its outputs are any two signals (r0, r1) such that r0 + 2 r1 is a
// representative of (a + b) mod 3 on every combination.  A shortest program ends in an
// output gate (a gate used by nothing could be dropped), so the search enumerates every
// program of L - 1 gates and solves the last one: for a choice of its three inputs, a
// truth table exists exactly when the values it must take are consistent within each of
// the 8 classes of input-bit patterns.  Gates that repeat an existing signal are skipped,
// as are repeats of a signal already tried at the same depth.
//
// Build and run (host only):  g++ -O2 -std=c++17 f3b_add_search.cpp -o s && ./s
// Prints the count of programs for each length up to 3 (all zero), then checks the
// four-gate program used by the library.
#include <cstdint>
#include <cstdio>
#include <vector>

typedef uint16_t T;
static T must1[2], must0[2], eqm;   // per output: combos forced to 1 / 0; combos with r0 == r1

static T gate(T x, T y, T z, int f) {
    T r = 0;
    for (int c = 0; c < 16; c++) {
        const int v = ((x >> c) & 1) | ((y >> c) & 1) << 1 | ((z >> c) & 1) << 2;
        if ((f >> v) & 1) r |= (T)(1u << c);
    }
    return r;
}
static bool fits(int o, T r) { return (r & must1[o]) == must1[o] && (r & must0[o]) == 0; }

// can one gate over (x, y, z) be output o, given the other output s?
static bool solvable(T x, T y, T z, int o, T s) {
    const T one = must1[o] | (eqm & s), zero = must0[o] | (eqm & (T)~s);
    for (int v = 0; v < 8; v++) {
        const T cls = (T)(((v & 1) ? x : (T)~x) & ((v & 2) ? y : (T)~y) & ((v & 4) ? z : (T)~z));
        if ((cls & one) && (cls & zero)) return false;
    }
    return true;
}

static std::vector<T> sig;
static long found;

static void last_gate() {
    const int n = (int)sig.size();
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            for (int k = j + 1; k < n; k++)
                for (int o = 0; o < 2; o++)
                    for (int s = 0; s < n; s++)
                        if (fits(1 - o, sig[s]) && solvable(sig[i], sig[j], sig[k], o, sig[s])) found++;
}

static void search(int gates_left) {
    if (gates_left == 1) {
        last_gate();
        return;
    }
    const int n = (int)sig.size();
    std::vector<T> tried;
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            for (int k = j + 1; k < n; k++)
                for (int f = 0; f < 256; f++) {
                    const T g = gate(sig[i], sig[j], sig[k], f);
                    bool skip = false;
                    for (T t : sig) skip |= t == g;
                    for (T t : tried) skip |= t == g;
                    if (skip) continue;
                    tried.push_back(g);
                    sig.push_back(g);
                    search(gates_left - 1);
                    sig.pop_back();
                }
}

int main() {
    T in[4];
    for (int i = 0; i < 4; i++) {
        in[i] = 0;
        for (int c = 0; c < 16; c++)
            if ((c >> i) & 1) in[i] |= (T)(1u << c);
    }
    for (int c = 0; c < 16; c++) {
        const int a = (c & 1) + 2 * ((c >> 1) & 1), b = ((c >> 2) & 1) + 2 * ((c >> 3) & 1);
        const int t = (a + b) % 3;
        if (t == 1) { must1[0] |= (T)(1u << c); must0[1] |= (T)(1u << c); }
        else if (t == 2) { must0[0] |= (T)(1u << c); must1[1] |= (T)(1u << c); }
        else eqm |= (T)(1u << c);
    }
    // no program shorter than four: lengths 1 (an output that is an input) to 3
    int ok_inputs = 0;
    for (int o = 0; o < 2; o++)
        for (T x : in) ok_inputs += fits(o, x);
    printf("length 0: %d outputs among the inputs\n", ok_inputs);
    for (int L = 1; L <= 3; L++) {
        sig.assign(in, in + 4);
        found = 0;
        search(L);
        printf("length %d: %ld programs\n", L, found);
        fflush(stdout);
    }
    // the four-gate program of gfq_field.h, gates written as f(x, y, z) with the truth-table
    // bit x + 2y + 4z: h1 = 0x17(a0, a1, b0), h2 = 0x49(a0, a1, b0), r0 = 0x96(a1, b1, h1),
    // r1 = 0x49(b1, h2, r0)
    const T h1 = gate(in[0], in[1], in[2], 0x17), h2 = gate(in[0], in[1], in[2], 0x49);
    const T r0 = gate(in[1], in[3], h1, 0x96), r1 = gate(in[3], h2, r0, 0x49);
    const bool ok = fits(0, r0) && fits(1, r1) && ((r0 ^ r1) & eqm) == 0;
    printf("four-gate program: %s\n", ok ? "correct" : "WRONG");
    return ok ? 0 : 1;
}
