// CPU check of the LDS placement of the NPR path matrices (host build of ppos, sp_npr_layout.h; compiled and run
// by tests/test_npr_layout_cpu.py). A plane holds one element of the 256 corner-pair matrices, one 16-byte word
// per pair; a word at position q of plane j sits at word offset NPR_PLANE j + q, so it occupies the four 4-byte
// banks of slot (NPR_PLANE j + q) mod 16 of a 64-bank LDS row. Checked:
//  1. ppos maps the 256 pairs (X, Y) one to one onto [0, 256);
//  2. the pairs a wavefront reads at once fall in 16 distinct slots: (X, Y) for the 16 X and one Y (the
//     contraction's U_{C,B} reads), (X, Y) for one X and the 16 Y (its U_{A,D} reads), and (X, X xor d) for the
//     16 X and one corner difference d (the recursion's reads of U_{A,A^mu} and U_{A^mu,D}, and its writes);
//  3. one pair's nine elements, in the nine planes, fall in nine distinct slots.
// Prints one line per check and exits non-zero at the first failure.
#include <cstdio>

#include "../paper_1511_00088_amd/csrc/sp_npr_layout.h"

static int distinct16(const int* q) {
    int seen = 0;
    for (int i = 0; i < 16; ++i) seen |= 1 << (q[i] & 15);
    return seen == 0xFFFF;
}

int main() {
    using sp::ppos;
    int hit[256] = {0};
    for (int X = 0; X < 16; ++X)
        for (int Y = 0; Y < 16; ++Y) {
            const int q = ppos(X, Y);
            if (q < 0 || q >= 256 || hit[q]++) {
                std::printf("FAILED: ppos(%d, %d) = %d is out of range or taken twice\n", X, Y, q);
                return 1;
            }
        }
    std::printf("bijection onto [0, 256): ok\n");
    int q[16];
    for (int Y = 0; Y < 16; ++Y) {
        for (int X = 0; X < 16; ++X) q[X] = ppos(X, Y);
        if (!distinct16(q)) { std::printf("FAILED: one Y = %d, all X\n", Y); return 1; }
    }
    for (int X = 0; X < 16; ++X) {
        for (int Y = 0; Y < 16; ++Y) q[Y] = ppos(X, Y);
        if (!distinct16(q)) { std::printf("FAILED: one X = %d, all Y\n", X); return 1; }
    }
    for (int d = 0; d < 16; ++d) {
        for (int X = 0; X < 16; ++X) q[X] = ppos(X, X ^ d);
        if (!distinct16(q)) { std::printf("FAILED: corner difference %d\n", d); return 1; }
    }
    std::printf("distinct slots for one Y, one X and one corner difference: ok\n");
    for (int p = 0; p < 256; ++p) {
        int seen = 0;
        for (int j = 0; j < 9; ++j) seen |= 1 << ((sp::NPR_PLANE * j + ppos(p >> 4, p & 15)) & 15);
        if (__builtin_popcount(seen) != 9) { std::printf("FAILED: planes of pair %d\n", p); return 1; }
    }
    std::printf("nine planes of a pair in distinct slots: ok\nALL OK\n");
    return 0;
}
