// Seven-card hand values from card bitmasks.
//
// Value layout: category << 20 | r1 << 16 | r2 << 12 | r3 << 8 | r4 << 4 | r5
// with category 0 high card, 1 pair, 2 two pair, 3 trips, 4 straight,
// 5 flush, 6 full house, 7 quads, 8 straight flush, and r1..r5 the ranks
// (0..12 = 2..A) that break ties, most significant first, unused ones 0.  A
// wheel straight has high rank 3.
//
// The evaluation works on per-suit 13-bit rank masks and rank multiplicities
// directly, without enumerating five-card subsets.
#include <cstring>

#include "host.hpp"

namespace pcfr {

ComboTable::ComboTable() {
    for (int a = 1; a < 52; a++)
        for (int b = 0; b < a; b++) {
            int k = combo_of(a, b);
            hi[k] = (uint8_t)a;
            lo[k] = (uint8_t)b;
        }
}

const ComboTable& combos() {
    static ComboTable t;
    return t;
}

namespace {

// High rank of the best straight in a 13-bit rank mask, or -1.
int straight_high(uint32_t m) {
    uint32_t w = (m << 1) | ((m >> 12) & 1u);   // bit k = rank k-1, bit 0 = ace low
    uint32_t run = w & (w >> 1) & (w >> 2) & (w >> 3) & (w >> 4);
    if (!run) return -1;
    return 31 - __builtin_clz(run) + 3;
}

// The n highest set ranks of mask m, written into out[0..n).
int top_ranks(uint32_t m, int n, int* out) {
    int k = 0;
    for (int r = 12; r >= 0 && k < n; r--)
        if (m >> r & 1u) out[k++] = r;
    return k;
}

uint32_t pack(int cat, const int* r, int n) {
    uint32_t v = (uint32_t)cat << 20;
    for (int i = 0; i < n; i++) v |= (uint32_t)r[i] << (16 - 4 * i);
    return v;
}

}  // namespace

uint32_t eval7_mask(uint64_t cards) {
    uint32_t suit[4] = {0, 0, 0, 0};
    for (int c = 0; c < 52; c++)
        if (cards >> c & 1ull) suit[c & 3] |= 1u << (c >> 2);
    uint32_t any = suit[0] | suit[1] | suit[2] | suit[3];
    // ranks held at least 2, 3, 4 times
    uint32_t two = (suit[0] & suit[1]) | (suit[0] & suit[2]) | (suit[0] & suit[3]) |
                   (suit[1] & suit[2]) | (suit[1] & suit[3]) | (suit[2] & suit[3]);
    uint32_t three = (suit[0] & suit[1] & suit[2]) | (suit[0] & suit[1] & suit[3]) |
                     (suit[0] & suit[2] & suit[3]) | (suit[1] & suit[2] & suit[3]);
    uint32_t four = suit[0] & suit[1] & suit[2] & suit[3];
    int r[5];

    int fs = -1;
    for (int s = 0; s < 4; s++)
        if (__builtin_popcount(suit[s]) >= 5) fs = s;
    if (fs >= 0) {
        int sh = straight_high(suit[fs]);
        if (sh >= 0) { r[0] = sh; return pack(8, r, 1); }
    }
    if (four) {
        int q = 31 - __builtin_clz(four);
        r[0] = q;
        top_ranks(any & ~(1u << q), 1, r + 1);
        return pack(7, r, 2);
    }
    if (three) {
        int t = 31 - __builtin_clz(three);
        uint32_t pairs = two & ~(1u << t);
        if (pairs) {
            r[0] = t;
            r[1] = 31 - __builtin_clz(pairs);
            return pack(6, r, 2);
        }
    }
    if (fs >= 0) {
        top_ranks(suit[fs], 5, r);
        return pack(5, r, 5);
    }
    int sh = straight_high(any);
    if (sh >= 0) { r[0] = sh; return pack(4, r, 1); }
    if (three) {
        int t = 31 - __builtin_clz(three);
        r[0] = t;
        top_ranks(any & ~(1u << t), 2, r + 1);
        return pack(3, r, 3);
    }
    if (two) {
        int p1 = 31 - __builtin_clz(two);
        uint32_t rest = two & ~(1u << p1);
        if (rest) {
            int p2 = 31 - __builtin_clz(rest);
            r[0] = p1; r[1] = p2;
            top_ranks(any & ~(1u << p1) & ~(1u << p2), 1, r + 2);
            return pack(2, r, 3);
        }
        r[0] = p1;
        top_ranks(any & ~(1u << p1), 3, r + 1);
        return pack(1, r, 4);
    }
    top_ranks(any, 5, r);
    return pack(0, r, 5);
}

}  // namespace pcfr
