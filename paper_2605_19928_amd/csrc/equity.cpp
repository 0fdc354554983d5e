// Pairwise check-down equity of two hands on a partial board: the mean, over
// every way to complete the board to five cards with cards neither hand
// holds, of sign(value(h) - value(o)).  This is the exact per-unit value of a
// depth-limit leaf where a player is all in (both just see the rest of the
// board), and the exact "stub" leaf model used when no network is attached.
//
// Per completion the hand values are computed once; the pair loop then only
// compares integers.  Rows are split over host threads.
#include <algorithm>
#include <thread>
#include <vector>

#include "host.hpp"

namespace pcfr {

void equity_matrix(uint64_t board, const std::vector<int32_t>& hand_combo, std::vector<double>& E) {
    const ComboTable& cc = combos();
    const int H = (int)hand_combo.size();
    const int nb = __builtin_popcountll(board);
    const int need = 5 - nb;
    std::vector<int> rest;
    for (int c = 0; c < 52; c++)
        if (!(board >> c & 1ull)) rest.push_back(c);
    std::vector<uint64_t> run;
    if (need == 0) run.push_back(0);
    else if (need == 1) for (int x : rest) run.push_back(1ull << x);
    else
        for (size_t i = 0; i < rest.size(); i++)
            for (size_t j = i + 1; j < rest.size(); j++) run.push_back((1ull << rest[i]) | (1ull << rest[j]));
    const int R = (int)run.size();
    std::vector<uint64_t> hm(H);
    for (int h = 0; h < H; h++) hm[h] = (1ull << cc.hi[hand_combo[h]]) | (1ull << cc.lo[hand_combo[h]]);
    std::vector<int32_t> rk((size_t)R * H);
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto par = [&](int n, auto fn) {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; t++)
            th.emplace_back([&, t] {
                for (int i = (int)t; i < n; i += (int)nt) fn(i);
            });
        for (auto& x : th) x.join();
    };
    par(R, [&](int r) {
        for (int h = 0; h < H; h++)
            rk[(size_t)r * H + h] = (hm[h] & run[r]) ? -1 : (int32_t)eval7_mask(hm[h] | board | run[r]);
    });
    // completions avoiding two disjoint hands: C(52 - nb - 4, need)
    const int left = 52 - nb - 4;
    const double cnt = need == 0 ? 1.0 : (need == 1 ? left : left * (left - 1) / 2.0);
    E.assign((size_t)H * H, 0.0);
    par(H, [&](int h) {
        std::vector<int> sum(H, 0);
        for (int r = 0; r < R; r++) {
            const int32_t a = rk[(size_t)r * H + h];
            if (a < 0) continue;
            const int32_t* row = &rk[(size_t)r * H];
            for (int o = 0; o < H; o++) {
                const int32_t b = row[o];
                if (b < 0) continue;
                sum[o] += (a > b) - (a < b);
            }
        }
        for (int o = 0; o < H; o++)
            if (!(hm[h] & hm[o])) E[(size_t)h * H + o] = sum[o] / cnt;
    });
}

}  // namespace pcfr
