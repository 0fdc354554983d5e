// Host-side structures of the library: card helpers, the public tree, and
// the per-board tables the showdown kernel reads.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pcfr.h"

namespace pcfr {

constexpr int kCombos = 1326;
constexpr int kMaxActions = 12;   // fold/check, call, 8 sizes, all-in: 11

inline int combo_of(int a, int b) {
    if (a < b) { int t = a; a = b; b = t; }
    return a * (a - 1) / 2 + b;
}

// card pair of every combo
struct ComboTable {
    uint8_t hi[kCombos], lo[kCombos];
    ComboTable();
};
const ComboTable& combos();

// Seven-card value from a 52-bit card mask (bit c = card c).
uint32_t eval7_mask(uint64_t cards);

// Error reporting (thread-local message).
void set_error(const std::string& msg);

struct Node {
    int32_t type, player, parent, action, depth, chance_card;
    int32_t first_child, n_child;
    int64_t contrib[2];
    uint64_t board_mask;   // all public cards at this node
};

struct Tree {
    pcfr_tree_spec spec;
    std::vector<Node> nodes;
    int32_t n_levels = 0;
    int64_t rows = 0;
    int64_t count[6] = {0, 0, 0, 0, 0, 0};
    uint64_t root_mask = 0;
};

int32_t build_tree(const pcfr_tree_spec& spec, Tree& out);

// Pairwise check-down equity E[h][o] over a hand list on a partial board.
void equity_matrix(uint64_t board, const std::vector<int32_t>& hand_combo, std::vector<double>& E);

}  // namespace pcfr

struct pcfr_tree {
    pcfr::Tree t;
};
