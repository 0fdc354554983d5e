// Host-side structures of the library: card helpers, the public tree, and
// the per-board tables the showdown kernel reads.
#pragma once
#include <array>
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
int32_t prune_tree(const Tree& in, const uint8_t* removed, Tree& out, std::vector<int32_t>& new_id);

// Lossless suit isomorphism at chance nodes (iso.cpp).  Node ids are those
// of the forest: subgame g's nodes follow the nodes of subgames 0 .. g-1.
struct IsoMap {
    std::vector<char> skip;       // per node: inside a subtree solved through its representative
    std::vector<int32_t> src;     // per chance child: the child whose values stand for it (itself for a
                                  // representative), -1 for other nodes
    std::vector<int8_t> perm;     // per chance child: index of the permutation taking the representative's
                                  // card to its own, -1 for representatives and other nodes
    std::vector<char> mapped;     // per chance node: some child is read through a permutation
    std::vector<int32_t> corr;    // per skipped node: the node it is the image of (one level up the chain
                                  // of representatives), else -1
    std::vector<int8_t> cperm;    // per skipped node: the permutation carrying corr's subtree onto its own
    std::vector<uint32_t> group;  // per subgame: bit q set when permutation q maps board and ranges onto themselves
};
const std::array<std::array<int8_t, 4>, 24>& suit_perms();
int suit_perm_compose(int q1, int q2);   // index of pi_q1 o pi_q2 (pi_q2 applied first)
int suit_perm_card(int q, int card);     // pi_q(card)
int32_t suit_iso_map(const std::vector<const Tree*>& trees, const double* ranges, IsoMap& out);
void suit_hand_maps(const std::vector<int32_t>& hand_combo, const std::vector<int32_t>& combo_hand, uint32_t group,
                    int64_t Hp, int16_t* out);

// Pairwise check-down equity E[h][o] over a hand list on a partial board.
void equity_matrix(uint64_t board, const std::vector<int32_t>& hand_combo, std::vector<double>& E);

}  // namespace pcfr

struct pcfr_tree {
    pcfr::Tree t;
};
