// Lossless suit isomorphism at chance nodes (Sec. 4.5, information
// abstraction: the experiments use lossless abstraction, which changes no
// result).
//
// A suit permutation pi (card 4 r + s -> 4 r + pi(s)) that maps the root
// board onto itself, leaves both root ranges unchanged (r_p(pi h) = r_p(h)
// for every combo h, compared exactly) and maps the tree onto itself (always
// true for a built tree; checked, for trees pruned unevenly) maps the
// subgame onto itself:
// every iterate of CFR is then invariant under pi.  Below a chance node
// whose dealt cards pi also fixes, the child dealt card pi(c) is the image
// of the child dealt c, and its values are v(h | pi c) = v(pi^-1 h | c).
// So only one child per orbit of the chance cards needs solving; the other
// children's subtrees are skipped and the chance node reads their values
// through the hand permutation.  With ranges that have no symmetry the map
// is the identity and nothing changes.
#include <algorithm>
#include <array>
#include <cstring>
#include <new>

#include "host.hpp"

namespace pcfr {

const std::array<std::array<int8_t, 4>, 24>& suit_perms() {
    static const std::array<std::array<int8_t, 4>, 24> tab = [] {
        std::array<std::array<int8_t, 4>, 24> t{};
        std::array<int8_t, 4> p = {0, 1, 2, 3};
        int i = 0;
        do { t[i++] = p; } while (std::next_permutation(p.begin(), p.end()));
        return t;
    }();
    return tab;
}

static inline int map_card(const std::array<int8_t, 4>& pi, int c) { return 4 * (c / 4) + pi[c % 4]; }

int suit_perm_card(int q, int card) { return map_card(suit_perms()[q], card); }

int suit_perm_compose(int q1, int q2) {
    const auto& perms = suit_perms();
    std::array<int8_t, 4> c{};
    for (int s = 0; s < 4; s++) c[s] = perms[q1][perms[q2][s]];
    for (int q = 0; q < 24; q++)
        if (perms[q] == c) return q;
    return 0;   // unreachable: S4 is closed under composition
}

static uint64_t map_mask(const std::array<int8_t, 4>& pi, uint64_t m) {
    uint64_t out = 0;
    for (int c = 0; c < 52; c++)
        if (m >> c & 1ull) out |= 1ull << map_card(pi, c);
    return out;
}

// True when the suit permutation pi maps the tree onto itself: every node and
// its image have the same type, player, action count and contributions,
// actions correspond in order and the chance child dealt c corresponds to the
// one dealt pi(c).  A built tree always is (betting does not depend on the
// cards); a tree pruned unevenly across chance children may not be, and then
// pi is no symmetry of the game.
static bool tree_invariant(const Tree& t, const std::array<int8_t, 4>& pi) {
    if (t.nodes.empty()) return true;
    std::vector<std::pair<int32_t, int32_t>> stack{{0, 0}};
    int card_child[52];
    while (!stack.empty()) {
        const auto [x, y] = stack.back();
        stack.pop_back();
        const Node& a = t.nodes[x];
        const Node& b = t.nodes[y];
        if (a.type != b.type || a.player != b.player || a.n_child != b.n_child || a.contrib[0] != b.contrib[0] ||
            a.contrib[1] != b.contrib[1])
            return false;
        if (a.type == PCFR_NODE_CHANCE) {
            std::fill(card_child, card_child + 52, -1);
            for (int e = 0; e < b.n_child; e++) card_child[t.nodes[b.first_child + e].chance_card] = b.first_child + e;
            for (int e = 0; e < a.n_child; e++) {
                const int ya = a.first_child + e;
                const int yb = card_child[map_card(pi, t.nodes[ya].chance_card)];
                if (yb < 0) return false;
                stack.push_back({ya, yb});
            }
        } else {
            for (int e = 0; e < a.n_child; e++) stack.push_back({a.first_child + e, b.first_child + e});
        }
    }
    return true;
}

int32_t suit_iso_map(const std::vector<const Tree*>& trees, const double* ranges, IsoMap& out) {
    const ComboTable& cc = combos();
    const auto& perms = suit_perms();
    const int32_t K = (int32_t)trees.size();
    int64_t N = 0;
    std::vector<int64_t> base(K);
    for (int32_t g = 0; g < K; g++) { base[g] = N; N += (int64_t)trees[g]->nodes.size(); }
    out.skip.assign(N, 0);
    out.src.assign(N, -1);
    out.perm.assign(N, -1);
    out.mapped.assign(N, 0);
    out.corr.assign(N, -1);
    out.cperm.assign(N, -1);
    out.group.assign(K, 0u);
    for (int32_t g = 0; g < K; g++) {
        const Tree& t = *trees[g];
        const double* r = ranges + (size_t)g * 2 * kCombos;
        // the group: permutations fixing the root board and both ranges
        uint32_t grp = 0;
        for (int q = 0; q < 24; q++) {
            const auto& pi = perms[q];
            if (map_mask(pi, t.root_mask) != t.root_mask) continue;
            bool ok = true;
            for (int k = 0; k < kCombos && ok; k++) {
                const int pk = combo_of(map_card(pi, cc.hi[k]), map_card(pi, cc.lo[k]));
                ok = r[pk] == r[k] && r[kCombos + pk] == r[kCombos + k];
            }
            if (ok && q != 0 && !tree_invariant(t, pi)) ok = false;
            if (ok) grp |= 1u << q;
        }
        out.group[g] = grp;
        // every chance child outside skipped subtrees stands for itself unless mapped below
        for (size_t i = 0; i < t.nodes.size(); i++)
            if (t.nodes[i].type == PCFR_NODE_CHANCE)
                for (int a = 0; a < t.nodes[i].n_child; a++)
                    out.src[base[g] + t.nodes[i].first_child + a] = (int32_t)(base[g] + t.nodes[i].first_child + a);
        if (grp == 1u) continue;   // identity only
        // breadth-first ids: a parent precedes its children, so skipping
        // propagates by one pass over the nodes
        for (size_t i = 0; i < t.nodes.size(); i++) {
            const Node& nd = t.nodes[i];
            const int64_t gi = base[g] + (int64_t)i;
            if (nd.parent >= 0 && out.skip[base[g] + nd.parent]) { out.skip[gi] = 1; continue; }
            if (nd.type != PCFR_NODE_CHANCE || nd.n_child < 1) continue;
            // permutations of the group that also fix the cards dealt above this node
            const uint64_t dealt = nd.board_mask & ~t.root_mask;
            std::vector<int> gn;
            for (int q = 0; q < 24; q++)
                if ((grp >> q & 1u) && map_mask(perms[q], dealt) == dealt) gn.push_back(q);
            if (gn.size() < 2) continue;
            int child_of_card[52];
            std::fill(child_of_card, child_of_card + 52, -1);
            for (int a = 0; a < nd.n_child; a++) child_of_card[t.nodes[nd.first_child + a].chance_card] = a;
            // orbits in card order: the smallest card of an orbit is its representative
            std::vector<char> done(nd.n_child, 0);
            for (int a = 0; a < nd.n_child; a++) {
                const int64_t ca = base[g] + nd.first_child + a;
                if (done[a]) continue;
                done[a] = 1;
                const int rep_card = t.nodes[nd.first_child + a].chance_card;
                for (int q : gn) {
                    const int img = map_card(perms[q], rep_card);
                    const int b = child_of_card[img];
                    if (b < 0) continue;   // cannot happen for a group fixing the board
                    const int64_t cb = base[g] + nd.first_child + b;
                    if (done[b]) continue;
                    // node-by-node correspondence of the two subtrees (actions in
                    // the same order, chance children by permuted card); a
                    // subtree of another shape (a tree pruned unevenly) is not
                    // the image and stays swept on its own
                    std::vector<std::pair<int32_t, int32_t>> pairs, stack{{(int32_t)(ca - base[g]), (int32_t)(cb - base[g])}};
                    bool same = true;
                    while (!stack.empty() && same) {
                        const auto [xa, xb] = stack.back();
                        stack.pop_back();
                        pairs.push_back({xa, xb});
                        const Node& na = t.nodes[xa];
                        const Node& nb = t.nodes[xb];
                        if (na.type != nb.type || na.n_child != nb.n_child || na.player != nb.player ||
                            na.contrib[0] != nb.contrib[0] || na.contrib[1] != nb.contrib[1]) {
                            same = false;
                            break;
                        }
                        if (na.type == PCFR_NODE_CHANCE) {
                            int bychild[52];
                            std::fill(bychild, bychild + 52, -1);
                            for (int e = 0; e < nb.n_child; e++) bychild[t.nodes[nb.first_child + e].chance_card] = nb.first_child + e;
                            for (int e = 0; e < na.n_child && same; e++) {
                                const int ya = na.first_child + e;
                                const int yb = bychild[map_card(perms[q], t.nodes[ya].chance_card)];
                                if (yb < 0) same = false;
                                else stack.push_back({ya, yb});
                            }
                        } else {
                            for (int e = 0; e < na.n_child; e++)
                                stack.push_back({na.first_child + e, nb.first_child + e});
                        }
                    }
                    if (!same) continue;
                    done[b] = 1;
                    out.src[cb] = ca;
                    out.perm[cb] = (int8_t)q;
                    out.skip[cb] = 1;
                    out.mapped[gi] = 1;
                    for (const auto& [xa, xb] : pairs) {
                        out.corr[base[g] + xb] = (int32_t)(base[g] + xa);
                        out.cperm[base[g] + xb] = (int8_t)q;
                    }
                }
            }
        }
    }
    return PCFR_OK;
}

// Hand index of pi^-1(h) for every hand h of a subgame, for each of the 24
// permutations (entries of permutations outside the subgame's group, and of
// padding hands, are the identity).
void suit_hand_maps(const std::vector<int32_t>& hand_combo, const std::vector<int32_t>& combo_hand, uint32_t group,
                    int64_t Hp, int16_t* out /* [24][Hp] */) {
    const ComboTable& cc = combos();
    const auto& perms = suit_perms();
    for (int q = 0; q < 24; q++) {
        int16_t* m = out + (size_t)q * Hp;
        for (int64_t h = 0; h < Hp; h++) m[h] = (int16_t)h;
        if (!(group >> q & 1u)) continue;
        std::array<int8_t, 4> inv{};
        for (int s = 0; s < 4; s++) inv[perms[q][s]] = (int8_t)s;
        for (size_t h = 0; h < hand_combo.size(); h++) {
            const int k = hand_combo[h];
            const int pk = combo_of(map_card(inv, cc.hi[k]), map_card(inv, cc.lo[k]));
            m[h] = (int16_t)combo_hand[pk];
        }
    }
}

}  // namespace pcfr

using namespace pcfr;

extern "C" int32_t pcfr_suit_iso_map(const pcfr_tree* tree, const double* ranges, uint32_t* group, int32_t* src,
                                     int32_t* perm, int8_t* skip) {
    if (!tree || !ranges || !group || !src || !perm || !skip) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    IsoMap m;
    try {
        std::vector<const Tree*> tv{&tree->t};
        int32_t rc = suit_iso_map(tv, ranges, m);
        if (rc) return rc;
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return PCFR_E_OUT_OF_MEMORY;
    }
    *group = m.group[0];
    for (size_t i = 0; i < m.skip.size(); i++) {
        src[i] = m.src[i];
        perm[i] = m.perm[i];
        skip[i] = m.skip[i];
    }
    return PCFR_OK;
}
