// C ABI: error reporting, tree construction/export, hand evaluation.
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "host.hpp"

namespace pcfr {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace pcfr

using namespace pcfr;

extern "C" {

int32_t pcfr_abi_version(void) { return PCFR_ABI_VERSION; }

const char* pcfr_last_error(void) { return g_err.c_str(); }

int32_t pcfr_build_tree(const pcfr_tree_spec* spec, pcfr_tree** out) {
    if (!spec || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    pcfr_tree* t = new (std::nothrow) pcfr_tree;
    if (!t) { set_error("out of host memory"); return PCFR_E_OUT_OF_MEMORY; }
    int32_t rc;
    try {
        rc = build_tree(*spec, t->t);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory building the tree");
        rc = PCFR_E_OUT_OF_MEMORY;
    }
    if (rc != PCFR_OK) { delete t; return rc; }
    *out = t;
    return PCFR_OK;
}

int32_t pcfr_tree_free(pcfr_tree* tree) {
    delete tree;
    return PCFR_OK;
}

int32_t pcfr_tree_prune(const pcfr_tree* tree, const uint8_t* removed, pcfr_tree** out, int32_t* new_id) {
    if (!tree || !removed || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    pcfr_tree* t = new (std::nothrow) pcfr_tree;
    if (!t) { set_error("out of host memory"); return PCFR_E_OUT_OF_MEMORY; }
    int32_t rc;
    std::vector<int32_t> ids;
    try {
        rc = prune_tree(tree->t, removed, t->t, ids);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory pruning the tree");
        rc = PCFR_E_OUT_OF_MEMORY;
    }
    if (rc != PCFR_OK) { delete t; return rc; }
    if (new_id) std::memcpy(new_id, ids.data(), ids.size() * sizeof(int32_t));
    *out = t;
    return PCFR_OK;
}

int32_t pcfr_tree_info(const pcfr_tree* tree, int64_t* out) {
    if (!tree || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    const Tree& t = tree->t;
    std::memset(out, 0, 16 * sizeof(int64_t));
    out[0] = (int64_t)t.nodes.size();
    for (int k = 0; k < 6; k++) out[1 + k] = t.count[k];
    out[7] = t.n_levels;
    out[8] = t.rows;
    int h = 0;
    const ComboTable& cc = combos();
    for (int k = 0; k < kCombos; k++)
        if (!((t.root_mask >> cc.hi[k] & 1ull) || (t.root_mask >> cc.lo[k] & 1ull))) h++;
    if (t.root_mask == 0) h = 169;   // a preflop root is solved over the hand classes
    out[9] = h;
    out[10] = (h + 63) / 64 * 64;
    return PCFR_OK;
}

int32_t pcfr_tree_export(const pcfr_tree* tree, int32_t* type, int32_t* player, int32_t* parent,
                         int32_t* action, int32_t* depth, int64_t* contrib, int32_t* chance_card,
                         int32_t* first_child, int32_t* n_child) {
    if (!tree || !type || !player || !parent || !action || !depth || !contrib || !chance_card ||
        !first_child || !n_child) {
        set_error("null argument");
        return PCFR_E_INVALID_ARG;
    }
    const Tree& t = tree->t;
    for (size_t i = 0; i < t.nodes.size(); i++) {
        const Node& n = t.nodes[i];
        type[i] = n.type; player[i] = n.player; parent[i] = n.parent; action[i] = n.action;
        depth[i] = n.depth; contrib[2 * i] = n.contrib[0]; contrib[2 * i + 1] = n.contrib[1];
        chance_card[i] = n.chance_card; first_child[i] = n.first_child; n_child[i] = n.n_child;
    }
    return PCFR_OK;
}

int32_t pcfr_equity_table(const pcfr_tree* tree, double* out) {
    if (!tree || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    const Tree& t = tree->t;
    if (__builtin_popcountll(t.root_mask) == 5) { set_error("the root board is complete"); return PCFR_E_INVALID_ARG; }
    const ComboTable& cc = combos();
    std::vector<int32_t> hands;
    for (int k = 0; k < kCombos; k++)
        if (!((t.root_mask >> cc.hi[k] & 1ull) || (t.root_mask >> cc.lo[k] & 1ull))) hands.push_back(k);
    std::vector<double> E;
    try {
        equity_matrix(t.root_mask, hands, E);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return PCFR_E_OUT_OF_MEMORY;
    }
    std::memset(out, 0, sizeof(double) * kCombos * kCombos);
    const size_t H = hands.size();
    for (size_t i = 0; i < H; i++)
        for (size_t j = 0; j < H; j++) out[(size_t)hands[i] * kCombos + hands[j]] = E[i * H + j];
    return PCFR_OK;
}

int32_t pcfr_eval7_batch(const int32_t* cards, int64_t n, int32_t* out) {
    if (!cards || !out || n < 0) { set_error("null argument or negative count"); return PCFR_E_INVALID_ARG; }
    for (int64_t i = 0; i < n; i++) {
        uint64_t m = 0;
        for (int j = 0; j < 7; j++) {
            int c = cards[i * 7 + j];
            if (c < 0 || c >= 52 || (m >> c & 1ull)) { set_error("cards must be 7 distinct ids in [0, 52)"); return PCFR_E_INVALID_ARG; }
            m |= 1ull << c;
        }
        out[i] = (int32_t)eval7_mask(m);
    }
    return PCFR_OK;
}

}  // extern "C"
