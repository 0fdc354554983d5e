// Public-tree construction for a hold'em subgame, breadth first.
//
// Betting rules (the paper fixes an action abstraction but not its rules;
// Sec. 5 "Game"): player 0 acts first on every street; facing a bet the
// actions are fold, call, then raises, otherwise check, then bets; a sized
// bet of pct% puts in the amount to call plus pct% of the pot after calling,
// rounded half up in whole chips, capped at the effective stack; all-in is
// one more action when enabled; duplicate targets and targets that do not
// exceed a call are dropped; bets+raises per street are capped, the opening
// bet included, and need chips behind.  A betting round ends on check-check
// or a call: at the river in a showdown, with a player all in in a chance
// runout to showdown (or an exact all-in leaf under a depth limit), under a
// depth limit in a leaf, else in a chance node dealing the next card.  A
// preflop root (no board) is built depth-limited only, with its leaves at
// the flop deal, and only when no betting line puts a player all in.
//
// Nodes are numbered in the order a FIFO queue pops them, so ids are
// breadth-first and the children of a node are consecutive.
#include <algorithm>
#include <deque>

#include "host.hpp"

namespace pcfr {

namespace {

struct Pending {
    int32_t type;            // node type decided when the node was created
    int32_t player;          // actor (decision) / folder (fold)
    int32_t parent, action, depth, chance_card;
    int64_t c[2];
    int32_t raises;          // bets+raises so far this street (decision nodes)
    uint64_t board;
    int32_t nb;
};

struct Builder {
    const pcfr_tree_spec& sp;
    int64_t cap;
    std::deque<Pending> q;
    Tree& t;

    Builder(const pcfr_tree_spec& s, Tree& out) : sp(s), t(out) {
        int64_t eff = sp.stack[0] < sp.stack[1] ? sp.stack[0] : sp.stack[1];
        cap = sp.pot / 2 + eff;
    }

    // Node that closes a betting round with contributions c.
    Pending round_over(const Pending& from, const int64_t c[2], int parent, int action,
                       int chance_card, uint64_t board, int nb) const {
        Pending p{};
        p.parent = parent; p.action = action; p.depth = from.depth + 1;
        p.chance_card = chance_card; p.c[0] = c[0]; p.c[1] = c[1];
        p.board = board; p.nb = nb; p.player = -1; p.raises = 0;
        bool allin = c[0] >= cap || c[1] >= cap;
        if (nb == 5) p.type = PCFR_NODE_SHOWDOWN;
        else if (sp.depth_limit) p.type = allin ? PCFR_NODE_ALLIN_LEAF : PCFR_NODE_LEAF;
        else p.type = PCFR_NODE_CHANCE;
        return p;
    }

    Pending decision(int player, const int64_t c[2], int raises, int parent, int action, int depth,
                     int chance_card, uint64_t board, int nb) const {
        Pending p{};
        p.type = PCFR_NODE_DECISION; p.player = player; p.parent = parent; p.action = action;
        p.depth = depth; p.chance_card = chance_card; p.c[0] = c[0]; p.c[1] = c[1];
        p.raises = raises; p.board = board; p.nb = nb;
        return p;
    }

    void expand(const Pending& n, int id, std::vector<Pending>& kids) {
        kids.clear();
        if (n.type == PCFR_NODE_DECISION) {
            int p = n.player, o = 1 - p;
            int64_t to_call = n.c[o] - n.c[p];
            int a = 0;
            if (to_call > 0) {
                Pending f{};
                f.type = PCFR_NODE_FOLD; f.player = p; f.parent = id; f.action = a++;
                f.depth = n.depth + 1; f.chance_card = -1; f.c[0] = n.c[0]; f.c[1] = n.c[1];
                f.board = n.board; f.nb = n.nb;
                kids.push_back(f);
                int64_t cc[2] = {n.c[0], n.c[1]};
                cc[p] = n.c[o];
                kids.push_back(round_over(n, cc, id, a++, -1, n.board, n.nb));
            } else if (p == 1) {
                kids.push_back(round_over(n, n.c, id, a++, -1, n.board, n.nb));
            } else {
                kids.push_back(decision(1, n.c, n.raises, id, a++, n.depth + 1, -1, n.board, n.nb));
            }
            if (n.raises < sp.max_raises && n.c[o] < cap) {
                std::vector<int64_t> tgt;
                int64_t after = n.c[0] + n.c[1] + to_call;
                for (int k = 0; k < sp.n_sizes; k++) {
                    int64_t put = to_call + (sp.size_pct[k] * after + 50) / 100;
                    tgt.push_back(std::min(n.c[p] + put, cap));
                }
                if (sp.allin) tgt.push_back(cap);
                std::sort(tgt.begin(), tgt.end());
                tgt.erase(std::unique(tgt.begin(), tgt.end()), tgt.end());
                for (int64_t x : tgt) {
                    if (x <= n.c[o]) continue;
                    int64_t cc[2] = {n.c[0], n.c[1]};
                    cc[p] = x;
                    kids.push_back(decision(o, cc, n.raises + 1, id, a++, n.depth + 1, -1, n.board, n.nb));
                }
            }
        } else if (n.type == PCFR_NODE_CHANCE) {
            bool allin = n.c[0] >= cap || n.c[1] >= cap;
            int a = 0;
            for (int card = 0; card < 52; card++) {
                if (n.board >> card & 1ull) continue;
                uint64_t nbm = n.board | (1ull << card);
                if (allin) kids.push_back(round_over(n, n.c, id, a++, card, nbm, n.nb + 1));
                else kids.push_back(decision(0, n.c, 0, id, a++, n.depth + 1, card, nbm, n.nb + 1));
            }
        }
    }
};

}  // namespace

int32_t build_tree(const pcfr_tree_spec& sp, Tree& t) {
    if ((sp.n_board != 0 && sp.n_board < 3) || sp.n_board > 5) { set_error("n_board must be 0, 3, 4 or 5"); return PCFR_E_INVALID_ARG; }
    if (sp.n_board == 0 && sp.depth_limit != 1) {
        set_error("a preflop root (n_board = 0) needs depth_limit = 1: its leaves sit at the flop deal");
        return PCFR_E_UNSUPPORTED;
    }
    if (sp.pot <= 0 || (sp.pot & 1)) { set_error("pot must be positive and even"); return PCFR_E_INVALID_ARG; }
    if (sp.stack[0] < 0 || sp.stack[1] < 0) { set_error("stacks must be >= 0"); return PCFR_E_INVALID_ARG; }
    if (sp.n_sizes < 0 || sp.n_sizes > 8) { set_error("n_sizes must be in [0, 8]"); return PCFR_E_INVALID_ARG; }
    if (sp.max_raises < 0) { set_error("max_raises must be >= 0"); return PCFR_E_INVALID_ARG; }
    if (sp.depth_limit != 0 && sp.depth_limit != 1) { set_error("depth_limit must be 0 or 1"); return PCFR_E_INVALID_ARG; }
    for (int k = 0; k < sp.n_sizes; k++) {
        if (sp.size_pct[k] <= 0 || sp.size_pct[k] > 100000) { set_error("bet sizes must be in (0, 100000] percent"); return PCFR_E_INVALID_ARG; }
        if (k && sp.size_pct[k] <= sp.size_pct[k - 1]) { set_error("bet sizes must ascend"); return PCFR_E_INVALID_ARG; }
    }
    uint64_t board = 0;
    for (int i = 0; i < sp.n_board; i++) {
        int c = sp.board[i];
        if (c < 0 || c >= 52 || (board >> c & 1ull)) { set_error("board cards must be distinct and in [0, 52)"); return PCFR_E_INVALID_ARG; }
        board |= 1ull << c;
    }
    t = Tree{};
    t.spec = sp;
    t.root_mask = board;
    Builder b(sp, t);
    int64_t c0[2] = {sp.pot / 2, sp.pot / 2};
    b.q.push_back(b.decision(0, c0, 0, -1, -1, 0, -1, board, sp.n_board));
    std::vector<Pending> kids;
    const size_t kMaxNodes = 1u << 26;
    while (!b.q.empty()) {
        Pending n = b.q.front();
        b.q.pop_front();
        int id = (int)t.nodes.size();
        if (t.nodes.size() >= kMaxNodes) { set_error("tree exceeds 2^26 nodes"); return PCFR_E_TOO_LARGE; }
        b.expand(n, id, kids);
        Node nd{};
        nd.type = n.type; nd.player = n.player; nd.parent = n.parent; nd.action = n.action;
        nd.depth = n.depth; nd.chance_card = n.chance_card;
        nd.contrib[0] = n.c[0]; nd.contrib[1] = n.c[1];
        nd.board_mask = n.board;
        nd.n_child = (int32_t)kids.size();
        // children are appended behind everything already queued: their ids
        // are this node's id + queue length + 1 onwards
        nd.first_child = kids.empty() ? -1 : (int32_t)(id + b.q.size() + 1);
        if (nd.n_child > kMaxActions && n.type == PCFR_NODE_DECISION) { set_error("too many actions"); return PCFR_E_TOO_LARGE; }
        for (auto& k : kids) b.q.push_back(k);
        t.nodes.push_back(nd);
        t.count[n.type]++;
        if (n.type == PCFR_NODE_DECISION) t.rows += nd.n_child;
        if (n.depth + 1 > t.n_levels) t.n_levels = n.depth + 1;
    }
    if (sp.n_board == 0 && t.count[PCFR_NODE_ALLIN_LEAF] > 0) {
        set_error("a preflop tree whose betting can put a player all in is not supported (the runout has five cards)");
        return PCFR_E_UNSUPPORTED;
    }
    return PCFR_OK;
}

// Online pruning (Sec. 5): the tree with the flagged actions removed before
// any iteration.  removed[n] != 0 on a child of a decision node drops the
// action leading to n and n's whole subtree.  Dropping whole subtrees keeps
// the surviving nodes in breadth-first order with siblings adjacent, so the
// reduced ids are the ranks of the kept nodes; new_id[n] is that rank, -1
// for a dropped node.  Children keep their order and their action index
// becomes their position among the kept siblings.
int32_t prune_tree(const Tree& in, const uint8_t* removed, Tree& out, std::vector<int32_t>& new_id) {
    const int32_t N = (int32_t)in.nodes.size();
    new_id.assign(N, -1);
    int32_t k = 0;
    for (int32_t i = 0; i < N; i++) {
        const Node& n = in.nodes[i];
        if (removed[i]) {
            if (n.parent < 0 || in.nodes[n.parent].type != PCFR_NODE_DECISION) {
                set_error("a pruning flag is set on a node that no decision action leads to");
                return PCFR_E_INVALID_ARG;
            }
            continue;
        }
        if (n.parent >= 0 && new_id[n.parent] < 0) continue;
        new_id[i] = k++;
    }
    Tree t{};
    t.spec = in.spec;
    t.root_mask = in.root_mask;
    t.nodes.reserve(k);
    for (int32_t i = 0; i < N; i++) {
        if (new_id[i] < 0) continue;
        const Node& src = in.nodes[i];
        Node nd = src;
        nd.parent = src.parent >= 0 ? new_id[src.parent] : -1;
        nd.first_child = -1;
        nd.n_child = 0;
        for (int32_t c = 0; c < src.n_child; c++) {
            const int32_t x = new_id[src.first_child + c];
            if (x < 0) continue;
            if (nd.first_child < 0) nd.first_child = x;
            nd.n_child++;
        }
        if (src.type == PCFR_NODE_DECISION && nd.n_child == 0) {
            set_error("pruning would remove every action of a decision node");
            return PCFR_E_INVALID_ARG;
        }
        t.nodes.push_back(nd);
        t.count[nd.type]++;
        if (nd.type == PCFR_NODE_DECISION) t.rows += nd.n_child;
        if (nd.depth + 1 > t.n_levels) t.n_levels = nd.depth + 1;
    }
    for (const Node& nd : t.nodes)
        for (int32_t c = 0; c < nd.n_child; c++) t.nodes[nd.first_child + c].action = c;
    out = std::move(t);
    return PCFR_OK;
}

}  // namespace pcfr
