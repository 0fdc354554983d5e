// Discounted CFR over a hold'em public tree on gfx950: device kernels, the
// solver runtime around them, and the solver half of the C ABI.
//
// Data layout (all in the caller's workspace):
//   every public node n owns a reach slot [2][Hp] and a value slot [2][Hp]
//   (player-major, hands contiguous, Hp = board-compatible hands padded to a
//   multiple of 64); decision node n owns rows rs..rs+A-1 of the regret
//   table R and the average-strategy table S, each row [Hp].  Hands are the
//   root-compatible combos in ascending combo order; padding lanes carry zero
//   reach and have no cards.
//
// One iteration (Sec. 4, Table 1), simultaneous for both players:
//   forward, level by level from the root (Stages 1-2): regret matching
//     (eq. rm) of each decision node, child reach = parent reach times the
//     actor's action probability, the other player's reach copied, chance
//     children masked by the dealt card; the average-strategy sum gets the
//     reach-weighted strategy and its DCFR discount in the same pass;
//   terminals, one workgroup per node (Stages 2-4): per-card and total
//     opponent reach, compatible mass by inclusion-exclusion over the two
//     cards of a hand, fold values; showdown values by a scan over hands
//     sorted by strength with per-card corrections;
//   backward, level by level to the root (Stages 6-7): eq. backward at the
//     actor's nodes, plain sums at the opponent's, 1/K-weighted sums at
//     chance nodes, and the regret update with DCFR discounting.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstddef>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "host.hpp"
#include "leafnet.hpp"

namespace pcfr {

enum { MODE_ITER = 0, MODE_BR = 1, MODE_EV = 2 };

struct __align__(16) DNode {
    int32_t type, player, first_child, n_child;
    int32_t rs, aux, sub, dead;   // aux: showdown board table, or chance divisor K;
                                  // dead: cards dealt since the root, c1 | c2 << 8 (0xff = none)
    int32_t slot[2];              // reach slot of each player (see below)
    int32_t id, pad;              // the node's own id (copies in the level sweep lists)
    double pay;                   // fold: folder's contribution; showdown: each contribution
};

// Reach slots.  A player's reach only changes at that player's own decision
// nodes, so a node shares the opponent's reach vector with its parent and a
// chance node's children share both of the parent's.  Slots 2g and 2g+1 hold
// subgame g's root ranges; the actor's reach after action a of the decision
// node with rows rs.. lives in slot 2 * n_sub + rs + a.  A slot read below a
// chance node still carries mass on hands holding a dealt card: every reader
// that needs those hands at zero (the average-strategy update, fold
// terminals) masks them with the node's dead cards; the showdown tables
// never list them.

// Per-iteration Stage-7 coefficients, computed on the device from t:
//   R <- (R + r) * (R + r > 0 ? dpos : dneg);   S <- (S + wadd * pi * sigma) * wmul
// DCFR: dpos = t^a/(t^a+1), dneg = t^b/(t^b+1), wadd = 1, wmul = (t/(t+1))^g.
// CFR+: dpos = 1, dneg = 0 (regrets floored at zero), wadd = t, wmul = 1.
// PCFR+: as CFR+ with wadd = t^2; the strategy matches on R + m, m the last
// instantaneous regret.
struct IterState {
    int64_t t;
    int32_t variant, pad;
    double dpos, dneg, wadd, wmul;
    double alpha, beta, gamma;    // set once at creation
    double thr0, thr;             // dynamic threshold: thr0 (set at creation), thr = thr0 / sqrt(t)
};

constexpr int kBlock = 256;       // terminal, leaf and helper kernels
constexpr int kFuseHands = 64;    // hands per workgroup of the level-fused sweeps
constexpr int kSweepMaxBlock = 512;
constexpr int kSdHeader = 64;     // card-list offsets per board table (53 used)
constexpr double kTieRel = 1e-10;  // instantaneous regrets this small against the actions' values are ties

// ------------------------------------------------------------ vector I/O
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
// NH consecutive hands of one row: the sweep kernels give each thread 4
// hands (one 16-byte access for FP32) where a level fills the GPU, 1 where
// a wave must cover one node's 64 hands.
template <typename T, int NH> struct VN { T e[NH]; };

template <int NH, typename T>
__device__ __forceinline__ VN<T, NH> ldv(const T* p) {
    VN<T, NH> v;
    if constexpr (NH == 4 && sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v.e[0] = q.x; v.e[1] = q.y; v.e[2] = q.z; v.e[3] = q.w;
    } else if constexpr (NH % 2 == 0 && sizeof(T) == 8) {
#pragma unroll
        for (int i = 0; i < NH / 2; i++) {
            const double2 q = reinterpret_cast<const double2*>(p)[i];
            v.e[2 * i] = q.x; v.e[2 * i + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < NH; i++) v.e[i] = p[i];
    }
    return v;
}
template <int NH, typename T>
__device__ __forceinline__ void stv(T* p, const VN<T, NH>& v) {
    if constexpr (NH == 4 && sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v.e[0], v.e[1], v.e[2], v.e[3]);
    } else if constexpr (NH % 2 == 0 && sizeof(T) == 8) {
#pragma unroll
        for (int i = 0; i < NH / 2; i++) reinterpret_cast<double2*>(p)[i] = make_double2(v.e[2 * i], v.e[2 * i + 1]);
    } else {
#pragma unroll
        for (int i = 0; i < NH; i++) p[i] = v.e[i];
    }
}

__device__ __forceinline__ bool has_card(uint32_t hc, int c) {
    return (int)(hc & 0xffu) == c || (int)(hc >> 8) == c;
}

// true when a hand's two cards (packed c1 | c2 << 8, 0xffff for padding) avoid both dead cards
__device__ __forceinline__ bool hand_alive(uint32_t hc, int dead) {
    const int a = hc & 0xff, b = hc >> 8, d1 = dead & 0xff, d2 = (dead >> 8) & 0xff;
    return a != 0xff && a != d1 && a != d2 && b != d1 && b != d2;
}

// ------------------------------------------------------------ iteration state
// Advances t and sets the coefficients; run by one thread of the first
// forward launch of an iteration (every later launch reads them).
__device__ void begin_iteration(IterState* st) {
    int64_t t = st->t + 1;
    st->t = t;
    double td = (double)t;
    st->thr = st->thr0 > 0.0 ? st->thr0 / sqrt(td) : 0.0;
    if (st->variant == PCFR_DCFR) {
        double ta = pow(td, st->alpha), tb = pow(td, st->beta);
        st->dpos = ta / (ta + 1.0);
        st->dneg = tb / (tb + 1.0);
        st->wadd = 1.0;
        st->wmul = pow(td / (td + 1.0), st->gamma);
    } else {
        st->dpos = 1.0;
        st->dneg = 0.0;
        st->wadd = st->variant == PCFR_CFRPLUS ? td : td * td;
        st->wmul = 1.0;
    }
}

// ------------------------------------------------------------ forward
// Strategy of one action for one hand: regret matching of R (MODE_ITER) or
// the normalised average-strategy sum S (other modes); uniform when the
// denominator vanishes.
template <typename T, int MODE>
__device__ __forceinline__ T strat(T x, T den, T inv_a) {
    if (MODE == MODE_ITER) return den > T(0) ? (x > T(0) ? x / den : T(0)) : inv_a;
    return den > T(0) ? x / den : inv_a;
}

// Dynamic thresholding: probabilities below thr become 0 and the others are
// renormalised (the largest probability is at least 1/A > thr, so one stays).
template <typename T, int A, int NH>
__device__ __forceinline__ void drop_below(T (&sg)[A][NH], T thr) {
    if (!(thr > T(0))) return;
#pragma unroll
    for (int j = 0; j < NH; j++) {
        T keep = T(0);
#pragma unroll
        for (int a = 0; a < A; a++) {
            if (sg[a][j] < thr) sg[a][j] = T(0);
            keep += sg[a][j];
        }
#pragma unroll
        for (int a = 0; a < A; a++) sg[a][j] /= keep;
    }
}

// Regret-based pruning flags: nzs[slot] != 0 when some hand has nonzero
// reach in that reach slot this iteration.  A node whose two slots are both
// unflagged is reached by no hand of either player.
__device__ __forceinline__ bool node_dead(const int32_t* nzs, const DNode& nd) {
    return nzs && nzs[nd.slot[0]] == 0 && nzs[nd.slot[1]] == 0;
}

// Sets nzs[slot] for the lanes whose rows hold a nonzero value, one atomic per
// distinct slot among those lanes of the wave (a wave can span two nodes).
__device__ __forceinline__ void flag_nonzero(int32_t* nzs, int slot, bool nz) {
    bool pending = nz;
    while (true) {
        const unsigned long long m = __ballot(pending);
        if (!m) break;
        const int lead = __ffsll(m) - 1;
        const int ls = __shfl(slot, lead);
        if (pending && slot == ls) {
            if ((int)__lane_id() == lead) atomicOr(&nzs[ls], 1);
            pending = false;
        }
    }
}

// Only the actor's reach is written: child a's actor slot gets the actor's
// reach times the probability of a; the other player's slot is shared.
template <typename T, int MODE, int A, int NH>
__device__ __forceinline__ void fwd_decision(const DNode& nd, int h, int Hp, int cbase, const T* __restrict__ R,
                                             const T* __restrict__ S, const T* __restrict__ Mp,
                                             T* __restrict__ reach, const IterState* __restrict__ st,
                                             int32_t* __restrict__ nzs, bool skip) {
    T* dst = reach + (int64_t)(cbase + nd.rs) * Hp + h;
    if (skip && node_dead(nzs, nd)) {
        // unreachable: the children's actor reach is zero; their flags stay clear
        const VN<T, NH> z = {};
#pragma unroll
        for (int a = 0; a < A; a++) stv<NH>(dst + (int64_t)a * Hp, z);
        return;
    }
    // (a select, not nd.slot[player]: a dynamic index would move nd to memory)
    const VN<T, NH> rp = ldv<NH>(reach + (int64_t)(nd.player ? nd.slot[1] : nd.slot[0]) * Hp + h);
    const T* src = (MODE == MODE_ITER ? R : S) + (int64_t)nd.rs * Hp + h;
    VN<T, NH> x[A];
#pragma unroll
    for (int a = 0; a < A; a++) x[a] = ldv<NH>(src + (int64_t)a * Hp);
    if (MODE == MODE_ITER && Mp) {
#pragma unroll
        for (int a = 0; a < A; a++) {
            const VN<T, NH> m = ldv<NH>(Mp + (int64_t)(nd.rs + a) * Hp + h);
#pragma unroll
            for (int j = 0; j < NH; j++) x[a].e[j] += m.e[j];
        }
    }
    T den[NH] = {};
#pragma unroll
    for (int a = 0; a < A; a++)
#pragma unroll
        for (int j = 0; j < NH; j++) den[j] += (MODE == MODE_ITER) ? (x[a].e[j] > T(0) ? x[a].e[j] : T(0)) : x[a].e[j];
    const T inv_a = T(1) / T(A);
    T sg[A][NH];
#pragma unroll
    for (int a = 0; a < A; a++)
#pragma unroll
        for (int j = 0; j < NH; j++) sg[a][j] = strat<T, MODE>(x[a].e[j], den[j], inv_a);
    if (MODE == MODE_ITER && st) drop_below<T, A, NH>(sg, (T)st->thr);
#pragma unroll
    for (int a = 0; a < A; a++) {
        VN<T, NH> q;
        bool nz = false;
#pragma unroll
        for (int j = 0; j < NH; j++) {
            q.e[j] = rp.e[j] * sg[a][j];
            nz |= q.e[j] != T(0);
        }
        stv<NH>(dst + (int64_t)a * Hp, q);
        if (nzs) flag_nonzero(nzs, cbase + nd.rs + a, nz);
    }
}

template <typename T, int MODE, int MAXA, int NH>
__device__ __forceinline__ void fwd_node(const DNode& nd, int h, int Hp, int cbase, const T* __restrict__ R,
                                         const T* __restrict__ S, const T* __restrict__ Mp, T* __restrict__ reach,
                                         const IterState* __restrict__ st, int32_t* __restrict__ nzs, bool skip) {
    switch (nd.n_child) {
#define PCFR_FWD_CASE(A) \
    case A:              \
        if constexpr (A <= MAXA) fwd_decision<T, MODE, A, NH>(nd, h, Hp, cbase, R, S, Mp, reach, st, nzs, skip); \
        break;
        PCFR_FWD_CASE(1) PCFR_FWD_CASE(2) PCFR_FWD_CASE(3) PCFR_FWD_CASE(4) PCFR_FWD_CASE(5) PCFR_FWD_CASE(6)
        PCFR_FWD_CASE(7) PCFR_FWD_CASE(8) PCFR_FWD_CASE(9) PCFR_FWD_CASE(10) PCFR_FWD_CASE(11) PCFR_FWD_CASE(12)
#undef PCFR_FWD_CASE
        default: break;
    }
}

// One thread per (decision node, 4 hands) of a level, the level's node
// records copied contiguously; chance nodes have no forward work (their
// children share their reach slots).
template <typename T, int MODE, int MAXA>
__global__ __launch_bounds__(kSweepMaxBlock) void k_forward(const DNode* __restrict__ level, int count, int Hp,
                                                            int cbase, const T* __restrict__ R,
                                                            const T* __restrict__ S, const T* __restrict__ Mp,
                                                            T* __restrict__ reach, IterState* begin,
                                                            const IterState* __restrict__ st, int32_t* __restrict__ nzs) {
    if (begin && blockIdx.x == 0 && threadIdx.x == 0) begin_iteration(begin);
    const int groups = Hp >> 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = gid / groups;
    if (k >= count) return;
    fwd_node<T, MODE, MAXA, 4>(level[k], (int)(gid - k * groups) * 4, Hp, cbase, R, S, Mp, reach, st, nzs, true);
}

// ------------------------------------------------------------ backward
// EARLY: load the average-strategy rows and own reach together with the
// regrets (more registers, one memory round trip less on the critical path;
// used where latency, not occupancy, limits).
// TF: children whose tv[a] is set (terminal values already evaluated by the
// calling workgroup into LDS rows [2][Hp]) are read there instead of from cfv.
template <typename T, int MODE, int A, int NH, bool EARLY, bool TF = false>
__device__ __forceinline__ void bwd_decision(const DNode& nd, int64_t n, int h, int Hp, T* __restrict__ R,
                                             T* __restrict__ S, T* __restrict__ Mp, const T* __restrict__ reach,
                                             T* __restrict__ cfv, const IterState* st,
                                             const uint16_t* __restrict__ hcards, T* __restrict__ root_dst,
                                             int upd, bool dead, const T* const* tv = nullptr) {
    // dead: no hand of either player reaches the node; its children's values
    // and its own reach are zero, so they are not loaded (regret-based pruning)
    using V = VN<T, NH>;
    const int p = nd.player, o = 1 - p;
    V x[A];
    V s_early[EARLY && MODE == MODE_ITER ? A : 1];
    V rp_early;
    T den[NH] = {};
    const T inv_a = T(1) / T(A);
    if (MODE != MODE_BR) {
        const T* src = (MODE == MODE_ITER ? (const T*)R : S) + (int64_t)nd.rs * Hp + h;
#pragma unroll
        for (int a = 0; a < A; a++) x[a] = ldv<NH>(src + (int64_t)a * Hp);
        if constexpr (EARLY && MODE == MODE_ITER) {
#pragma unroll
            for (int a = 0; a < A; a++) s_early[a] = ldv<NH>(S + (int64_t)(nd.rs + a) * Hp + h);
            if (dead) rp_early = V{};
            else rp_early = ldv<NH>(reach + (int64_t)(p ? nd.slot[1] : nd.slot[0]) * Hp + h);
        }
        if (MODE == MODE_ITER && Mp) {
            // the strategy of this iteration matched R + m; R itself is read again below
#pragma unroll
            for (int a = 0; a < A; a++) {
                const V m = ldv<NH>(Mp + (int64_t)(nd.rs + a) * Hp + h);
#pragma unroll
                for (int j = 0; j < NH; j++) x[a].e[j] += m.e[j];
            }
        }
#pragma unroll
        for (int a = 0; a < A; a++)
#pragma unroll
            for (int j = 0; j < NH; j++)
                den[j] += (MODE == MODE_ITER) ? (x[a].e[j] > T(0) ? x[a].e[j] : T(0)) : x[a].e[j];
    }
    // this iteration's strategy of each action (unused for a best response)
    T sg[MODE == MODE_BR ? 1 : A][NH];
    if constexpr (MODE != MODE_BR) {
#pragma unroll
        for (int a = 0; a < A; a++)
#pragma unroll
            for (int j = 0; j < NH; j++) sg[a][j] = strat<T, MODE>(x[a].e[j], den[j], inv_a);
        if (MODE == MODE_ITER) drop_below<T, A, NH>(sg, (T)st->thr);
    }
    // children's values, read once
    V c[A];
    V vp = {}, vo = {};
#pragma unroll
    for (int a = 0; a < A; a++) {
        const T* cc = cfv + (int64_t)(nd.first_child + a) * 2 * Hp;
        V d = {};
        if (dead) c[a] = V{};
        else if (TF && tv[a]) {
            c[a] = ldv<NH>(tv[a] + (int64_t)p * Hp + h);
            d = ldv<NH>(tv[a] + (int64_t)o * Hp + h);
        } else {
            c[a] = ldv<NH>(cc + (int64_t)p * Hp + h);
            d = ldv<NH>(cc + (int64_t)o * Hp + h);
        }
#pragma unroll
        for (int j = 0; j < NH; j++) {
            vo.e[j] += d.e[j];
            if constexpr (MODE == MODE_BR) vp.e[j] = (a == 0 || c[a].e[j] > vp.e[j]) ? c[a].e[j] : vp.e[j];
            else vp.e[j] += sg[a][j] * c[a].e[j];
        }
    }
    T* me = cfv + n * 2 * Hp;
    stv<NH>(me + (int64_t)p * Hp + h, vp);
    stv<NH>(me + (int64_t)o * Hp + h, vo);
    if (root_dst) {
        // with alternating updates each half keeps only the updated player's root values
        T* rd = root_dst + (int64_t)nd.sub * 2 * Hp;
        if (upd < 0 || upd == p) stv<NH>(rd + (int64_t)p * Hp + h, vp);
        if (upd < 0 || upd == o) stv<NH>(rd + (int64_t)o * Hp + h, vo);
    }
    if (MODE == MODE_ITER && (upd < 0 || upd == p)) {
        // Stage 7: regret update, and the reach-weighted strategy added to the
        // average-strategy sum (Stage 1's accumulation, done here so that one
        // pass reads and writes both tables), each with its DCFR discount.
        const T dpos = (T)st->dpos, dneg = (T)st->dneg, wadd = (T)st->wadd, wmul = (T)st->wmul;
        V rp;
        if constexpr (EARLY) rp = rp_early;
        else if (dead) rp = V{};
        else rp = ldv<NH>(reach + (int64_t)(p ? nd.slot[1] : nd.slot[0]) * Hp + h);
        if (nd.dead != 0xffff) {
            const uint16_t* hc = hcards + (int64_t)nd.sub * Hp + h;
#pragma unroll
            for (int j = 0; j < NH; j++)
                if (!hand_alive(hc[j], nd.dead)) rp.e[j] = T(0);
        }
        // ties: an instantaneous regret of at most kTieRel of the largest
        // action value of the information set is an exact tie (zero), since
        // regrets that vanish in exact arithmetic leave rounding residues of
        // either sign, which regret matching would follow
        T tie[NH];
#pragma unroll
        for (int j = 0; j < NH; j++) {
            T mx = T(0);
#pragma unroll
            for (int a = 0; a < A; a++) mx = fmax(mx, fabs(c[a].e[j]));
            tie[j] = T(kTieRel) * mx;
        }
#pragma unroll
        for (int a = 0; a < A; a++) {
            T* sp = S + (int64_t)(nd.rs + a) * Hp + h;
            T* rptr = R + (int64_t)(nd.rs + a) * Hp + h;
            V sv;
            if constexpr (EARLY) sv = s_early[a];
            else sv = ldv<NH>(sp);
            const V r0 = Mp ? ldv<NH>(rptr) : x[a];
            V y, inst;
#pragma unroll
            for (int j = 0; j < NH; j++) {
                // v(I.a) - v(I) as sum_b sigma_b (v_a - v_b): exactly tied actions
                // get exactly zero regret, whatever the rounding of v(I)
                T ia = T(0);
#pragma unroll
                for (int b = 0; b < A; b++) ia += sg[b][j] * (c[a].e[j] - c[b].e[j]);
                inst.e[j] = fabs(ia) <= tie[j] ? T(0) : ia;
                T r = r0.e[j] + inst.e[j];
                y.e[j] = r * (r > T(0) ? dpos : dneg);
                sv.e[j] = (sv.e[j] + wadd * (rp.e[j] * sg[a][j])) * wmul;
            }
            stv<NH>(rptr, y);
            stv<NH>(sp, sv);
            if (Mp) stv<NH>(Mp + (int64_t)(nd.rs + a) * Hp + h, inst);
        }
    }
}

// Suit isomorphism tables (null when off): cmap[2 node] = the child whose
// values stand for a chance child, cmap[2 node + 1] = the permutation taking
// that representative's card to the child's (-1: the child itself);
// hmap[(subgame * 24 + q) * Hp + h] = the hand pi_q^-1(h).
struct IsoTabs {
    const int32_t* cmap;
    const int16_t* hmap;
};

// Backward work of one node (decision or chance) for NH hands.
template <typename T, int MODE, int MAXA, int NH, bool EARLY>
__device__ __forceinline__ void bwd_node(const DNode& nd, int h, int Hp, T* __restrict__ R, T* __restrict__ S,
                                         T* __restrict__ Mp, const T* __restrict__ reach, T* __restrict__ cfv,
                                         const IterState* __restrict__ st, const uint16_t* __restrict__ hcards,
                                         T* __restrict__ root_dst, int upd, IsoTabs iso, const int32_t* __restrict__ nzs) {
    using V = VN<T, NH>;
    const int64_t n = nd.id;
    const bool dead = MODE == MODE_ITER && node_dead(nzs, nd);
    if (dead && nd.type == PCFR_NODE_CHANCE) {
        T* me = cfv + n * 2 * Hp;
        stv<NH>(me + h, V{});
        stv<NH>(me + Hp + h, V{});
        return;
    }
    if (nd.type == PCFR_NODE_CHANCE && nd.pad) {
        // some children solved through a suit-isomorphic representative:
        // v(h | pi c) = v(pi^-1 h | c); children added in their order
        V a0 = {}, a1 = {};
        for (int j = 0; j < nd.n_child; j++) {
            const int64_t ch = nd.first_child + j;
            const int32_t src = iso.cmap[2 * ch], q = iso.cmap[2 * ch + 1];
            const T* cc = cfv + (int64_t)src * 2 * Hp;
            V u, w;
            if (q < 0) {
                u = ldv<NH>(cc + h);
                w = ldv<NH>(cc + Hp + h);
            } else {
                const int16_t* mp = iso.hmap + ((int64_t)nd.sub * 24 + q) * Hp + h;
#pragma unroll
                for (int e = 0; e < NH; e++) {
                    const int hm = mp[e];
                    u.e[e] = cc[hm];
                    w.e[e] = cc[Hp + hm];
                }
            }
#pragma unroll
            for (int e = 0; e < NH; e++) { a0.e[e] += u.e[e]; a1.e[e] += w.e[e]; }
        }
        const T inv_k = T(1) / T(nd.aux);
#pragma unroll
        for (int e = 0; e < NH; e++) { a0.e[e] *= inv_k; a1.e[e] *= inv_k; }
        T* me = cfv + n * 2 * Hp;
        stv<NH>(me + h, a0);
        stv<NH>(me + Hp + h, a1);
        return;
    }
    if (nd.type == PCFR_NODE_CHANCE) {
        // children in groups of 4: all loads of a group are issued before the
        // adds, which keep the children's order
        constexpr int G = 4;
        V a0 = {}, a1 = {};
        for (int c0 = 0; c0 < nd.n_child; c0 += G) {
            V u[G], w[G];
#pragma unroll
            for (int q = 0; q < G; q++) {
                if (c0 + q < nd.n_child) {
                    const T* cc = cfv + (int64_t)(nd.first_child + c0 + q) * 2 * Hp;
                    u[q] = ldv<NH>(cc + h);
                    w[q] = ldv<NH>(cc + Hp + h);
                }
            }
#pragma unroll
            for (int q = 0; q < G; q++) {
                if (c0 + q < nd.n_child) {
#pragma unroll
                    for (int j = 0; j < NH; j++) { a0.e[j] += u[q].e[j]; a1.e[j] += w[q].e[j]; }
                }
            }
        }
        const T inv_k = T(1) / T(nd.aux);
#pragma unroll
        for (int j = 0; j < NH; j++) { a0.e[j] *= inv_k; a1.e[j] *= inv_k; }
        T* me = cfv + n * 2 * Hp;
        stv<NH>(me + h, a0);
        stv<NH>(me + Hp + h, a1);
        return;
    }
    switch (nd.n_child) {
#define PCFR_BWD_CASE(A) \
    case A:              \
        if constexpr (A <= MAXA) bwd_decision<T, MODE, A, NH, EARLY && (sizeof(T) == 4 || A <= 8)>(nd, n, h, Hp, R, S, Mp, reach, cfv, st, hcards, root_dst, upd, dead); \
        break;
        PCFR_BWD_CASE(1) PCFR_BWD_CASE(2) PCFR_BWD_CASE(3) PCFR_BWD_CASE(4) PCFR_BWD_CASE(5) PCFR_BWD_CASE(6)
        PCFR_BWD_CASE(7) PCFR_BWD_CASE(8) PCFR_BWD_CASE(9) PCFR_BWD_CASE(10) PCFR_BWD_CASE(11) PCFR_BWD_CASE(12)
#undef PCFR_BWD_CASE
        default: break;
    }
}

// One thread per (node, 4 hands) of a level, decision and chance nodes.
// root_dst (the last launch of an iteration only) also receives each root's
// values, which later evaluation sweeps do not overwrite.  upd >= 0 limits
// Stage 7 (and the root values kept) to that player: alternating updates.
template <typename T, int MODE, int MAXA>
__global__ __launch_bounds__(kSweepMaxBlock) void k_backward(const DNode* __restrict__ level, int count, int Hp,
                                                             T* __restrict__ R, T* __restrict__ S, T* __restrict__ Mp,
                                                             const T* __restrict__ reach, T* __restrict__ cfv,
                                                             const IterState* __restrict__ st,
                                                             const uint16_t* __restrict__ hcards,
                                                             T* __restrict__ root_dst, int upd, IsoTabs iso,
                                                             const int32_t* __restrict__ nzs) {
    const int groups = Hp >> 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = gid / groups;
    if (k >= count) return;
    bwd_node<T, MODE, MAXA, 4, false>(level[k], (int)(gid - k * groups) * 4, Hp, R, S, Mp, reach, cfv, st, hcards,
                                      root_dst, upd, iso, nzs);
}

// Level-fused sweeps for runs of levels too small to fill the GPU.  A node's
// reach at hand h depends only on its parent's at h, and its values at h only
// on its children's at h, so a workgroup that owns a slice of kFuseHands
// hands can run consecutive levels for that slice with workgroup barriers
// in between: one launch instead of one per level.  Each wave takes one
// node at a time, one hand per lane, so that the node (its record, its
// action count, its kind) is the same across the wave: scalar record loads
// and no divergence between nodes of different shapes.  The workgroup's
// kFuseWaves waves are its node lanes; lvl_off holds the level starts in the
// record list.
constexpr int kFuseWaves = 16;
constexpr int kFuseBlock = kFuseWaves * 64;
static_assert(kFuseHands == 64, "one hand per lane of a wave");

__device__ __forceinline__ int fuse_lane() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

template <typename T, int MODE, int MAXA>
__global__ __launch_bounds__(kFuseBlock) void k_forward_fused(const DNode* __restrict__ rec,
                                                              const int64_t* __restrict__ lvl_off, int l0, int l1,
                                                              int Hp, int cbase, const T* __restrict__ R,
                                                              const T* __restrict__ S, const T* __restrict__ Mp,
                                                              T* __restrict__ reach, IterState* begin,
                                                              const IterState* __restrict__ st,
                                                              int32_t* __restrict__ nzs) {
    if (begin && blockIdx.x == 0 && threadIdx.x == 0) begin_iteration(begin);
    const int h = blockIdx.x * kFuseHands + (int)(threadIdx.x & 63), lane = fuse_lane();
    // The pruning flags of a node's slots are set by every workgroup of this
    // launch (each owns a slice of hands), so they are incomplete here: the
    // fused levels set flags for later launches but skip nothing (an
    // unreachable node's rows are zero and come out zero anyway).
    for (int l = l0; l < l1; l++) {
        if (l > l0) __syncthreads();
        const int64_t e = lvl_off[l + 1];
        for (int64_t k = lvl_off[l] + lane; k < e; k += kFuseWaves)
            fwd_node<T, MODE, MAXA, 1>(rec[k], h, Hp, cbase, R, S, Mp, reach, st, nzs, false);
    }
}

// Levels l_hi - 1 down to l_lo; root_dst as in k_backward (used when l_lo is 0).
template <typename T, int MODE, int MAXA>
__global__ __launch_bounds__(kFuseBlock) void k_backward_fused(const DNode* __restrict__ rec,
                                                               const int64_t* __restrict__ lvl_off, int l_lo,
                                                               int l_hi, int Hp, T* __restrict__ R,
                                                               T* __restrict__ S, T* __restrict__ Mp,
                                                               const T* __restrict__ reach, T* __restrict__ cfv,
                                                               const IterState* __restrict__ st,
                                                               const uint16_t* __restrict__ hcards,
                                                               T* __restrict__ root_dst, int upd, IsoTabs iso,
                                                               const int32_t* __restrict__ nzs) {
    const int h = blockIdx.x * kFuseHands + (int)(threadIdx.x & 63), lane = fuse_lane();
    for (int l = l_hi - 1; l >= l_lo; l--) {
        if (l < l_hi - 1) __syncthreads();
        const int64_t e = lvl_off[l + 1];
        for (int64_t k = lvl_off[l] + lane; k < e; k += kFuseWaves)
            bwd_node<T, MODE, MAXA, 1, true>(rec[k], h, Hp, R, S, Mp, reach, cfv, st, hcards,
                                             l == 0 ? root_dst : nullptr, upd, iso, nzs);
    }
}

// ------------------------------------------------------------ terminals
// Both terminal kinds are latency-bound (a few thousand hands per workgroup),
// so every stage first issues all of a thread's global loads (fixed trip
// counts, predicated) and only then consumes them, and block reductions and
// scans use wave shuffles with one LDS exchange between the 4 waves.
constexpr int kMaxHp = 1216;                          // flop: 1176 compatible combos padded to 64
constexpr int kHandIt = (kMaxHp + kBlock - 1) / kBlock;
constexpr int kWaves = kBlock / 64;

// Copy n int16 values (n a multiple of 8, both pointers 16-byte aligned) to LDS.
template <int MAXV>
__device__ __forceinline__ void copy_i16(int16_t* dst, const int16_t* __restrict__ src, int n) {
    const int nv = n >> 3;
    u32x4 v[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; i++) {
        const int j = threadIdx.x + i * kBlock;
        if (j < nv) v[i] = reinterpret_cast<const u32x4*>(src)[j];
    }
#pragma unroll
    for (int i = 0; i < MAXV; i++) {
        const int j = threadIdx.x + i * kBlock;
        if (j < nv) reinterpret_cast<u32x4*>(dst)[j] = v[i];
    }
}

// Sum over the workgroup of a and b (every thread gets both totals);
// xch: LDS scratch of 2 * kWaves values.
template <typename T>
__device__ __forceinline__ void block_sum2(T& a, T& b, T* xch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { xch[w] = a; xch[kWaves + w] = b; }
    __syncthreads();
    a = T(0);
    b = T(0);
#pragma unroll
    for (int i = 0; i < kWaves; i++) { a += xch[i]; b += xch[kWaves + i]; }
}

// Sums over the workgroup of a, b, c, d (every thread gets all four totals);
// xch: LDS scratch of 4 * kWaves values.
template <typename T>
__device__ __forceinline__ void block_sum4(T& a, T& b, T& c, T& d, T* xch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        c += __shfl_xor(c, o);
        d += __shfl_xor(d, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { xch[w] = a; xch[kWaves + w] = b; xch[2 * kWaves + w] = c; xch[3 * kWaves + w] = d; }
    __syncthreads();
    a = b = c = d = T(0);
#pragma unroll
    for (int i = 0; i < kWaves; i++) {
        a += xch[i]; b += xch[kWaves + i]; c += xch[2 * kWaves + i]; d += xch[3 * kWaves + i];
    }
}

// Exclusive scan over the workgroup of a and b in thread order; the totals
// come back in ta, tb.  xch: LDS scratch of 2 * kWaves values.  With
// c, d given, their plain workgroup sums come back in them, through the
// same exchange (xch then holds 4 * kWaves values).
template <typename T, bool SUM2 = false>
__device__ __forceinline__ void block_exscan2(T& a, T& b, T& ta, T& tb, T* xch, T* c = nullptr, T* d = nullptr) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T ia = a, ib = b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T ua = __shfl_up(ia, o), ub = __shfl_up(ib, o);
        if (lane >= o) { ia += ua; ib += ub; }
    }
    T sc = T(0), sd = T(0);
    if constexpr (SUM2) {
        sc = *c;
        sd = *d;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sc += __shfl_xor(sc, o);
            sd += __shfl_xor(sd, o);
        }
    }
    if (lane == 63) {
        xch[w] = ia;
        xch[kWaves + w] = ib;
        if constexpr (SUM2) { xch[2 * kWaves + w] = sc; xch[3 * kWaves + w] = sd; }
    }
    __syncthreads();
    T oa = T(0), ob = T(0);
    ta = T(0);
    tb = T(0);
    if constexpr (SUM2) { *c = T(0); *d = T(0); }
#pragma unroll
    for (int i = 0; i < kWaves; i++) {
        if (i < w) { oa += xch[i]; ob += xch[kWaves + i]; }
        ta += xch[i];
        tb += xch[kWaves + i];
        if constexpr (SUM2) { *c += xch[2 * kWaves + i]; *d += xch[3 * kWaves + i]; }
    }
    a = oa + ia - a;
    b = ob + ib - b;
}

// Fold: v_i(h) = -+ c_f * M_{-i}(h) where M(h) is the opponent reach over
// hands sharing no card with h: total - per-card(a) - per-card(b) + r(h)
// (the hand itself was removed twice).  Both reach vectors and the per-card
// hand lists are staged in LDS first, so the 104 per-card sums read LDS only;
// hands holding a card dealt below the root are staged as zero reach.  The
// same inclusion-exclusion over counts of hands with nonzero reach tells
// when no compatible opponent hand has reach at all: M is then exactly 0 (as
// a sum over those hands is), not the rounding residue of the difference,
// so hands whose every action is worth nothing tie exactly.
// Core of the fold terminal: a[i], b[i] are the two players' reach of the
// thread's hands tid + i * kBlock (read by the caller), v0 / v1 receive the
// node's values (global or LDS rows of Hp).
template <typename T>
__device__ void term_fold_core(const DNode& nd, int Hp, T (&a)[kHandIt], T (&b)[kHandIt],
                               const uint16_t* __restrict__ hc, const int32_t* __restrict__ coff,
                               const int16_t* __restrict__ chands, T* lds, T* v0, T* v1) {
    T* x0 = lds;                  // [Hp]
    T* x1 = x0 + Hp;              // [Hp]
    T* pc = x1 + Hp;              // [2][52], two half-sums per card first: [208]
    T* xch = pc + 208;            // [2 * kWaves] sums, then [2 * kWaves] counts; padded to 2 * kBlock
    int16_t* lst = reinterpret_cast<int16_t*>(xch + 2 * kBlock);     // [2 * Hp]
    int32_t* pcn = reinterpret_cast<int32_t*>(lst + 2 * Hp);         // [208]: per-card counts, as pc
    const int tid = threadIdx.x;
    const int nl = coff[52];
    copy_i16<(2 * kMaxHp / 8 + kBlock - 1) / kBlock>(lst, chands, (nl + 7) & ~7);
    uint32_t c[kHandIt];
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        if (h < Hp) c[i] = hc[h];
    }
    T s0 = T(0), s1 = T(0), n0 = T(0), n1 = T(0);
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        if (h < Hp) {
            if (!hand_alive(c[i], nd.dead)) { a[i] = T(0); b[i] = T(0); }
            x0[h] = a[i];
            x1[h] = b[i];
            s0 += a[i];
            s1 += b[i];
            n0 += a[i] != T(0) ? T(1) : T(0);
            n1 += b[i] != T(0) ? T(1) : T(0);
        }
    }
    __syncthreads();
    if (tid < 208) {
        // two threads per (player, card), each summing half of the card's list
        const int pcix = tid >> 1, half = tid & 1;
        const int p = pcix / 52, cd = pcix - p * 52;
        const T* x = p ? x1 : x0;
        const int lo = coff[cd], hi = coff[cd + 1], mid = lo + ((hi - lo) >> 1);
        T acc = T(0);
        int cnt = 0;
        // eight list entries per step: their index loads, then their value
        // loads, are issued together (one LDS round trip each per step
        // instead of per entry); the sum keeps its sequential order
        int j = half ? mid : lo;
        const int je = half ? hi : mid;
        for (; j + 8 <= je; j += 8) {
            int ix[8];
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) ix[u] = lst[j + u];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = x[ix[u]];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                acc += v[u];
                cnt += v[u] != T(0);
            }
        }
        for (; j < je; j++) {
            const T v = x[lst[j]];
            acc += v;
            cnt += v != T(0);
        }
        pc[tid] = acc;
        pcn[tid] = cnt;
    }
    block_sum4(s0, s1, n0, n1, xch);   // synchronises: the half-sums are visible after it
    T pcv0 = T(0), pcv1 = T(0);
    int pcn0 = 0, pcn1 = 0;
    if (tid < 104) { pcv0 = pc[2 * tid]; pcv1 = pc[2 * tid + 1]; pcn0 = pcn[2 * tid]; pcn1 = pcn[2 * tid + 1]; }
    __syncthreads();
    if (tid < 104) { pc[tid] = pcv0 + pcv1; pcn[tid] = pcn0 + pcn1; }
    __syncthreads();
    const int nz0 = (int)n0, nz1 = (int)n1;
    const int f = nd.player;
    const T pay = (T)nd.pay;
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        if (h >= Hp) break;
        const int ca = c[i] & 0xff, cb = c[i] >> 8;
        T m0 = T(0), m1 = T(0);
        if (hand_alive(c[i], nd.dead)) {
            if (nz0 - pcn[ca] - pcn[cb] + (x0[h] != T(0)) > 0) m0 = s0 - pc[ca] - pc[cb] + x0[h];
            if (nz1 - pcn[52 + ca] - pcn[52 + cb] + (x1[h] != T(0)) > 0) m1 = s1 - pc[52 + ca] - pc[52 + cb] + x1[h];
        }
        v0[h] = (f == 0 ? -pay : pay) * m1;
        v1[h] = (f == 1 ? -pay : pay) * m0;
    }
}

template <typename T>
__device__ void term_fold(const DNode& nd, int64_t n, int Hp, const T* __restrict__ reach, T* __restrict__ cfv,
                          const uint16_t* __restrict__ hc, const int32_t* __restrict__ coff,
                          const int16_t* __restrict__ chands, T* lds) {
    const T* r0 = reach + (int64_t)nd.slot[0] * Hp;
    const T* r1 = reach + (int64_t)nd.slot[1] * Hp;
    T a[kHandIt], b[kHandIt];
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = threadIdx.x + i * kBlock;
        if (h < Hp) { a[i] = r0[h]; b[i] = r1[h]; }
    }
    T* v0 = cfv + n * 2 * Hp;
    term_fold_core<T>(nd, Hp, a, b, hc, coff, chands, lds, v0, v0 + Hp);
}

// Showdown on a five-card board: hands sorted by value ascending (perm),
// with tie groups [glo, ghi) in sorted positions; every card has the list of
// sorted positions of hands holding it, ascending, followed by one slot for
// the list total; [alo, ahi) and [blo, bhi) are the tie group of a hand inside
// the lists of its two cards.  W = opponent reach of compatible weaker hands,
// L = of compatible stronger ones; ties pay nothing.  The board's table
// lists only hands alive on it, so no dealt-card masking is needed.  As for
// folds, a hand none of whose compatible opponent hands has nonzero reach
// (counted by the same inclusion-exclusion) gets exactly 0; and W or L is
// exactly 0 when no compatible weaker (stronger) hand has nonzero reach, so
// a hand whose reaching opponents all tie with it is worth exactly 0 (the
// differences of prefixes would leave rounding residues whose signs regret
// matching then follows).  Those counts come from bitmasks of the nonzero
// reaches, in sorted order and in card-list order, with per-word prefix
// counts; they are taken only where W and L are both within rounding of 0.
// Core of the showdown terminal: ra[i], rb[i] are the two players' reach of
// hand tid + i * kBlock in hand order (read by the caller); v0 / v1 receive
// the node's values.
template <typename T>
__device__ void term_showdown_core(const DNode& nd, int Hp, T (&ra)[kHandIt], T (&rb)[kHandIt],
                                   const int16_t* __restrict__ tb, int Hb, T* lds, T* v0, T* v1) {
    const int QN = 2 * Hp + kSdHeader;
    T* xs0 = lds;                 // [Hp + 4]: sorted reach, then its exclusive prefix
    T* xs1 = xs0 + (Hp + 4);
    T* q0 = xs1 + (Hp + 4);       // [QN]: card-list exclusive prefixes
    T* q1 = q0 + QN;
    T* xch = q1 + QN;             // [2 * kWaves] scan, then [2 * kWaves] counts; padded to 2 * kBlock
    int16_t* coff = reinterpret_cast<int16_t*>(xch + 2 * kBlock);     // [kSdHeader]
    int16_t* clist = coff + kSdHeader;                                // [QN]
    int16_t* perm = clist + QN;                                       // [Hp]
    int32_t* cnz = reinterpret_cast<int32_t*>(perm + Hp);             // [2][52]: hands with reach per card
    // nonzero-reach bitmasks: card-list order [2][NW], sorted order [2][NS],
    // and their exclusive per-word prefix counts ([2][NW], [2][NS + 1]); the
    // byte offset of lw is a multiple of 8 since Hp is a multiple of 64
    const int NW = (QN + 63) >> 6, NS = Hp >> 6;
    uint64_t* lw = reinterpret_cast<uint64_t*>(cnz + 104);
    uint64_t* sw = lw + 2 * NW;
    int32_t* lpre = reinterpret_cast<int32_t*>(sw + 2 * NS);
    int32_t* spre = lpre + 2 * NW;
    const int16_t* glo = tb + Hp;
    const int16_t* ghi = tb + 2 * Hp;
    const int16_t* alo = tb + 3 * Hp;
    const int16_t* ahi = tb + 4 * Hp;
    const int16_t* blo = tb + 5 * Hp;
    const int16_t* bhi = tb + 6 * Hp;
    const int tid = threadIdx.x;

    // Every global load first, none through the permutation: the card-list
    // offsets and lists (2 * Hb + 52 entries <= QN), the permutation, this
    // thread's table entries and the cards of its sorted hands, and both
    // reach rows in hand order (coalesced).  The reach rows are staged in q0 /
    // q1, which the card-list prefixes overwrite only after the permuted
    // gather below has read them from LDS.
    copy_i16<((kSdHeader + 2 * kMaxHp + kSdHeader) / 8 + kBlock - 1) / kBlock>(coff, tb + 8 * Hp, kSdHeader + QN);
    copy_i16<(kMaxHp / 8 + kBlock - 1) / kBlock>(perm, tb, Hp);
    const uint16_t* scard = reinterpret_cast<const uint16_t*>(tb + 7 * Hp);
    int s_gl[kHandIt], s_gh[kHandIt], s_al[kHandIt], s_ah[kHandIt], s_bl[kHandIt], s_bh[kHandIt];
    uint32_t cc[kHandIt];
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int s = tid + i * kBlock;
        if (s < Hb) {
            s_gl[i] = glo[s]; s_gh[i] = ghi[s]; s_al[i] = alo[s];
            s_ah[i] = ahi[s]; s_bl[i] = blo[s]; s_bh[i] = bhi[s];
            cc[i] = scard[s];
        }
    }
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        if (h < Hp) { q0[h] = ra[i]; q1[h] = rb[i]; }
    }
    __syncthreads();
    int hh[kHandIt];
    T a[kHandIt], b[kHandIt];
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int s = tid + i * kBlock;
        hh[i] = s < Hp ? perm[s] : 0;
        if (s < Hb) { a[i] = q0[hh[i]]; b[i] = q1[hh[i]]; }
    }
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int s = tid + i * kBlock;
        if (s < Hb) { xs0[s] = a[i]; xs1[s] = b[i]; }
        // the wave's 64 positions form one word of the sorted bitmasks
        const uint64_t m0 = __ballot(s < Hb && a[i] != T(0));
        const uint64_t m1 = __ballot(s < Hb && b[i] != T(0));
        const int wd = (i * kBlock >> 6) + wv;
        if (lane == 0 && wd < NS) { sw[wd] = m0; sw[NS + wd] = m1; }
    }
    __syncthreads();
    if (tid < 104) {
        const int p = tid / 52, c = tid - p * 52;
        const T* xs = p ? xs1 : xs0;
        T* q = p ? q1 : q0;
        const int lo = coff[c], hi = coff[c + 1] - 1;
        T acc = T(0);
        int nz = 0;
        int j = lo;
        // eight entries per step: index loads, then value loads, issued
        // together; the prefix keeps its sequential order
        for (; j + 8 <= hi; j += 8) {
            int ix[8];
            T y[8];
#pragma unroll
            for (int u = 0; u < 8; u++) ix[u] = clist[j + u];
#pragma unroll
            for (int u = 0; u < 8; u++) y[u] = xs[ix[u]];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                q[j + u] = acc;
                acc += y[u];
                nz += y[u] != T(0);
            }
        }
        for (; j < hi; j++) { const T y = xs[clist[j]]; q[j] = acc; acc += y; nz += y != T(0); }
        q[hi] = acc;
        cnz[tid] = nz;
    }
    if (wv >= 2) {
        // meanwhile the last two waves build the card-list bitmasks, one
        // 64-entry word per ballot (a list's total slot holds -1: no bit),
        // ten words per step with their loads issued together
        constexpr int kMaxNW = (2 * kMaxHp + kSdHeader + 63) / 64;
        constexpr int kStep = 10;
        const int nl = coff[52];
#pragma unroll
        for (int k0 = 0; k0 < (kMaxNW + 1) / 2; k0 += kStep) {
            int ix[kStep];
            T y0[kStep], y1[kStep];
#pragma unroll
            for (int u = 0; u < kStep; u++) {
                const int j = ((wv - 2) + 2 * (k0 + u)) * 64 + lane;
                ix[u] = j < nl ? clist[j] : -1;
            }
#pragma unroll
            for (int u = 0; u < kStep; u++) {
                const int x = ix[u] < 0 ? 0 : ix[u];
                y0[u] = xs0[x];
                y1[u] = xs1[x];
            }
#pragma unroll
            for (int u = 0; u < kStep; u++) {
                const int wd = (wv - 2) + 2 * (k0 + u);
                const uint64_t m0 = __ballot(ix[u] >= 0 && y0[u] != T(0));
                const uint64_t m1 = __ballot(ix[u] >= 0 && y1[u] != T(0));
                if (lane == 0 && wd < NW) { lw[wd] = m0; lw[NW + wd] = m1; }
            }
        }
    }
    // exclusive scan of xs0 / xs1 over [0, Hb) in sorted order: each thread
    // owns a contiguous chunk, chunk sums are scanned across the workgroup
    constexpr int kMaxChunk = (kMaxHp + kBlock - 1) / kBlock;
    const int chunk = (Hb + kBlock - 1) / kBlock;
    const int beg = tid * chunk;
    T l0[kMaxChunk], l1[kMaxChunk];
    T s0 = T(0), s1 = T(0), n0 = T(0), n1 = T(0);
#pragma unroll
    for (int i = 0; i < kMaxChunk; i++) {
        const int s = beg + i;
        const bool in = i < chunk && s < Hb;
        l0[i] = in ? xs0[s] : T(0);
        l1[i] = in ? xs1[s] : T(0);
        s0 += l0[i];
        s1 += l1[i];
        n0 += l0[i] != T(0) ? T(1) : T(0);
        n1 += l1[i] != T(0) ? T(1) : T(0);
    }
    T tot0, tot1;
    block_exscan2<T, true>(s0, s1, tot0, tot1, xch, &n0, &n1);   // synchronises: every chunk was read above
    const int nz0 = (int)n0, nz1 = (int)n1;
    {
        // exclusive per-word prefix counts of the four bitmasks, one wave each
        // (the bitmasks are complete: the scan above synchronised)
        static_assert(kWaves >= 4, "one wave per bitmask");
        if (wv < 4) {
            const int n = wv < 2 ? NW : NS;
            const uint64_t* src = wv < 2 ? lw + wv * NW : sw + (wv - 2) * NS;
            int32_t* dst = wv < 2 ? lpre + wv * NW : spre + (wv - 2) * (NS + 1);
            const int c = lane < n ? __popcll(src[lane]) : 0;
            int inc = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(inc, o);
                if (lane >= o) inc += u;
            }
            if (lane < n) dst[lane] = inc - c;
            if (wv >= 2 && lane == n - 1) dst[n] = inc;
        }
    }
    __syncthreads();                          // all reads of xs done before it is overwritten
#pragma unroll
    for (int i = 0; i < kMaxChunk; i++) {
        const int s = beg + i;
        if (i < chunk && s < Hb) {
            xs0[s] = s0;
            xs1[s] = s1;
            s0 += l0[i];
            s1 += l1[i];
        }
    }
    if (tid == 0) { xs0[Hb] = tot0; xs1[Hb] = tot1; }
    __syncthreads();

    const T pay = (T)nd.pay;
    // hands with nonzero reach of player p among sorted positions [0, x) and
    // among card-list positions [0, x)
    auto cnt_sorted = [&](int p, int x) {
        const int k = x >> 6, r = x & 63;
        int c = spre[p * (NS + 1) + k];
        if (r) c += __popcll(sw[p * NS + k] & ((1ull << r) - 1));
        return c;
    };
    auto cnt_list = [&](int p, int x) {
        const int k = x >> 6, r = x & 63;
        int c = lpre[p * NW + k];
        if (r) c += __popcll(lw[p * NW + k] & ((1ull << r) - 1));
        return c;
    };
    // a bound on the rounding error of W and L (sums of at most Hb terms,
    // each prefix at most the player's total reach, five prefixes and four
    // differences): beyond it the exact value is certainly nonzero
    constexpr T kEps = sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-07);
    const T e0 = T(8 * (Hb + 1)) * kEps * tot0, e1 = T(8 * (Hb + 1)) * kEps * tot1;
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int s = tid + i * kBlock;
        if (s >= Hp) break;
        const int h = hh[i];
        if (s >= Hb) { v0[h] = T(0); v1[h] = T(0); continue; }
        const int ca = cc[i] & 0xff, cb = cc[i] >> 8;
        const int ae = coff[ca + 1] - 1, be = coff[cb + 1] - 1;
        const int gl = s_gl[i], gh = s_gh[i], al = s_al[i], ah = s_ah[i], bl = s_bl[i], bh = s_bh[i];
        // against player 1's reach (value of player 0)
        T w1 = xs1[gl] - q1[al] - q1[bl];
        T lo1 = (tot1 - xs1[gh]) - (q1[ae] - q1[ah]) - (q1[be] - q1[bh]);
        T w0 = xs0[gl] - q0[al] - q0[bl];
        T lo0 = (tot0 - xs0[gh]) - (q0[ae] - q0[ah]) - (q0[be] - q0[bh]);
        const bool any1 = nz1 - cnz[52 + ca] - cnz[52 + cb] + (b[i] != T(0)) > 0;
        const bool any0 = nz0 - cnz[ca] - cnz[cb] + (a[i] != T(0)) > 0;
        const int la = coff[ca], lb = coff[cb];
        if (any1 && fabs(w1) <= e1 && fabs(lo1) <= e1) {
            if (cnt_sorted(1, gl) - (cnt_list(1, al) - cnt_list(1, la)) - (cnt_list(1, bl) - cnt_list(1, lb)) == 0)
                w1 = T(0);
            if ((nz1 - cnt_sorted(1, gh)) - (cnt_list(1, ae) - cnt_list(1, ah)) - (cnt_list(1, be) - cnt_list(1, bh)) == 0)
                lo1 = T(0);
        }
        if (any0 && fabs(w0) <= e0 && fabs(lo0) <= e0) {
            if (cnt_sorted(0, gl) - (cnt_list(0, al) - cnt_list(0, la)) - (cnt_list(0, bl) - cnt_list(0, lb)) == 0)
                w0 = T(0);
            if ((nz0 - cnt_sorted(0, gh)) - (cnt_list(0, ae) - cnt_list(0, ah)) - (cnt_list(0, be) - cnt_list(0, bh)) == 0)
                lo0 = T(0);
        }
        v0[h] = any1 ? pay * (w1 - lo1) : T(0);
        v1[h] = any0 ? pay * (w0 - lo0) : T(0);
    }
}

template <typename T>
__device__ void term_showdown(const DNode& nd, int64_t n, int Hp, const T* __restrict__ reach, T* __restrict__ cfv,
                              const uint16_t* __restrict__ hc, const int16_t* __restrict__ tb, int Hb, T* lds) {
    const T* r0 = reach + (int64_t)nd.slot[0] * Hp;
    const T* r1 = reach + (int64_t)nd.slot[1] * Hp;
    T ra[kHandIt], rb[kHandIt];
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int s = threadIdx.x + i * kBlock;
        if (s < Hp) { ra[i] = r0[s]; rb[i] = r1[s]; }
    }
    T* v0 = cfv + n * 2 * Hp;
    term_showdown_core<T>(nd, Hp, ra, rb, tb, Hb, lds, v0, v0 + Hp);
}

// One workgroup per terminal node of one kind (KIND 0: folds, 1: showdowns):
// a kernel per kind, so that the lighter fold path is not held to the
// registers of the showdown path.  recs: the nodes' records in launch order
// (each carries its id), so a workgroup's first load has a known address.
template <typename T, int KIND>
__global__ __launch_bounds__(kBlock) void k_terminal(const DNode* __restrict__ recs,
                                                     int Hp, const T* __restrict__ reach, T* __restrict__ cfv,
                                                     const uint16_t* __restrict__ hcards, const int32_t* __restrict__ coff,
                                                     const int16_t* __restrict__ chands, int chand_stride,
                                                     const int16_t* __restrict__ sd, int64_t sd_stride,
                                                     const int32_t* __restrict__ sd_n,
                                                     const int32_t* __restrict__ nzs) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    const DNode nd = recs[blockIdx.x];
    const int64_t n = nd.id;
    if (node_dead(nzs, nd)) {
        // unreachable (regret-based pruning): both value rows are zero
        T* v = cfv + n * 2 * Hp;
        for (int i = threadIdx.x; i < 2 * Hp; i += blockDim.x) v[i] = T(0);
        return;
    }
    const uint16_t* hc = hcards + (int64_t)nd.sub * Hp;
    if constexpr (KIND == 0)
        term_fold<T>(nd, n, Hp, reach, cfv, hc, coff + nd.sub * 53, chands + (int64_t)nd.sub * chand_stride, lds);
    else
        term_showdown<T>(nd, n, Hp, reach, cfv, hc, sd + (int64_t)nd.aux * sd_stride, sd_n[nd.aux], lds);
}

// ------------------------------------------------------------ terminal-fused backward
// A decision node whose children include fold or showdown nodes, swept by
// one workgroup over all its hands: the terminal children are evaluated into
// LDS (the same arithmetic as k_terminal, from the reach rows the forward
// sweep wrote), then the node's backward work reads them there instead of a
// round trip of their value rows through memory.  At most two such children
// per node (a fold and a showdown).  val: LDS [2][2][Hp] after the terminal
// scratch.
template <typename T, int A>
__device__ void tf_node(const DNode& nd, const DNode* __restrict__ nodes, int Hp, T* __restrict__ R,
                        T* __restrict__ S, T* __restrict__ Mp, const T* __restrict__ reach, T* __restrict__ cfv,
                        const IterState* __restrict__ st, const uint16_t* __restrict__ hcards,
                        const int32_t* __restrict__ coff, const int16_t* __restrict__ chands, int chand_stride,
                        const int16_t* __restrict__ sd, int64_t sd_stride, const int32_t* __restrict__ sd_n,
                        T* __restrict__ root_dst, int upd, const int32_t* __restrict__ nzs, T* lds, T* val) {
    const bool dead = node_dead(nzs, nd);
    const T* tv[A];
#pragma unroll
    for (int a = 0; a < A; a++) tv[a] = nullptr;
    if (!dead) {
        int k = 0;
        for (int a = 0; a < A; a++) {
            const DNode ch = nodes[nd.first_child + a];
            if (ch.type != PCFR_NODE_FOLD && ch.type != PCFR_NODE_SHOWDOWN) continue;
            if (k) __syncthreads();   // the previous evaluation's LDS scratch is consumed
            T* out = val + (int64_t)k * 2 * Hp;
            const T* r0 = reach + (int64_t)ch.slot[0] * Hp;
            const T* r1 = reach + (int64_t)ch.slot[1] * Hp;
            T xa[kHandIt], xb[kHandIt];
#pragma unroll
            for (int i = 0; i < kHandIt; i++) {
                const int h = threadIdx.x + i * kBlock;
                if (h < Hp) { xa[i] = r0[h]; xb[i] = r1[h]; }
            }
            const uint16_t* hc = hcards + (int64_t)ch.sub * Hp;
            if (ch.type == PCFR_NODE_FOLD)
                term_fold_core<T>(ch, Hp, xa, xb, hc, coff + ch.sub * 53, chands + (int64_t)ch.sub * chand_stride, lds,
                                  out, out + Hp);
            else
                term_showdown_core<T>(ch, Hp, xa, xb, sd + (int64_t)ch.aux * sd_stride, sd_n[ch.aux], lds, out,
                                      out + Hp);
            tv[a] = out;
            k++;
        }
        __syncthreads();   // every terminal value visible to every thread
    }
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = threadIdx.x + i * kBlock;
        if (h < Hp)
            bwd_decision<T, MODE_ITER, A, 1, false, true>(nd, nd.id, h, Hp, R, S, Mp, reach, cfv, st, hcards, root_dst,
                                                          upd, dead, tv);
    }
}

template <typename T, int MAXA>
__global__ __launch_bounds__(kBlock) void k_backward_tf(const DNode* __restrict__ rec, const DNode* __restrict__ nodes,
                                                        int Hp, T* __restrict__ R, T* __restrict__ S,
                                                        T* __restrict__ Mp, const T* __restrict__ reach,
                                                        T* __restrict__ cfv, const IterState* __restrict__ st,
                                                        const uint16_t* __restrict__ hcards,
                                                        const int32_t* __restrict__ coff,
                                                        const int16_t* __restrict__ chands, int chand_stride,
                                                        const int16_t* __restrict__ sd, int64_t sd_stride,
                                                        const int32_t* __restrict__ sd_n, T* __restrict__ root_dst,
                                                        int upd, const int32_t* __restrict__ nzs, int val_off) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    T* val = reinterpret_cast<T*>(smem + val_off);
    const DNode nd = rec[blockIdx.x];
    switch (nd.n_child) {
#define PCFR_TF_CASE(A) \
    case A:             \
        if constexpr (A <= MAXA) tf_node<T, A>(nd, nodes, Hp, R, S, Mp, reach, cfv, st, hcards, coff, chands, chand_stride, sd, sd_stride, sd_n, root_dst, upd, nzs, lds, val); \
        break;
        PCFR_TF_CASE(1) PCFR_TF_CASE(2) PCFR_TF_CASE(3) PCFR_TF_CASE(4) PCFR_TF_CASE(5) PCFR_TF_CASE(6)
        PCFR_TF_CASE(7) PCFR_TF_CASE(8) PCFR_TF_CASE(9) PCFR_TF_CASE(10) PCFR_TF_CASE(11) PCFR_TF_CASE(12)
#undef PCFR_TF_CASE
        default: break;
    }
}

// ------------------------------------------------------------ persistent launch
// Every phase of an iteration in one resident grid: the level sweeps stride
// over the level's (node, 4-hand) work items, the terminals over their
// nodes one workgroup at a time, and a grid barrier separates the phases
// (each level needs the level above it, resp. below it, complete).  The
// grid is launched cooperatively, so all its workgroups are resident, and
// runs `iters` iterations before it exits.  Every workgroup takes every
// barrier: the loop bounds come from the same device arrays for all, and no
// workgroup leaves the loops early.  The per-node arithmetic is that of the
// per-level kernels, so the iterates are bitwise those of the graph of
// launches.  For forests of subgames played to showdown (no depth-limit
// leaves), simultaneous updates, no suit isomorphism.
// hands per work item of the persistent sweeps (4, as the per-level kernels;
// 2 hands with twice the resident workgroups measured slower: 4.19 against
// 3.60 ms per iteration of the 256-subgame forest)
constexpr int kPersistNH = 4;

struct PersistArgs {
    const DNode* nodes;
    const DNode* dec_rec;
    const DNode* fwd_rec;
    const int64_t* dec_off;
    const int64_t* fwd_off;
    const int32_t* term;
    const uint16_t* hcards;
    const int32_t* coff;
    const int16_t* chands;
    const int16_t* sd;
    const int32_t* sdn;
    void *R, *S, *Mp, *reach, *cfv, *root;
    IterState* st;
    int32_t* nzs;                 // pruning flags (null: no pruning)
    int64_t sd_stride;
    int32_t levels, Hp, cbase, n_term, chand_stride, iters, n_slots;
};

template <typename T, int MAXA>
__global__ __launch_bounds__(kBlock) void k_iterate_persistent(PersistArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    T* R = static_cast<T*>(a.R);
    T* S = static_cast<T*>(a.S);
    T* Mp = static_cast<T*>(a.Mp);
    T* reach = static_cast<T*>(a.reach);
    T* cfv = static_cast<T*>(a.cfv);
    T* root = static_cast<T*>(a.root);
    const int Hp = a.Hp, groups = Hp / kPersistNH;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const IsoTabs no_iso = {nullptr, nullptr};
    for (int it = 0; it < a.iters; it++) {
        // t, the Stage-7 coefficients and the threshold, and cleared pruning
        // flags of the action slots (the roots' stay set), before the forward
        if (blockIdx.x == 0 && threadIdx.x == 0) begin_iteration(a.st);
        if (a.nzs)
            for (int64_t i = a.cbase + gtid; i < a.n_slots; i += nthreads) a.nzs[i] = 0;
        grid.sync();
        for (int l = 0; l < a.levels; l++) {
            const int64_t b = a.dec_off[l], cnt = a.dec_off[l + 1] - b;
            if (cnt == 0) continue;
            for (int64_t i = gtid; i < cnt * groups; i += nthreads) {
                const int64_t k = i / groups;
                fwd_node<T, MODE_ITER, MAXA, kPersistNH>(a.dec_rec[b + k], (int)(i - k * groups) * kPersistNH, Hp,
                                                         a.cbase, R, S, Mp, reach, a.st, a.nzs, true);
            }
            grid.sync();
        }
        for (int w = blockIdx.x; w < a.n_term; w += gridDim.x) {
            __syncthreads();   // the previous node's LDS is consumed
            const int64_t n = a.term[w];
            const DNode nd = a.nodes[n];
            if (node_dead(a.nzs, nd)) {
                T* v = cfv + n * 2 * Hp;
                for (int i = threadIdx.x; i < 2 * Hp; i += blockDim.x) v[i] = T(0);
                continue;
            }
            const uint16_t* hc = a.hcards + (int64_t)nd.sub * Hp;
            if (nd.type == PCFR_NODE_FOLD)
                term_fold<T>(nd, n, Hp, reach, cfv, hc, a.coff + nd.sub * 53, a.chands + (int64_t)nd.sub * a.chand_stride,
                             lds);
            else
                term_showdown<T>(nd, n, Hp, reach, cfv, hc, a.sd + (int64_t)nd.aux * a.sd_stride, a.sdn[nd.aux], lds);
        }
        grid.sync();
        for (int l = a.levels - 1; l >= 0; l--) {
            const int64_t b = a.fwd_off[l], cnt = a.fwd_off[l + 1] - b;
            if (cnt == 0) continue;
            for (int64_t i = gtid; i < cnt * groups; i += nthreads) {
                const int64_t k = i / groups;
                bwd_node<T, MODE_ITER, MAXA, kPersistNH, false>(a.fwd_rec[b + k], (int)(i - k * groups) * kPersistNH, Hp,
                                                                R, S, Mp, reach, cfv, a.st, a.hcards,
                                                                l == 0 ? root : nullptr, -1, no_iso, a.nzs);
            }
            grid.sync();
        }
    }
}

// ------------------------------------------------------------ depth-limit leaves
// Exact leaf values from pairwise check-down equity (all-in leaves, and every
// leaf when no network is attached): v_i(h) = c * sum_o E(h,o) r_{-i}(o).
// Et is stored transposed, [o][h], so consecutive threads read consecutive h.
// The sum over o is split into kEqSplit slices, each slice of a group of up
// to J leaves of one subgame (so one table, [n_et][Hp][Hp]) one workgroup
// with the slice of their reach vectors in LDS; a second kernel adds the
// slices in a fixed order (deterministic) and applies the contribution.
constexpr int kEqSplit = 32;

template <typename T, int J>
__global__ __launch_bounds__(kBlock) void k_equity_partial(const DNode* __restrict__ nodes,
                                                           const int32_t* __restrict__ leaves, int n_leaves, int Hp,
                                                           const int4* __restrict__ groups,
                                                           const T* __restrict__ Et, const T* __restrict__ reach,
                                                           T* __restrict__ part) {
    constexpr int kChunk = (kMaxHp + kEqSplit - 1) / kEqSplit;
    __shared__ T rr[J][2][kChunk];
    const int4 gr = groups[blockIdx.y];    // first leaf, count (<= J), equity table
    const int j0 = gr.x;
    const int nj = gr.y;
    Et += (int64_t)gr.z * Hp * Hp;
    const int chunk = (Hp + kEqSplit - 1) / kEqSplit;
    const int o0 = blockIdx.z * chunk, o1 = min(Hp, o0 + chunk);
    for (int i = threadIdx.x; i < nj * 2 * chunk; i += kBlock) {
        const int j = i / (2 * chunk), rest = i - j * 2 * chunk, p = rest / chunk, o = o0 + rest - p * chunk;
        const DNode& lf = nodes[leaves[j0 + j]];
        rr[j][p][o - o0] = o < o1 ? reach[(int64_t)(p ? lf.slot[1] : lf.slot[0]) * Hp + o] : T(0);
    }
    __syncthreads();
    const int h = blockIdx.x * kBlock + threadIdx.x;
    if (h >= Hp) return;
    T acc[J][2];
#pragma unroll
    for (int j = 0; j < J; j++) { acc[j][0] = T(0); acc[j][1] = T(0); }
    // 8 rows of Et in flight at a time; the sums still run in row order
    constexpr int G = 8;
    for (int ob = o0; ob < o1; ob += G) {
        T e[G];
#pragma unroll
        for (int q = 0; q < G; q++) e[q] = ob + q < o1 ? Et[(int64_t)(ob + q) * Hp + h] : T(0);
#pragma unroll
        for (int q = 0; q < G; q++) {
            if (ob + q >= o1) break;
#pragma unroll
            for (int j = 0; j < J; j++) {
                acc[j][0] += e[q] * rr[j][1][ob + q - o0];   // player 0 against player 1's reach
                acc[j][1] += e[q] * rr[j][0][ob + q - o0];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < J; j++) {
        if (j >= nj) break;
        T* dst = part + (((int64_t)blockIdx.z * n_leaves + j0 + j) * 2) * Hp + h;
        dst[0] = acc[j][0];
        dst[Hp] = acc[j][1];
    }
}

template <typename T>
__global__ void k_equity_reduce(const int32_t* __restrict__ leaves, const double* __restrict__ pay, int n_leaves,
                                int Hp, const T* __restrict__ part, T* __restrict__ cfv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = 2 * (int64_t)Hp;
    if (i >= per * n_leaves) return;
    const int64_t j = i / per, rest = i - j * per;
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < kEqSplit; k++) acc += part[((int64_t)k * n_leaves + j) * per + rest];
    cfv[(int64_t)leaves[j] * per + rest] = (T)pay[j] * acc;
}

__device__ __forceinline__ int combo_index(int a, int b) {
    const int hi = a > b ? a : b, lo = a > b ? b : a;
    return hi * (hi - 1) / 2 + lo;
}

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Stage a leaf's reach (both players) in LDS x[2][kMaxHp]; per-card sums of
// each player in cs[2][52] and the totals, all in A (the accumulation type).
template <typename T, typename A>
__device__ __forceinline__ void stage_leaf(const T* __restrict__ r0, const T* __restrict__ r1, int Hp,
                                           const int32_t* __restrict__ coff, const int16_t* __restrict__ chands,
                                           T (*x)[kMaxHp], A (*cs)[52], A* xch, A& t0, A& t1) {
    const int tid = threadIdx.x;
    T a[kHandIt], b[kHandIt];
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        if (h < Hp) { a[i] = r0[h]; b[i] = r1[h]; }
    }
    t0 = A(0);
    t1 = A(0);
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        if (h < Hp) { x[0][h] = a[i]; x[1][h] = b[i]; t0 += (A)a[i]; t1 += (A)b[i]; }
    }
    __syncthreads();
    if (tid < 104) {
        const int p = tid / 52, c = tid - p * 52;
        A acc = A(0);
        for (int j = coff[c]; j < coff[c + 1]; j++) acc += (A)x[p][chands[j]];
        cs[p][c] = acc;
    }
    block_sum2(t0, t1, xch);      // synchronises: cs is visible after it
}

// Per-leaf reach aggregates shared by the zero-sum and combine kernels:
// agg[leaf] = [2][53], each player's 52 per-card sums (reach of the hands
// holding the card) then the total; written by k_leaf_input (group 0).
constexpr int kAgg = 106;

// Stage 2's batched leaf input (Sec. 4.2) for Stage 5's network (Sec. 4.3):
// one row per (leaf, next card c): each player's reach with the hands
// holding c removed, normalised to sum 1, over the 1326 combos; then the
// board after c as 52 one-hot entries; then the stack-to-pot ratio at the
// leaf; bf16, zero padded to ldx.
//
// One workgroup per (leaf, group of next cards).  Each rebuilds the leaf's
// dense combo-indexed ranges in LDS, the per-card sums C_p(c) and, per card,
// the reciprocal of S_p(c) = total - C_p(c), the reach of the hands without c
// (zero when nothing is left) -- the same sums in the same order in every
// group -- then writes its cards' rows, 8 consecutive columns per step (one
// 16-byte store).  Normalised entries are formed in double and rounded once
// to float, as r / S would be.  Group 0 also stores the ranges (Rc) and the
// aggregates (agg) read by the zero-sum and combine kernels.
constexpr int kComboPad = 1344;           // 1326 combos padded to 64
template <typename T>
__global__ __launch_bounds__(kBlock) void k_leaf_input(const DNode* __restrict__ nodes,
                                                       const int32_t* __restrict__ leaves, int Hp,
                                                       const T* __restrict__ reach,
                                                       const int16_t* __restrict__ combo_hand /* [n_sub][kComboPad] */,
                                                       T* __restrict__ Rc, T* __restrict__ agg,
                                                       const float* __restrict__ spr, int n_next, int cards_per_group,
                                                       const int8_t* __restrict__ next_cards /* [n_sub][64] */,
                                                       const int4* __restrict__ boards /* [n_sub] */, int ldx,
                                                       uint16_t* __restrict__ X) {
    constexpr int RI = (2 * kComboPad + kBlock - 1) / kBlock;
    __shared__ T x[2][kMaxHp];
    __shared__ double xc[2][kComboPad];
    __shared__ double sv[2][52];
    __shared__ double dxch[2 * kWaves], nxch[2 * kWaves];
    const int li = blockIdx.x, tid = threadIdx.x;
    const bool lead = blockIdx.y == 0;
    const DNode nd = nodes[leaves[li]];
    const T* r0 = reach + (int64_t)nd.slot[0] * Hp;
    const T* r1 = reach + (int64_t)nd.slot[1] * Hp;
    combo_hand += (int64_t)nd.sub * kComboPad;
    // every load of the thread first: its hands' reach and its combos' hands
    T a[kHandIt], b[kHandIt];
    int hk[RI];
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        a[i] = h < Hp ? r0[h] : T(0);
        b[i] = h < Hp ? r1[h] : T(0);
    }
#pragma unroll
    for (int i = 0; i < RI; i++) {
        const int k = tid + i * kBlock, kk = k >= kComboPad ? k - kComboPad : k;
        hk[i] = (k < 2 * kComboPad && kk < kCombos) ? combo_hand[kk] : -1;
    }
#pragma unroll
    for (int i = 0; i < kHandIt; i++) {
        const int h = tid + i * kBlock;
        if (h < Hp) { x[0][h] = a[i]; x[1][h] = b[i]; }
    }
    __syncthreads();
    // dense combo-indexed ranges (to LDS for the rows and sums, and from
    // group 0 to memory for the zero-sum and combine kernels)
    T* rc = Rc + (int64_t)li * 2 * kComboPad;
    double t0 = 0.0, t1 = 0.0, n0 = 0.0, n1 = 0.0;   // totals and counts of combos with reach
#pragma unroll
    for (int i = 0; i < RI; i++) {
        const int k = tid + i * kBlock;
        if (k < 2 * kComboPad) {
            const int p = k >= kComboPad, kk = k - p * kComboPad;
            const T v = hk[i] >= 0 ? x[p][hk[i]] : T(0);
            if (lead) rc[k] = v;
            xc[p][kk] = (double)v;
            if (p) { t1 += (double)v; n1 += v != T(0) ? 1.0 : 0.0; }
            else { t0 += (double)v; n0 += v != T(0) ? 1.0 : 0.0; }
        }
    }
    block_sum2(t0, t1, dxch);      // synchronises: xc is visible after it
    block_sum2(n0, n1, nxch);
    if (tid < 104) {
        // per-card sums over the 51 combos holding the card, then 1/S for each card
        const int p = tid / 52, c = tid - p * 52;
        double cs = 0.0, nc = 0.0;
#pragma unroll
        for (int xi = 0; xi < 51; xi++) {
            const double v = xc[p][combo_index(c, xi < c ? xi : xi + 1)];
            cs += v;
            nc += v != 0.0 ? 1.0 : 0.0;
        }
        if (lead) agg[(int64_t)li * kAgg + p * 53 + c] = (T)cs;
        // The row is empty exactly when no combo without c has reach (an
        // integer count, as the plain sum's test for zero); otherwise S is
        // total - C(c), or, where that difference has cancelled below 1e-6
        // of the total, the direct sum of the combos without c.
        const double tot = p ? t1 : t0, left = (p ? n1 : n0) - nc;
        double rest = tot - cs;
        if (left > 0.0 && !(rest > 1e-6 * tot)) {
            rest = 0.0;
            int k = 0;
            for (int a = 1; a < 52; a++)
                for (int b = 0; b < a; b++, k++)
                    if (a != c && b != c) rest += xc[p][k];
        }
        sv[p][c] = left > 0.0 && rest > 0.0 ? 1.0 / rest : 0.0;
    }
    if (lead && tid == 0) { agg[(int64_t)li * kAgg + 52] = (T)t0; agg[(int64_t)li * kAgg + 105] = (T)t1; }
    __syncthreads();
    const int4 board = boards[nd.sub];
    const float ratio = spr[li];
    const int8_t* nc = next_cards + nd.sub * 64;
    const int k0 = blockIdx.y * cards_per_group, k1 = min(n_next, k0 + cards_per_group);
    const int chunks = ldx / 8;
    for (int it = tid; it < (k1 - k0) * chunks; it += kBlock) {
        const int q = it / chunks, ci = k0 + q, col0 = (it - q * chunks) * 8;
        const int c = nc[ci];
        const double s0 = sv[0][c], s1 = sv[1][c];
        // cards (a > b) of the combo in column col0 of its player's block
        int k = col0 >= kCombos ? col0 - kCombos : col0;
        if (k >= kCombos) k = 0;            // past both blocks: unused
        int ca = (int)((1.f + sqrtf(1.f + 8.f * (float)k)) * 0.5f);
        if (ca * (ca - 1) / 2 > k) ca--;
        else if ((ca + 1) * ca / 2 <= k) ca++;
        int cb = k - ca * (ca - 1) / 2;
        uint16_t v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int col = col0 + j;
            float xv = 0.f;
            if (col < 2 * kCombos) {
                if (col == kCombos) { ca = 1; cb = 0; }      // player 1's block restarts at combo 0
                const int pp = col >= kCombos;
                if (ca != c && cb != c) xv = (float)(xc[pp][col - pp * kCombos] * (pp ? s1 : s0));
                if (++cb == ca) { ca++; cb = 0; }
            } else if (col < 2 * kCombos + 52) {
                const int card = col - 2 * kCombos;
                xv = (card == c || card == board.x || card == board.y || card == board.z || card == board.w) ? 1.f : 0.f;
            } else if (col == 2 * kCombos + 52) {
                xv = ratio;
            }
            v[j] = to_bf16(xv);
        }
        *reinterpret_cast<u32x4*>(X + ((int64_t)li * n_next + ci) * ldx + col0) =
            u32x4{(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                  (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16)};
    }
}

// Zero-sum correction of the network's outputs (a reading: the paper does not
// say how leaf values are kept consistent).  For one row (leaf, next card c)
// the values pot * EV_i(h | c) weighted by own reach and by the opponent's
// compatible reach M_{-i}(h | c) should sum to zero over both players, as the
// solved targets do; the kernel finds the shift d = e / (2 z) with
// e = sum_h r0 M1 EV0 + sum_h r1 M0 EV1 and z = sum_h r0 M1 (= sum_h r1 M0),
// which the combine subtracts from both players' EVs of that row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_leaf_zerosum(int n_next, const int32_t* __restrict__ leaf_sub,
                                                         const int8_t* __restrict__ next_cards /* [n_sub][64] */,
                                                         const T* __restrict__ Rc, const T* __restrict__ agg,
                                                         const float* __restrict__ Y, int ldy, T* __restrict__ delta) {
    constexpr int CI = (kCombos + kBlock - 1) / kBlock;
    __shared__ T rs[2][kComboPad];
    __shared__ T ag[kAgg];
    __shared__ T xch[2 * kWaves];
    const int row = blockIdx.x, li = row / n_next, kc = row - li * n_next;
    const int c = next_cards[leaf_sub[li] * 64 + kc];
    const int tid = threadIdx.x;
    // every global load first: the leaf's combo-indexed ranges, aggregates and this row's outputs
    const T* rc = Rc + (int64_t)li * 2 * kComboPad;
    T rv[2][CI];
    float y0[CI], y1[CI];
    const float* y = Y + (int64_t)row * ldy;
#pragma unroll
    for (int i = 0; i < CI; i++) {
        const int k = tid + i * kBlock, kk = k < kCombos ? k : 0;
        rv[0][i] = rc[kk];
        rv[1][i] = rc[kComboPad + kk];
        y0[i] = y[kk];
        y1[i] = y[kCombos + kk];
    }
    const T agv = tid < kAgg ? agg[(int64_t)li * kAgg + tid] : T(0);
#pragma unroll
    for (int i = 0; i < CI; i++) {
        const int k = tid + i * kBlock;
        if (k < kCombos) { rs[0][k] = rv[0][i]; rs[1][k] = rv[1][i]; }
    }
    if (tid < kAgg) ag[tid] = agv;
    __syncthreads();
    const T s0 = ag[52] - ag[c], s1 = ag[105] - ag[53 + c];     // totals without the hands holding c
    T e = T(0), z = T(0);
#pragma unroll
    for (int i = 0; i < CI; i++) {
        const int k = tid + i * kBlock;
        if (k >= kCombos) continue;
        int a = (int)((1.f + sqrtf(1.f + 8.f * (float)k)) * 0.5f);
        if (a * (a - 1) / 2 > k) a--;
        else if ((a + 1) * a / 2 <= k) a++;
        const int b = k - a * (a - 1) / 2;
        if (a == c || b == c) continue;
        const int ka = combo_index(a, c), kb = combo_index(b, c);
        const T x0 = rs[0][k], x1 = rs[1][k];
        // blocked combos carry zero range, so they add nothing here
        const T m1 = s1 - ag[53 + a] - ag[53 + b] + x1 + rs[1][ka] + rs[1][kb];
        const T m0 = s0 - ag[a] - ag[b] + x0 + rs[0][ka] + rs[0][kb];
        e += x0 * m1 * (T)y0[i] + x1 * m0 * (T)y1[i];
        z += x0 * m1;
    }
    block_sum2(e, z, xch);
    if (tid == 0) delta[row] = z > T(0) ? e / (T(2) * z) : T(0);
}

// Leaf counterfactual values from the network's per-card outputs (Sec. 4.4:
// leaf predictions weighted by the opponent's counterfactual reach and the
// chance probability): v_i(h) = pot/K * sum_{c not in h} EV_i(h | c) *
// M_{-i}(h | c), where M(h | c) is the opponent reach over hands sharing no
// card with h or c:  T - C[a] - C[b] - C[c] + r(ab) + r(ac) + r(bc).
// One workgroup per (leaf, tile of 64 hands); its 4 waves take every 4th
// next card and the partial sums are added in a fixed order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_leaf_combine(const DNode* __restrict__ nodes,
                                                         const int32_t* __restrict__ leaves,
                                                         const double* __restrict__ pot_over_k, int n_next,
                                                         const int8_t* __restrict__ next_cards /* [n_sub][64] */,
                                                         int Hp, int H,
                                                         const T* __restrict__ reach, T* __restrict__ cfv,
                                                         const uint16_t* __restrict__ hcards /* [n_sub][Hp] */,
                                                         const int16_t* __restrict__ hand_combo /* [n_sub][Hp] */,
                                                         const int16_t* __restrict__ combo_hand /* [n_sub][kComboPad] */,
                                                         const float* __restrict__ Y, int ldy,
                                                         const T* __restrict__ agg, const T* __restrict__ delta) {
    __shared__ T x[2][kMaxHp];
    __shared__ __align__(16) int16_t c2h[kCombos];
    __shared__ int8_t nxt[52];
    __shared__ T dl[52];
    __shared__ T cs[2][52];
    __shared__ T red[2][kBlock];
    const int li = blockIdx.x;
    const int64_t n = leaves[li];
    const DNode nd = nodes[n];
    const T* r0 = reach + (int64_t)nd.slot[0] * Hp;
    const T* r1 = reach + (int64_t)nd.slot[1] * Hp;
    hcards += (int64_t)nd.sub * Hp;
    hand_combo += (int64_t)nd.sub * Hp;
    combo_hand += (int64_t)nd.sub * kComboPad;   // 16-byte aligned rows for copy_i16
    next_cards += nd.sub * 64;
    const int tid = threadIdx.x;
    {
        T a[kHandIt], b[kHandIt];
#pragma unroll
        for (int i = 0; i < kHandIt; i++) {
            const int h = tid + i * kBlock;
            if (h < Hp) { a[i] = r0[h]; b[i] = r1[h]; }
        }
#pragma unroll
        for (int i = 0; i < kHandIt; i++) {
            const int h = tid + i * kBlock;
            if (h < Hp) { x[0][h] = a[i]; x[1][h] = b[i]; }
        }
    }
    copy_i16<(kCombos + 7) / 8 / kBlock + 1>(c2h, combo_hand, kCombos / 8 * 8);
    if (tid < kCombos - kCombos / 8 * 8) c2h[kCombos / 8 * 8 + tid] = combo_hand[kCombos / 8 * 8 + tid];
    if (tid < n_next) {
        nxt[tid] = next_cards[tid];
        dl[tid] = delta ? delta[li * n_next + tid] : T(0);
    }
    const T* ag = agg + (int64_t)li * kAgg;
    if (tid < 104) cs[tid / 52][tid % 52] = ag[(tid / 52) * 53 + tid % 52];
    const T t0 = ag[52], t1 = ag[105];
    __syncthreads();
    __syncthreads();   // red is reused for the partial sums below
    const int lane = tid & 63, grp = tid >> 6;
    const int h = blockIdx.y * 64 + lane;
    T acc0 = T(0), acc1 = T(0);
    const bool live = h < H;
    int a = 0, b = 0, combo = 0;
    T base0 = T(0), base1 = T(0);
    if (live) {
        const uint32_t hc = hcards[h];
        a = hc & 0xff;
        b = hc >> 8;
        combo = hand_combo[h];
        // every output load of this hand first (next cards grp, grp + 4, ...)
        constexpr int KI = (52 + 3) / 4;
        float ya[KI], yb[KI];
        const float* y = Y + (int64_t)li * n_next * ldy;
#pragma unroll
        for (int i = 0; i < KI; i++) {
            const int k = grp + 4 * i, kk = k < n_next ? k : 0;
            ya[i] = y[(int64_t)kk * ldy + combo];
            yb[i] = y[(int64_t)kk * ldy + kCombos + combo];
        }
        base0 = t0 - cs[0][a] - cs[0][b] + x[0][h];
        base1 = t1 - cs[1][a] - cs[1][b] + x[1][h];
#pragma unroll
        for (int i = 0; i < KI; i++) {
            const int k = grp + 4 * i;
            if (k >= n_next) break;
            const int c = nxt[k];
            if (c == a || c == b) continue;
            const int ha = c2h[combo_index(a, c)], hb = c2h[combo_index(b, c)];
            const T m1 = base1 - cs[1][c] + (ha >= 0 ? x[1][ha] : T(0)) + (hb >= 0 ? x[1][hb] : T(0));
            const T m0 = base0 - cs[0][c] + (ha >= 0 ? x[0][ha] : T(0)) + (hb >= 0 ? x[0][hb] : T(0));
            acc0 += ((T)ya[i] - dl[k]) * m1;
            acc1 += ((T)yb[i] - dl[k]) * m0;
        }
    }
    red[0][tid] = acc0;
    red[1][tid] = acc1;
    __syncthreads();
    if (grp == 0 && h < Hp) {
        T* v0 = cfv + n * 2 * Hp;
        T* v1 = v0 + Hp;
        if (!live) { v0[h] = T(0); v1[h] = T(0); return; }
        const T scale = (T)pot_over_k[li];
        const T f0 = ((red[0][lane] + red[0][64 + lane]) + red[0][128 + lane]) + red[0][192 + lane];
        const T f1 = ((red[1][lane] + red[1][64 + lane]) + red[1][128 + lane]) + red[1][192 + lane];
        v0[h] = scale * f0;
        v1[h] = scale * f1;
    }
}

// ------------------------------------------------------------ preflop roots
// A preflop root (no board) is solved over the 169 hand classes -- pairs,
// suited and offsuit rank pairs.  Its root ranges are suit-symmetric (equal
// on the combos of each class), so every iterate is too (a suit permutation
// maps the game onto itself; the lossless suit abstraction of Sec. 4.5): one
// "hand" per class carries the reach, regrets and values that each of its
// combos has.  Its leaves sit at the flop deal, where the flop-level network
// (Sec. 4.3) is queried on the canonical flops only.

// Fold over classes: M_{-i}(c) = sum_{c'} N[c][c'] r_{-i}(c'), with N[c][c']
// the number of combos of class c' sharing no card with a combo of class c
// (the same for every combo of c); the folder loses its contribution times
// M, the other player wins it.  One workgroup per fold node, one class per
// thread; sums of nonnegative terms in a fixed order, so zero mass is an
// exact zero.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fold_class(const DNode* __restrict__ nodes, const int32_t* __restrict__ folds,
                                                       int Hp, int Hc, const T* __restrict__ reach, T* __restrict__ cfv,
                                                       const uint8_t* __restrict__ ncompat /* [Hc][Hc] */,
                                                       const int32_t* __restrict__ nzs) {
    __shared__ T x[2][kBlock];
    const int64_t n = folds[blockIdx.x];
    const DNode nd = nodes[n];
    const int tid = threadIdx.x;
    T* v0 = cfv + n * 2 * Hp;
    T* v1 = v0 + Hp;
    if (node_dead(nzs, nd)) {
        for (int h = tid; h < Hp; h += kBlock) { v0[h] = T(0); v1[h] = T(0); }
        return;
    }
    const T* r0 = reach + (int64_t)nd.slot[0] * Hp;
    const T* r1 = reach + (int64_t)nd.slot[1] * Hp;
    if (tid < Hc) { x[0][tid] = r0[tid]; x[1][tid] = r1[tid]; }
    __syncthreads();
    const T pay = (T)nd.pay, s0 = nd.player == 0 ? -pay : pay;
    for (int c = tid; c < Hp; c += kBlock) {
        T m1 = T(0), m0 = T(0);
        if (c < Hc) {
            const uint8_t* row = ncompat + (int64_t)c * Hc;
            for (int j = 0; j < Hc; j++) {
                const T w = (T)row[j];
                m1 += w * x[1][j];
                m0 += w * x[0][j];
            }
        }
        v0[c] = s0 * m1;
        v1[c] = -s0 * m0;
    }
}

__device__ __forceinline__ void combo_cards(int k, int& a, int& b) {
    a = (int)((1.f + sqrtf(1.f + 8.f * (float)k)) * 0.5f);
    if (a * (a - 1) / 2 > k) a--;
    else if ((a + 1) * a / 2 <= k) a++;
    b = k - a * (a - 1) / 2;
}

// Network rows of the preflop leaves: one per (leaf, canonical flop f):
// each player's per-combo reach with the combos holding a flop card removed,
// normalised to sum 1 (zero if nothing is left), the flop's cards one-hot,
// the stack-to-pot ratio; bf16, zero padded to ldx.  One workgroup per
// (leaf, group of flops); each row's sums are direct sums in double over the
// kept combos.  Group 0 also stores the leaf's combo-indexed reach (Rc) and
// its per-card sums and totals (agg) for the zero-sum and combine kernels.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flop_leaf_input(const DNode* __restrict__ nodes,
                                                            const int32_t* __restrict__ leaves, int Hp,
                                                            const T* __restrict__ reach,
                                                            const int16_t* __restrict__ combo_hand /* [n_sub][kComboPad] */,
                                                            T* __restrict__ Rc, T* __restrict__ agg,
                                                            const float* __restrict__ spr, int n_flops, int flops_per_group,
                                                            const int8_t* __restrict__ flops /* [n_flops][4] */, int ldx,
                                                            uint16_t* __restrict__ X) {
    constexpr int CI = (kCombos + kBlock - 1) / kBlock;
    __shared__ double xc[2][kComboPad];
    __shared__ double xch[2 * kWaves];
    __shared__ uint16_t kc[kComboPad];   // cards of each combo, lo | hi << 8
    const int li = blockIdx.x, tid = threadIdx.x;
    const bool lead = blockIdx.y == 0;
    const DNode nd = nodes[leaves[li]];
    const T* r0 = reach + (int64_t)nd.slot[0] * Hp;
    const T* r1 = reach + (int64_t)nd.slot[1] * Hp;
    combo_hand += (int64_t)nd.sub * kComboPad;
    T* rc = Rc + (int64_t)li * 2 * kComboPad;
    int ka[CI], kb[CI];
#pragma unroll
    for (int i = 0; i < CI; i++) {
        const int k = tid + i * kBlock;
        ka[i] = -1;
        kb[i] = -1;
        if (k < kCombos) {
            combo_cards(k, ka[i], kb[i]);
            kc[k] = (uint16_t)(kb[i] | (ka[i] << 8));
            const int h = combo_hand[k];
            const T v0 = h >= 0 ? r0[h] : T(0), v1 = h >= 0 ? r1[h] : T(0);
            xc[0][k] = (double)v0;
            xc[1][k] = (double)v1;
            if (lead) { rc[k] = v0; rc[kComboPad + k] = v1; }
        }
    }
    __syncthreads();
    if (lead) {
        if (tid < 104) {
            const int p = tid / 52, c = tid - p * 52;
            double cs = 0.0;
            for (int j = 0; j < 51; j++) cs += xc[p][combo_index(c, j < c ? j : j + 1)];
            agg[(int64_t)li * kAgg + p * 53 + c] = (T)cs;
        }
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int i = 0; i < CI; i++)
            if (ka[i] >= 0) { t0 += xc[0][tid + i * kBlock]; t1 += xc[1][tid + i * kBlock]; }
        block_sum2(t0, t1, xch);
        if (tid == 0) { agg[(int64_t)li * kAgg + 52] = (T)t0; agg[(int64_t)li * kAgg + 105] = (T)t1; }
        __syncthreads();   // xch is reused below
    }
    const float ratio = spr[li];
    const int chunks = ldx / 8;
    const int f0 = blockIdx.y * flops_per_group, f1 = min(n_flops, f0 + flops_per_group);
    // one wave per flop: its sums are wave reductions, no workgroup barrier
    const int lane = tid & 63;
    constexpr int CW = (kCombos + 63) / 64;
    for (int f = f0 + (tid >> 6); f < f1; f += kWaves) {
        const int x = flops[4 * f], y = flops[4 * f + 1], z = flops[4 * f + 2];
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 0; i < CW; i++) {
            const int k = lane + i * 64;
            if (k >= kCombos) break;
            const int a = kc[k] >> 8, b = kc[k] & 0xff;
            if (a == x || a == y || a == z || b == x || b == y || b == z) continue;
            s0 += xc[0][k];
            s1 += xc[1][k];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s0 += __shfl_xor(s0, o);
            s1 += __shfl_xor(s1, o);
        }
        const double i0 = s0 > 0.0 ? 1.0 / s0 : 0.0, i1 = s1 > 0.0 ? 1.0 / s1 : 0.0;
        uint16_t* xr = X + ((int64_t)li * n_flops + f) * ldx;
        for (int it = lane; it < chunks; it += 64) {
            const int col0 = it * 8;
            uint16_t v[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int col = col0 + j;
                float xv = 0.f;
                if (col < 2 * kCombos) {
                    const int pp = col >= kCombos, k = col - pp * kCombos;
                    const int a = kc[k] >> 8, b = kc[k] & 0xff;
                    if (a != x && a != y && a != z && b != x && b != y && b != z)
                        xv = (float)(xc[pp][k] * (pp ? i1 : i0));
                } else if (col < 2 * kCombos + 52) {
                    const int card = col - 2 * kCombos;
                    xv = (card == x || card == y || card == z) ? 1.f : 0.f;
                } else if (col == 2 * kCombos + 52) {
                    xv = ratio;
                }
                v[j] = to_bf16(xv);
            }
            *reinterpret_cast<u32x4*>(xr + col0) =
                u32x4{(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                      (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16)};
        }
    }
}

// M_p(h | f): player p's reach over the combos sharing no card with combo ab
// or flop xyz, by inclusion-exclusion over those five cards (a combo holds
// two cards, so the series stops at the pairs): T - sum of the five per-card
// sums + the reach of the ten combos they pair into (ab itself among them).
template <typename T>
__device__ __forceinline__ T flop_mass(const T* rs, const T* cs, T tot, int a, int b, int x, int y, int z) {
    return tot - cs[a] - cs[b] - cs[x] - cs[y] - cs[z] + rs[combo_index(a, b)] + rs[combo_index(a, x)] +
           rs[combo_index(a, y)] + rs[combo_index(a, z)] + rs[combo_index(b, x)] + rs[combo_index(b, y)] +
           rs[combo_index(b, z)] + rs[combo_index(x, y)] + rs[combo_index(x, z)] + rs[combo_index(y, z)];
}

// Preflop leaf values, first pass: one workgroup per (leaf, group of
// canonical flops) reads each flop's network row once, coalesced (thread t
// owns combos t, t + 256, ...).  Per row it forms M_{-i}(x | f) for its
// combos, the row's zero-sum shift d = e / (2 z) (as k_leaf_zerosum, with
// e = sum_x r0 M1 EV0 + r1 M0 EV1 and z = sum_x r0 M1 over the combos clear
// of the flop) when the correction is on, and adds orbit(f) x
// (EV_i(x | f) - d) M_{-i}(x | f) to its combos' sums, flop by flop.  At the
// end each hand's sum over its combos (in hlist order) goes to
// part[leaf][group][player][hand].  With suit-symmetric reach, the flops of
// f's orbit give f's sum with a class's combos permuted among themselves, so
// the canonical flops weighted by their orbits stand for all flops.
constexpr int kFlopsPerGroup = 8;   // canonical flops per workgroup of the first pass

template <typename T>
__global__ __launch_bounds__(kBlock) void k_flop_leaf_sums(const DNode* __restrict__ nodes,
                                                           const int32_t* __restrict__ leaves, int n_flops,
                                                           int flops_per_group, const int8_t* __restrict__ flops,
                                                           const int32_t* __restrict__ orbit,
                                                           const int32_t* __restrict__ hoff /* [n_sub][Hp + 1] */,
                                                           const int16_t* __restrict__ hlist /* [n_sub][kComboPad] */,
                                                           int Hp, int H, const float* __restrict__ Y, int ldy,
                                                           const T* __restrict__ Rc, const T* __restrict__ agg,
                                                           int zero_sum, T* __restrict__ part) {
    constexpr int CI = (kCombos + kBlock - 1) / kBlock;
    __shared__ T rs[2][kComboPad];
    __shared__ T cs[2][52];
    __shared__ T xch[2 * kWaves];
    const int li = blockIdx.x, grp = blockIdx.y, tid = threadIdx.x;
    const DNode nd = nodes[leaves[li]];
    const T* rc = Rc + (int64_t)li * 2 * kComboPad;
    for (int k = tid; k < kCombos; k += kBlock) { rs[0][k] = rc[k]; rs[1][k] = rc[kComboPad + k]; }
    if (tid < 104) cs[tid / 52][tid % 52] = agg[(int64_t)li * kAgg + (tid / 52) * 53 + tid % 52];
    const T t0 = agg[(int64_t)li * kAgg + 52], t1 = agg[(int64_t)li * kAgg + 105];
    int ka[CI], kb[CI];
    T acc0[CI], acc1[CI];
#pragma unroll
    for (int i = 0; i < CI; i++) {
        const int k = tid + i * kBlock;
        ka[i] = -1;
        kb[i] = -1;
        if (k < kCombos) combo_cards(k, ka[i], kb[i]);
        acc0[i] = T(0);
        acc1[i] = T(0);
    }
    __syncthreads();
    const int f0 = grp * flops_per_group, f1 = min(n_flops, f0 + flops_per_group);
    // the next flop's outputs are loaded while this flop's are used (the
    // barriers below order LDS only, so those loads stay in flight)
    float ny0[CI], ny1[CI];
    auto load_row = [&](int f) {
        const float* yr = Y + ((int64_t)li * n_flops + f) * ldy;
#pragma unroll
        for (int i = 0; i < CI; i++) {
            const int k = tid + i * kBlock, kk = k < kCombos ? k : 0;
            ny0[i] = yr[kk];
            ny1[i] = yr[kCombos + kk];
        }
    };
    if (f0 < f1) load_row(f0);
    for (int f = f0; f < f1; f++) {
        const int x = flops[4 * f], y = flops[4 * f + 1], z = flops[4 * f + 2];
        float cy0[CI], cy1[CI];
#pragma unroll
        for (int i = 0; i < CI; i++) { cy0[i] = ny0[i]; cy1[i] = ny1[i]; }
        if (f + 1 < f1) load_row(f + 1);
        T m0[CI], m1[CI], y0[CI], y1[CI];
        T e = T(0), zz = T(0);
#pragma unroll
        for (int i = 0; i < CI; i++) {
            const int a = ka[i], b = kb[i];
            const int k = tid + i * kBlock;
            const bool live = a >= 0 && a != x && a != y && a != z && b != x && b != y && b != z;
            y0[i] = live ? (T)cy0[i] : T(0);
            y1[i] = live ? (T)cy1[i] : T(0);
            m1[i] = live ? flop_mass(rs[1], cs[1], t1, a, b, x, y, z) : T(0);
            m0[i] = live ? flop_mass(rs[0], cs[0], t0, a, b, x, y, z) : T(0);
            if (live) {
                e += rs[0][k] * m1[i] * y0[i] + rs[1][k] * m0[i] * y1[i];
                zz += rs[0][k] * m1[i];
            }
        }
        T d = T(0);
        if (zero_sum) {
            // workgroup sums of e and z, the same order as block_sum2, with
            // barriers that wait for LDS traffic only
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                e += __shfl_xor(e, o);
                zz += __shfl_xor(zz, o);
            }
            if ((tid & 63) == 0) { xch[tid >> 6] = e; xch[kWaves + (tid >> 6)] = zz; }
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            e = T(0);
            zz = T(0);
#pragma unroll
            for (int w = 0; w < kWaves; w++) { e += xch[w]; zz += xch[kWaves + w]; }
            d = zz > T(0) ? e / (T(2) * zz) : T(0);
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");   // xch is rewritten by the next flop
        }
        const T w = (T)orbit[f];
#pragma unroll
        for (int i = 0; i < CI; i++) {
            acc0[i] += w * ((y0[i] - d) * m1[i]);
            acc1[i] += w * ((y1[i] - d) * m0[i]);
        }
    }
    // per-combo sums to LDS (the reach rows are no longer needed), then per hand
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CI; i++) {
        const int k = tid + i * kBlock;
        if (k < kCombos) { rs[0][k] = acc0[i]; rs[1][k] = acc1[i]; }
    }
    __syncthreads();
    const int32_t* ho = hoff + (int64_t)nd.sub * (Hp + 1);
    const int16_t* hl = hlist + (int64_t)nd.sub * kComboPad;
    T* out = part + ((int64_t)li * gridDim.y + grp) * 2 * Hp;
    for (int h = tid; h < Hp; h += kBlock) {
        T s0 = T(0), s1 = T(0);
        if (h < H)
            for (int j = ho[h]; j < ho[h + 1]; j++) { s0 += rs[0][hl[j]]; s1 += rs[1][hl[j]]; }
        out[h] = s0;
        out[Hp + h] = s1;
    }
}

// Second pass: v_i(h) = pot / C(48,3) / |h| x the sum over the groups, in
// group order; zero on padding hands.
// One workgroup per (leaf, 64 value entries); its 4 waves take every 4th
// group, eight loads in flight per step, and add their sums in wave order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flop_leaf_values(const int32_t* __restrict__ leaves,
                                                             const double* __restrict__ pot_over_k,
                                                             const DNode* __restrict__ nodes,
                                                             const int32_t* __restrict__ hoff, int n_groups, int Hp,
                                                             int H, const T* __restrict__ part, T* __restrict__ cfv) {
    static_assert(kWaves == 4, "the wave sums are added as four terms");
    __shared__ T red[kWaves][64];
    const int li = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = blockIdx.y * 64 + lane;           // entry (player, hand) of 2 * Hp
    const int64_t n = leaves[li];
    const DNode nd = nodes[n];
    const T* pp = part + (int64_t)li * n_groups * 2 * Hp + q;
    T acc = T(0);
    if (q < 2 * Hp) {
        int g = wv;
        for (; g + 7 * kWaves < n_groups; g += 8 * kWaves) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = pp[(int64_t)(g + u * kWaves) * 2 * Hp];
#pragma unroll
            for (int u = 0; u < 8; u++) acc += v[u];
        }
        for (; g < n_groups; g += kWaves) acc += pp[(int64_t)g * 2 * Hp];
    }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && q < 2 * Hp) {
        const T tot = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        const int h = q < Hp ? q : q - Hp;
        const int32_t* ho = hoff + (int64_t)nd.sub * (Hp + 1);
        cfv[n * 2 * Hp + q] = h < H ? (T)(pot_over_k[li] / (double)(ho[h + 1] - ho[h])) * tot : T(0);
    }
}

// ------------------------------------------------------------ leaf-network samples
// One training sample per subgame of a solved batch, in the leaf network's
// input/output layout: x = both root ranges normalised to sum 1 over the 1326
// combos, the board one-hot (52), the stack-to-pot ratio; y = each hand's
// root value under the average strategies per unit of pot and of compatible
// opponent reach, v_i(h) / (pot * M_{-i}(h)); mask = 1 where M > 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_samples(const int32_t* __restrict__ roots, const float* __restrict__ pot_spr,
                                                    const uint8_t* __restrict__ boards, int Hp,
                                                    const T* __restrict__ reach, const T* __restrict__ cfv,
                                                    const uint16_t* __restrict__ hcards,
                                                    const int16_t* __restrict__ combo_hand /* [n_sub][1326] */,
                                                    const int32_t* __restrict__ coff, const int16_t* __restrict__ chands,
                                                    int chand_stride, float* __restrict__ x, int ldx,
                                                    float* __restrict__ y, float* __restrict__ mask, int ldy) {
    __shared__ T cs[2][52];
    __shared__ double red[2][kBlock];
    const int g = blockIdx.x, tid = threadIdx.x;
    const int64_t n = roots[g];
    const T* r0 = reach + (int64_t)(2 * g) * Hp;
    const T* r1 = r0 + Hp;
    const T* v0 = cfv + n * 2 * Hp;
    const T* v1 = v0 + Hp;
    const uint16_t* hc = hcards + (int64_t)g * Hp;
    const int16_t* c2h = combo_hand + (int64_t)g * kCombos;
    if (tid < 104) {
        const int p = tid / 52, c = tid - p * 52;
        const T* r = p ? r1 : r0;
        const int32_t* co = coff + g * 53;
        const int16_t* ch = chands + (int64_t)g * chand_stride;
        T acc = T(0);
        for (int j = co[c]; j < co[c + 1]; j++) acc += r[ch[j]];
        cs[p][c] = acc;
    }
    double s0 = 0.0, s1 = 0.0;
    for (int h = tid; h < Hp; h += kBlock) { s0 += (double)r0[h]; s1 += (double)r1[h]; }
    red[0][tid] = s0;
    red[1][tid] = s1;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (tid < w) { red[0][tid] += red[0][tid + w]; red[1][tid] += red[1][tid + w]; }
        __syncthreads();
    }
    const double S0 = red[0][0], S1 = red[1][0];
    const float pot = pot_spr[2 * g], spr = pot_spr[2 * g + 1];
    float* xr = x + (int64_t)g * ldx;
    float* yr = y + (int64_t)g * ldy;
    float* mr = mask + (int64_t)g * ldy;
    for (int col = tid; col < ldx; col += kBlock) {
        float v = 0.f;
        if (col < 2 * kCombos) {
            const int p = col >= kCombos;
            const int h = c2h[col - p * kCombos];
            const double S = p ? S1 : S0;
            if (h >= 0 && S > 0.0) v = (float)((double)(p ? r1[h] : r0[h]) / S);
        } else if (col < 2 * kCombos + 52) {
            v = boards[(int64_t)g * 52 + (col - 2 * kCombos)] ? 1.f : 0.f;
        } else if (col == 2 * kCombos + 52) {
            v = spr;
        }
        xr[col] = v;
    }
    for (int col = tid; col < ldy; col += kBlock) {
        float t = 0.f, m = 0.f;
        if (col < 2 * kCombos) {
            const int p = col >= kCombos;
            const int h = c2h[col - p * kCombos];
            if (h >= 0) {
                const uint32_t c = hc[h];
                const int a = c & 0xff, b = c >> 8;
                const int o = 1 - p;
                const T* ro = o ? r1 : r0;
                const T tot = (T)(o ? S1 : S0);
                const T M = tot - cs[o][a] - cs[o][b] + ro[h];
                if (M > T(0)) {
                    t = (float)((p ? v1[h] : v0[h]) / ((T)pot * M));
                    m = 1.f;
                }
            }
        }
        yr[col] = t;
        mr[col] = m;
    }
}

// ------------------------------------------------------------ small kernels
__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_begin_iteration(IterState* st) { begin_iteration(st); }

// Strategy of one decision node for every hand: which 0 = average, 1 =
// current (regret matching, then the threshold of the next iteration).
template <typename T>
__global__ void k_strategy(const T* __restrict__ src, const T* __restrict__ pred, int rs, int A, int Hp, int which,
                           const IterState* __restrict__ st, T* __restrict__ out) {
    int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= Hp) return;
    T den = T(0);
    for (int a = 0; a < A; a++) {
        T x = src[(int64_t)(rs + a) * Hp + h] + (pred ? pred[(int64_t)(rs + a) * Hp + h] : T(0));
        den += which ? (x > T(0) ? x : T(0)) : x;
    }
    for (int a = 0; a < A; a++) {
        T x = src[(int64_t)(rs + a) * Hp + h] + (pred ? pred[(int64_t)(rs + a) * Hp + h] : T(0));
        out[(int64_t)a * Hp + h] = den > T(0) ? ((which && !(x > T(0))) ? T(0) : x / den) : T(1) / T(A);
    }
    const T thr = (which && st->thr0 > 0.0) ? (T)(st->thr0 / sqrt((double)(st->t + 1))) : T(0);
    if (thr > T(0)) {
        T keep = T(0);
        for (int a = 0; a < A; a++) {
            T& q = out[(int64_t)a * Hp + h];
            if (q < thr) q = T(0);
            keep += q;
        }
        for (int a = 0; a < A; a++) out[(int64_t)a * Hp + h] /= keep;
    }
}

// ------------------------------------------------------------ host runtime
static int32_t hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return PCFR_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PCFR_E_DEVICE;
}
#define HIPCHK(call)                                             \
    do {                                                         \
        int32_t _rc = hip_check((call), #call);                  \
        if (_rc != PCFR_OK) return _rc;                          \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
    int64_t N, rows, Hp, H, n_boards, term, fwd, dec, slots, chand_stride, sd_stride, n_eq, n_net, n_next;
    size_t esz;
    size_t off_nodes, off_fwd, off_dec, off_fwdoff, off_decoff, off_term, off_hc, off_coff, off_chands, off_sd, off_sdn, off_state,
        off_R, off_S, off_reach, off_cfv, off_root, off_stage, off_et, off_eq, off_eqpay, off_net, off_spr,
        off_potk, off_zs, off_agg, off_rc, off_next, off_c2h, off_h2c, off_roots, off_M, off_samp, off_eqpart,
        off_eqgrp, off_nsub, off_b4, off_nzs, off_tfrec, off_tfrest, off_tfterm, off_termrec, off_tftermrec,
        off_cmap, off_hmap, off_ncompat, off_flops, off_orbit, off_hoff, off_hlist, off_fpart, total;
    int64_t n_fgrp = 0;                   // preflop leaves: flop groups of the first pass
    size_t lds_bytes, lds_fold, lds_show;
    int64_t n_grp = 0, n_grp_allin = 0;   // equity groups: all leaves, the all-in prefix
    int eq_J = 0;                         // leaves per equity group at most
    int64_t H_leaf = 0;                   // hands of the subgames holding depth-limit leaves
};

struct Prepared {
    // forest of subgames: node ids are global, subgame k's nodes start at node_base[k]
    int32_t n_sub = 0;
    std::vector<int64_t> node_base, root_node;
    std::vector<DNode> nodes;
    std::vector<int32_t> fwd, term;       // fwd: decision and chance nodes by level (backward sweep)
    std::vector<int64_t> fwd_off;         // per level start into fwd (size levels+1)
    std::vector<int32_t> dec;             // decision nodes only, by level (forward sweep)
    std::vector<int64_t> dec_off;
    std::vector<DNode> fwd_rec, dec_rec;  // node records in the order of fwd and dec
    std::vector<int32_t> lvl_maxa;        // per level: most actions of a decision node
    std::vector<char> lvl_perm;           // per level: holds a chance node reading children through a hand permutation
    std::vector<int32_t> folds, shows;    // terminal lists by kind
    std::vector<uint16_t> hcards;         // [n_sub][Hp]
    std::vector<int32_t> coff;            // [n_sub][53]
    std::vector<int16_t> chands;          // [n_sub][chand_stride]
    int64_t chand_stride = 0;
    std::vector<int16_t> sd;              // [boards][sd_stride]
    std::vector<int32_t> sdn;
    std::vector<std::vector<int32_t>> hand_combo;   // per subgame [H_k]
    std::vector<std::vector<int32_t>> combo_hand;   // per subgame [1326], -1 if blocked
    std::vector<int64_t> Hs;              // hands per subgame
    std::vector<uint64_t> root_mask;
    int64_t Hp = 0, H = 0, sd_stride = 0;  // H: hands of subgame 0
    int32_t levels = 0, max_a = 0;
    // depth-limit leaves of every subgame: all-in leaves first, then
    // network leaves (so the all-in prefix is what stays exact when a
    // network is attached); subgames holding leaves share one board size
    std::vector<int32_t> eq_leaves;
    std::vector<int32_t> eq_sub;           // per leaf: its subgame
    std::vector<int32_t> et_slot;          // per subgame: its equity table, -1 without leaves
    int32_t n_et = 0;                      // subgames holding depth-limit leaves
    std::vector<double> eq_pay;
    int64_t n_allin = 0;
    int leaf_board = -1;                   // board size of the subgames with leaves
    int64_t leaf_H = 0;                    // their hands
    std::vector<int32_t> net_leaves;
    std::vector<int32_t> net_sub;          // per network leaf: its subgame
    std::vector<int32_t> board4s;          // [n_sub][4] root boards, -1 past the last card
    std::vector<int8_t> next_all;          // [n_sub][64] cards that can come next, -1 past the last
    std::vector<float> net_spr;
    std::vector<double> net_potk;
    std::vector<int8_t> next_cards;
    std::vector<int32_t> board;           // root board cards (subgame 0)
    // preflop roots (every subgame, or none): hands are the 169 classes
    bool preflop = false;
    std::vector<uint8_t> ncompat;          // [169][169] combos of class c' clear of a combo of class c
    std::vector<int8_t> flops;             // [n_flops][4] canonical flops (3 cards, pad)
    std::vector<int32_t> flop_orbit;       // [n_flops]
    std::vector<int32_t> hoff;             // [n_sub][Hp + 1] start of each hand's combos in hlist
    std::vector<int16_t> hlist;            // [n_sub][kComboPad] combos grouped by hand
};

// Hand class of combo k (cards hi > lo): 0..12 pairs by rank, then the 78
// suited and the 78 offsuit rank pairs, each by (high rank, low rank).
static int hand_class(int hi, int lo) {
    const int ra = hi / 4, rb = lo / 4;
    if (ra == rb) return ra;
    const int r1 = ra > rb ? ra : rb, r2 = ra > rb ? rb : ra;
    const int pair_idx = r1 * (r1 - 1) / 2 + r2;   // 0..77
    return 13 + (hi % 4 == lo % 4 ? 0 : 78) + pair_idx;
}

// Canonical flops: the flops that no suit permutation maps to a smaller
// 52-bit mask, by their sorted cards in lexicographic order, with the number
// of flops in each one's orbit.
static void canonical_flops(std::vector<int8_t>& cards, std::vector<int32_t>& orbit) {
    auto canon = [](uint64_t m) {
        uint64_t best = m;
        for (int q = 0; q < 24; q++) {
            uint64_t x = 0;
            for (int c = 0; c < 52; c++)
                if (m >> c & 1ull) x |= 1ull << suit_perm_card(q, c);
            best = std::min(best, x);
        }
        return best;
    };
    std::vector<uint64_t> masks, canons;
    for (int x = 0; x < 52; x++)
        for (int y = x + 1; y < 52; y++)
            for (int z = y + 1; z < 52; z++) {
                const uint64_t m = (1ull << x) | (1ull << y) | (1ull << z);
                masks.push_back(m);
                canons.push_back(canon(m));
            }
    std::map<uint64_t, int32_t> count;
    for (uint64_t c : canons) count[c]++;
    cards.clear();
    orbit.clear();
    for (size_t i = 0; i < masks.size(); i++) {
        if (canons[i] != masks[i]) continue;
        for (int c = 0; c < 52; c++)
            if (masks[i] >> c & 1ull) cards.push_back((int8_t)c);
        cards.push_back(-1);
        orbit.push_back(count[masks[i]]);
    }
}

// Host preprocessing of a forest of subgames: node records, merged level work
// lists, hand cards, per-card hand lists, and one strength-sorted table per
// (subgame, showdown board).
static int32_t prepare(const std::vector<const Tree*>& trees, Prepared& P, const IsoMap* iso = nullptr) {
    const ComboTable& cc = combos();
    const int32_t K = (int32_t)trees.size();
    P.n_sub = K;
    P.hand_combo.assign(K, {});
    P.combo_hand.assign(K, std::vector<int32_t>(kCombos, -1));
    P.Hs.assign(K, 0);
    P.root_mask.assign(K, 0);
    int64_t Hmax = 0;
    int n_pre = 0;
    for (int32_t g = 0; g < K; g++) n_pre += trees[g]->root_mask == 0;
    if (n_pre && n_pre != K) { set_error("a batch mixes preflop roots with other subgames"); return PCFR_E_UNSUPPORTED; }
    P.preflop = n_pre > 0;
    for (int32_t g = 0; g < K; g++) {
        const uint64_t rm = trees[g]->root_mask;
        P.root_mask[g] = rm;
        if (P.preflop) {
            // one hand per class, represented by its first combo
            P.hand_combo[g].assign(169, -1);
            for (int k = 0; k < kCombos; k++) {
                const int c = hand_class(cc.hi[k], cc.lo[k]);
                P.combo_hand[g][k] = c;
                if (P.hand_combo[g][c] < 0) P.hand_combo[g][c] = k;
            }
        } else {
            for (int k = 0; k < kCombos; k++) {
                if ((rm >> cc.hi[k] & 1ull) || (rm >> cc.lo[k] & 1ull)) continue;
                P.combo_hand[g][k] = (int32_t)P.hand_combo[g].size();
                P.hand_combo[g].push_back(k);
            }
        }
        P.Hs[g] = (int64_t)P.hand_combo[g].size();
        Hmax = std::max(Hmax, P.Hs[g]);
    }
    if (P.preflop) {
        P.ncompat.assign(169 * 169, 0);
        for (int c = 0; c < 169; c++) {
            const int k = P.hand_combo[0][c];
            const uint64_t m = (1ull << cc.hi[k]) | (1ull << cc.lo[k]);
            for (int j = 0; j < kCombos; j++)
                if (!(m >> cc.hi[j] & 1ull) && !(m >> cc.lo[j] & 1ull)) P.ncompat[(size_t)c * 169 + P.combo_hand[0][j]]++;
        }
        canonical_flops(P.flops, P.flop_orbit);
    }
    P.H = P.Hs[0];
    P.Hp = (Hmax + 63) / 64 * 64;
    if (P.Hp > kMaxHp) { set_error("more compatible hands than the kernels support"); return PCFR_E_TOO_LARGE; }
    const int64_t Hp = P.Hp;
    P.hcards.assign((size_t)K * Hp, 0xffff);
    P.coff.assign((size_t)K * 53, 0);
    P.chand_stride = (2 * Hmax + 7) / 8 * 8;    // 16-byte aligned per subgame (read in 8-entry vectors)
    P.chands.assign((size_t)K * P.chand_stride, 0);
    for (int32_t g = 0; g < K; g++) {
        for (int64_t h = 0; h < P.Hs[g]; h++) {
            int k = P.hand_combo[g][h];
            P.hcards[(size_t)g * Hp + h] = (uint16_t)(cc.hi[k] | (cc.lo[k] << 8));
        }
        std::vector<std::vector<int16_t>> lists(52);
        for (int64_t h = 0; h < P.Hs[g]; h++) {
            int k = P.hand_combo[g][h];
            lists[cc.hi[k]].push_back((int16_t)h);
            lists[cc.lo[k]].push_back((int16_t)h);
        }
        int32_t pos = 0;
        for (int c = 0; c < 52; c++) {
            P.coff[(size_t)g * 53 + c] = pos;
            for (auto x : lists[c]) P.chands[(size_t)g * P.chand_stride + pos++] = x;
        }
        P.coff[(size_t)g * 53 + 52] = pos;
    }
    // combos of each hand, grouped by hand (one each, or a class's combos)
    P.hoff.assign((size_t)K * (Hp + 1), 0);
    P.hlist.assign((size_t)K * kComboPad, 0);
    for (int32_t g = 0; g < K; g++) {
        std::vector<std::vector<int16_t>> per(Hp);
        for (int k = 0; k < kCombos; k++)
            if (P.combo_hand[g][k] >= 0) per[P.combo_hand[g][k]].push_back((int16_t)k);
        int32_t pos = 0;
        for (int64_t h = 0; h < Hp; h++) {
            P.hoff[(size_t)g * (Hp + 1) + h] = pos;
            for (auto k : per[h]) P.hlist[(size_t)g * kComboPad + pos++] = k;
        }
        P.hoff[(size_t)g * (Hp + 1) + Hp] = pos;
    }
    P.sd_stride = (8 * Hp + kSdHeader + 2 * Hp + kSdHeader + 63) / 64 * 64;
    std::map<std::pair<int32_t, uint64_t>, int32_t> board_id;
    int64_t N = 0;
    P.node_base.assign(K, 0);
    P.root_node.assign(K, 0);
    P.levels = 0;
    for (int32_t g = 0; g < K; g++) {
        P.node_base[g] = N;
        P.root_node[g] = N;
        N += (int64_t)trees[g]->nodes.size();
        P.levels = std::max(P.levels, trees[g]->n_levels);
    }
    P.nodes.resize(N);
    std::vector<std::vector<int32_t>> per_level(P.levels);
    // subgames with depth-limit leaves must share their board size, so that
    // every leaf has the same number of network rows and hands
    int leaf_board = -1;
    for (int32_t g = 0; g < K && leaf_board < 0; g++)
        if (trees[g]->count[PCFR_NODE_LEAF] + trees[g]->count[PCFR_NODE_ALLIN_LEAF] > 0)
            leaf_board = __builtin_popcountll(trees[g]->root_mask);
    int64_t rows = 0;
    for (int32_t g = 0; g < K; g++) {
        const Tree& t = *trees[g];
        const int64_t base = P.node_base[g];
        for (size_t i = 0; i < t.nodes.size(); i++) {
            const Node& s = t.nodes[i];
            const int64_t gi = base + (int64_t)i;
            DNode d{};
            d.type = s.type; d.player = s.player; d.n_child = s.n_child;
            d.first_child = s.first_child < 0 ? -1 : (int32_t)(base + s.first_child);
            d.rs = -1; d.aux = 0; d.sub = g; d.pay = 0.0;
            d.slot[0] = d.slot[1] = -1;
            const bool swept = !(iso && iso->skip[gi]);
            if (iso && iso->mapped[gi]) d.pad = 1;   // chance node reading some children through a permutation
            uint64_t extra = s.board_mask & ~t.root_mask;
            int dd[2] = {0xff, 0xff}, nd = 0;
            for (int c = 0; c < 52 && nd < 2; c++) if (extra >> c & 1ull) dd[nd++] = c;
            d.dead = dd[0] | (dd[1] << 8);
            if (s.type == PCFR_NODE_DECISION) {
                d.rs = (int32_t)rows;
                rows += s.n_child;
                if (s.n_child > kMaxActions || s.n_child < 1) { set_error("unsupported action count"); return PCFR_E_TOO_LARGE; }
                P.max_a = std::max(P.max_a, s.n_child);
                if (swept) per_level[s.depth].push_back((int32_t)gi);
            } else if (s.type == PCFR_NODE_CHANCE) {
                d.aux = 52 - __builtin_popcountll(s.board_mask) - 4;
                if (swept) per_level[s.depth].push_back((int32_t)gi);
            } else if (s.type == PCFR_NODE_FOLD) {
                d.pay = (double)s.contrib[s.player];
                if (swept) P.term.push_back((int32_t)gi);
            } else if (s.type == PCFR_NODE_SHOWDOWN) {
                d.pay = (double)s.contrib[0];
                if (swept) {
                    auto key = std::make_pair(g, s.board_mask);
                    auto it = board_id.find(key);
                    if (it == board_id.end()) it = board_id.emplace(key, (int32_t)board_id.size()).first;
                    d.aux = it->second;
                    P.term.push_back((int32_t)gi);
                }
            } else if (s.type == PCFR_NODE_ALLIN_LEAF || s.type == PCFR_NODE_LEAF) {
                if (__builtin_popcountll(t.root_mask) != leaf_board) {
                    set_error("batched depth-limited subgames must have boards of one size");
                    return PCFR_E_UNSUPPORTED;
                }
                if (s.contrib[0] != s.contrib[1]) { set_error("leaf with unequal contributions"); return PCFR_E_INVALID_ARG; }
                if (s.board_mask != t.root_mask) { set_error("depth-limit leaf below a chance node"); return PCFR_E_UNSUPPORTED; }
            } else {
                set_error("unknown node type");
                return PCFR_E_INVALID_ARG;
            }
            P.nodes[gi] = d;
        }
        if (rows > (int64_t)INT32_MAX) { set_error("too many action rows"); return PCFR_E_TOO_LARGE; }
    }
    if (2 * (int64_t)K + rows > (int64_t)INT32_MAX) { set_error("too many reach slots"); return PCFR_E_TOO_LARGE; }
    for (int32_t g = 0; g < K; g++)
        if (P.nodes[P.node_base[g]].type != PCFR_NODE_DECISION) { set_error("subgame root is not a decision node"); return PCFR_E_UNSUPPORTED; }
    // reach slots, parents before children (breadth-first ids)
    for (int32_t g = 0; g < K; g++) {
        DNode& r = P.nodes[P.node_base[g]];
        r.slot[0] = 2 * g;
        r.slot[1] = 2 * g + 1;
    }
    for (int64_t i = 0; i < (int64_t)P.nodes.size(); i++) {
        const DNode& d = P.nodes[i];
        if (d.type != PCFR_NODE_DECISION && d.type != PCFR_NODE_CHANCE) continue;
        for (int a = 0; a < d.n_child; a++) {
            DNode& c = P.nodes[d.first_child + a];
            c.slot[0] = d.slot[0];
            c.slot[1] = d.slot[1];
            if (d.type == PCFR_NODE_DECISION) c.slot[d.player] = (int32_t)(2 * K + d.rs + a);
        }
    }
    if (N > (int64_t)INT32_MAX) { set_error("too many nodes"); return PCFR_E_TOO_LARGE; }
    // depth-limit leaves of every subgame: all-in leaves first (exact
    // equity), then the others (the network's, or exact equity without one)
    P.n_allin = 0;
    P.leaf_board = leaf_board;
    P.leaf_H = 0;
    for (int32_t g = 0; g < K; g++)
        if (__builtin_popcountll(P.root_mask[g]) == leaf_board) { P.leaf_H = P.Hs[g]; break; }
    for (int pass = 0; pass < 2; pass++)
        for (int32_t g = 0; g < K; g++) {
            const Tree& t = *trees[g];
            const int64_t eff = std::min(t.spec.stack[0], t.spec.stack[1]);
            const int64_t cap = t.spec.pot / 2 + eff;
            for (size_t i = 0; i < t.nodes.size(); i++) {
                const Node& s = t.nodes[i];
                if (s.type != (pass == 0 ? PCFR_NODE_ALLIN_LEAF : PCFR_NODE_LEAF)) continue;
                P.eq_leaves.push_back((int32_t)(P.node_base[g] + (int64_t)i));
                P.eq_sub.push_back(g);
                P.eq_pay.push_back((double)s.contrib[0]);
                if (pass == 0) P.n_allin++;
                if (pass == 1) {
                    const int nb = __builtin_popcountll(s.board_mask);
                    P.net_leaves.push_back((int32_t)(P.node_base[g] + (int64_t)i));
                    P.net_sub.push_back(g);
                    P.net_spr.push_back((float)((double)(cap - s.contrib[0]) / (double)(2 * s.contrib[0])));
                    // chance weight per history: 1 / (next cards, or flops, clear of both hands)
                    P.net_potk.push_back((double)(2 * s.contrib[0]) / (nb == 0 ? 17296.0 : (double)(52 - nb - 4)));
                }
            }
        }
    // an equity table only for the subgames that hold leaves
    P.et_slot.assign(K, -1);
    P.n_et = 0;
    for (int32_t g : P.eq_sub)
        if (P.et_slot[g] < 0 && !P.preflop) P.et_slot[g] = P.n_et++;   // preflop leaves: the network only
    // per subgame: the root board (up to 4 cards, -1 past the last) and the
    // cards that can come next (one table row of 64 per subgame)
    P.board4s.assign((size_t)K * 4, -1);
    P.next_all.assign((size_t)K * 64, -1);
    for (int32_t g = 0; g < K; g++) {
        int nb = 0, nn = 0;
        for (int c = 0; c < 52; c++) {
            if (P.root_mask[g] >> c & 1ull) {
                if (nb < 4) P.board4s[(size_t)g * 4 + nb] = c;
                nb++;
                if (g == 0) P.board.push_back(c);
            } else {
                P.next_all[(size_t)g * 64 + nn++] = (int8_t)c;
                if (g == 0) P.next_cards.push_back((int8_t)c);
            }
        }
    }
    P.fwd_off.assign(P.levels + 1, 0);
    P.dec_off.assign(P.levels + 1, 0);
    P.lvl_maxa.assign(P.levels, 0);
    P.lvl_perm.assign(P.levels, 0);
    for (int l = 0; l < P.levels; l++) {
        P.fwd_off[l] = (int64_t)P.fwd.size();
        P.dec_off[l] = (int64_t)P.dec.size();
        for (auto x : per_level[l]) {
            if (P.nodes[x].type == PCFR_NODE_CHANCE && P.nodes[x].pad) P.lvl_perm[l] = 1;
            P.fwd.push_back(x);
            if (P.nodes[x].type == PCFR_NODE_DECISION) {
                P.dec.push_back(x);
                P.lvl_maxa[l] = std::max(P.lvl_maxa[l], P.nodes[x].n_child);
            }
        }
    }
    P.dec_off[P.levels] = (int64_t)P.dec.size();
    for (auto x : P.term) (P.nodes[x].type == PCFR_NODE_FOLD ? P.folds : P.shows).push_back(x);
    P.term.clear();
    P.term.insert(P.term.end(), P.folds.begin(), P.folds.end());
    P.term.insert(P.term.end(), P.shows.begin(), P.shows.end());
    P.fwd_off[P.levels] = (int64_t)P.fwd.size();
    for (int64_t i = 0; i < (int64_t)P.nodes.size(); i++) P.nodes[i].id = (int32_t)i;
    P.fwd_rec.clear();
    P.dec_rec.clear();
    for (auto x : P.fwd) P.fwd_rec.push_back(P.nodes[x]);
    for (auto x : P.dec) P.dec_rec.push_back(P.nodes[x]);
    // strength tables
    const int64_t nbds = (int64_t)board_id.size();
    P.sd.assign((size_t)std::max<int64_t>(nbds, 1) * P.sd_stride, 0);
    P.sdn.assign(std::max<int64_t>(nbds, 1), 0);
    for (auto& kv : board_id) {
        const int32_t g = kv.first.first;
        const uint64_t bm = kv.first.second;
        const std::vector<int32_t>& hcmb = P.hand_combo[g];
        int16_t* tb = P.sd.data() + (size_t)kv.second * P.sd_stride;
        std::vector<std::pair<uint32_t, int32_t>> alive;
        std::vector<char> is_alive(Hp, 0);
        for (int64_t h = 0; h < P.Hs[g]; h++) {
            int k = hcmb[h];
            uint64_t hm = (1ull << cc.hi[k]) | (1ull << cc.lo[k]);
            if (hm & bm) continue;
            alive.push_back({eval7_mask(hm | bm), (int32_t)h});
            is_alive[h] = 1;
        }
        std::sort(alive.begin(), alive.end());
        const int Hb = (int)alive.size();
        P.sdn[kv.second] = Hb;
        int16_t *perm = tb, *glo = tb + Hp, *ghi = tb + 2 * Hp, *alo = tb + 3 * Hp, *ahi = tb + 4 * Hp,
                *blo = tb + 5 * Hp, *bhi = tb + 6 * Hp, *scard = tb + 7 * Hp, *coff = tb + 8 * Hp,
                *clist = coff + kSdHeader;
        int s = 0;
        for (auto& x : alive) {
            const int k = hcmb[x.second];
            scard[s] = (int16_t)(uint16_t)(cc.hi[k] | (cc.lo[k] << 8));
            perm[s++] = (int16_t)x.second;
        }
        for (int64_t h = 0; h < Hp; h++) if (!is_alive[h]) perm[s++] = (int16_t)h;
        for (int i = 0; i < Hb;) {
            int j = i;
            while (j < Hb && alive[j].first == alive[i].first) j++;
            for (int q = i; q < j; q++) { glo[q] = (int16_t)i; ghi[q] = (int16_t)j; }
            i = j;
        }
        // per-card lists of sorted positions, each followed by a total slot
        std::vector<std::vector<int>> lists(52);
        for (int q = 0; q < Hb; q++) {
            int k = hcmb[alive[q].second];
            lists[cc.hi[k]].push_back(q);
            lists[cc.lo[k]].push_back(q);
        }
        int pos = 0;
        std::vector<int> where_hi(Hb), where_lo(Hb);
        for (int c = 0; c < 52; c++) {
            coff[c] = (int16_t)pos;
            for (int q : lists[c]) {
                int k = hcmb[alive[q].second];
                if (cc.hi[k] == c) where_hi[q] = pos; else where_lo[q] = pos;
                clist[pos++] = (int16_t)q;
            }
            clist[pos++] = -1;
        }
        coff[52] = (int16_t)pos;
        auto group = [&](int c, int at, int16_t& lo, int16_t& hi) {
            uint32_t v = alive[clist[at]].first;
            int a = at, b = at;
            while (a > coff[c] && alive[clist[a - 1]].first == v) a--;
            while (b + 1 < coff[c + 1] - 1 && alive[clist[b + 1]].first == v) b++;
            lo = (int16_t)a;
            hi = (int16_t)(b + 1);
        };
        for (int q = 0; q < Hb; q++) {
            int k = hcmb[alive[q].second];
            group(cc.hi[k], where_hi[q], alo[q], ahi[q]);
            group(cc.lo[k], where_lo[q], blo[q], bhi[q]);
        }
    }
    return PCFR_OK;
}

// Workgroup groups of the equity kernel: runs of up to J consecutive leaves of
// one subgame, never across the end of the all-in prefix; {first, count,
// equity table of the subgame, 0} each.  n_allin_groups: the groups of the all-in prefix.
static void equity_groups(const Prepared& P, int J, std::vector<int32_t>& out, int64_t& n_allin_groups) {
    out.clear();
    n_allin_groups = 0;
    const int64_t n = (int64_t)P.eq_leaves.size();
    for (int64_t i = 0; i < n;) {
        int64_t j = i + 1;
        while (j < n && j - i < J && P.eq_sub[j] == P.eq_sub[i] && j != P.n_allin) j++;
        out.insert(out.end(), {(int32_t)i, (int32_t)(j - i), P.et_slot[P.eq_sub[i]], 0});
        if (j <= P.n_allin) n_allin_groups++;
        i = j;
    }
}

// One subgame: narrow groups keep many workgroups in flight (its table stays
// in cache across them).  Several: wide groups, so each subgame's table is
// streamed from HBM about once per iteration rather than once per few leaves.
static int equity_group_width(size_t esz, int32_t n_sub) {
    if (n_sub > 1) return esz == 8 ? 8 : 16;
    return esz == 8 ? 2 : 4;
}

static void make_plan(const Prepared& P, int64_t rows, int dtype, int variant, bool iso, Plan& L) {
    L.N = (int64_t)P.nodes.size();
    L.rows = rows;
    L.Hp = P.Hp;
    L.H = P.H;
    L.n_boards = (int64_t)P.sdn.size();
    L.term = (int64_t)P.term.size();
    L.fwd = (int64_t)P.fwd.size();
    L.dec = (int64_t)P.dec.size();
    L.slots = 2 * (int64_t)P.n_sub + rows;
    L.chand_stride = P.chand_stride;
    L.sd_stride = P.sd_stride;
    L.esz = dtype == PCFR_F64 ? 8 : 4;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.off_nodes = take(sizeof(DNode) * L.N);
    L.off_fwd = take(sizeof(DNode) * std::max<int64_t>(L.fwd, 1));
    L.off_dec = take(sizeof(DNode) * std::max<int64_t>(L.dec, 1));
    L.off_fwdoff = take(sizeof(int64_t) * (P.levels + 1));
    L.off_decoff = take(sizeof(int64_t) * (P.levels + 1));
    L.off_term = take(sizeof(int32_t) * std::max<int64_t>(L.term, 1));
    L.off_hc = take(sizeof(uint16_t) * L.Hp * P.n_sub);
    L.off_coff = take(sizeof(int32_t) * 53 * P.n_sub);
    L.off_chands = take(sizeof(int16_t) * std::max<int64_t>(L.chand_stride, 1) * P.n_sub);
    L.off_sd = take(sizeof(int16_t) * L.n_boards * L.sd_stride);
    L.off_sdn = take(sizeof(int32_t) * L.n_boards);
    L.off_state = take(sizeof(IterState));
    L.off_R = take(L.esz * L.rows * L.Hp);
    L.off_S = take(L.esz * L.rows * L.Hp);
    L.off_reach = take(L.esz * L.slots * L.Hp);
    L.off_cfv = take(L.esz * L.N * 2 * L.Hp);
    L.off_root = take(L.esz * 2 * L.Hp * P.n_sub);
    L.off_stage = take(L.esz * kMaxActions * L.Hp);
    L.n_eq = (int64_t)P.eq_leaves.size();
    L.n_net = (int64_t)P.net_leaves.size();
    {
        std::vector<int32_t> grp;
        L.eq_J = equity_group_width(L.esz, P.n_sub);
        equity_groups(P, L.eq_J, grp, L.n_grp_allin);
        L.n_grp = (int64_t)grp.size() / 4;
    }
    L.H_leaf = P.leaf_H;
    L.n_next = P.preflop ? (int64_t)P.flop_orbit.size()
                         : P.leaf_board >= 0 ? 52 - P.leaf_board : (int64_t)P.next_cards.size();
    // one pairwise equity table per subgame holding leaves, [n_et][Hp][Hp]
    L.off_et = take(L.esz * L.Hp * L.Hp * (size_t)P.n_et);
    L.off_eqgrp = take(sizeof(int32_t) * 4 * std::max<int64_t>(L.n_grp, 1));
    L.off_nsub = take(sizeof(int32_t) * std::max<int64_t>(L.n_net, 1));
    L.off_b4 = take(sizeof(int32_t) * 4 * P.n_sub);
    L.off_eq = take(sizeof(int32_t) * std::max<int64_t>(L.n_eq, 1));
    L.off_eqpay = take(sizeof(double) * std::max<int64_t>(L.n_eq, 1));
    L.off_net = take(sizeof(int32_t) * std::max<int64_t>(L.n_net, 1));
    L.off_spr = take(sizeof(float) * std::max<int64_t>(L.n_net, 1));
    L.off_potk = take(sizeof(double) * std::max<int64_t>(L.n_net, 1));
    L.off_zs = take(L.esz * std::max<int64_t>(L.n_net * L.n_next, 1));
    L.off_agg = take(L.esz * kAgg * std::max<int64_t>(L.n_net, 1));
    L.off_rc = take(L.esz * 2 * kComboPad * std::max<int64_t>(L.n_net, 1));
    // suit isomorphism: per node (source child, permutation); per subgame and permutation, the hand map
    L.off_cmap = take(iso ? sizeof(int32_t) * 2 * L.N : 0);
    L.off_hmap = take(iso ? sizeof(int16_t) * 24 * L.Hp * P.n_sub : 0);
    L.off_next = take(64 * (size_t)P.n_sub);
    L.off_c2h = take(sizeof(int16_t) * kComboPad * P.n_sub);   // rows padded: 16-byte aligned per subgame
    L.off_h2c = take(sizeof(int16_t) * L.Hp * P.n_sub);
    L.off_roots = take(sizeof(int32_t) * P.n_sub);
    L.off_M = take(variant == PCFR_PCFRPLUS ? L.esz * L.rows * L.Hp : 0);
    L.off_samp = take(align256(sizeof(float) * 2 * P.n_sub) + align256((size_t)P.n_sub * 52) +
                      align256(sizeof(int16_t) * (size_t)P.n_sub * kCombos));
    L.off_eqpart = take(L.esz * kEqSplit * L.n_eq * 2 * L.Hp);
    L.off_ncompat = take(P.ncompat.size());
    L.off_flops = take(P.flops.size());
    L.off_orbit = take(sizeof(int32_t) * P.flop_orbit.size());
    L.off_hoff = take(sizeof(int32_t) * P.hoff.size());
    L.off_hlist = take(sizeof(int16_t) * P.hlist.size());
    L.n_fgrp = P.preflop ? (L.n_next + kFlopsPerGroup - 1) / kFlopsPerGroup : 0;
    L.off_fpart = take(L.esz * L.n_net * L.n_fgrp * 2 * L.Hp);
    L.off_nzs = take(sizeof(int32_t) * (size_t)(2 * P.n_sub + L.rows));   // pruning flags per reach slot
    // terminal fusion: node records of the fused and the remaining backward work, terminals left over
    L.off_tfrec = take(sizeof(DNode) * std::max<size_t>(P.dec.size(), 1));
    L.off_tfrest = take(sizeof(DNode) * std::max<size_t>(P.fwd.size(), 1));
    L.off_tfterm = take(sizeof(int32_t) * std::max<size_t>(P.term.size(), 1));
    // terminal records in the terminal launches' order, and the same for the
    // terminals left to those launches by terminal fusion
    L.off_termrec = take(sizeof(DNode) * std::max<size_t>(P.term.size(), 1));
    L.off_tftermrec = take(sizeof(DNode) * std::max<size_t>(P.term.size(), 1));
    L.total = o;
    const size_t qn = 2 * L.Hp + kSdHeader;
    const size_t sd_nw = (qn + 63) / 64, sd_ns = L.Hp / 64;   // nonzero-reach bitmask words
    const size_t sd_lds = L.esz * (2 * (L.Hp + 4) + 2 * qn + 2 * kBlock) + sizeof(int16_t) * (kSdHeader + qn + L.Hp) +
                          sizeof(int32_t) * 104 + sizeof(uint64_t) * 2 * (sd_nw + sd_ns) +
                          sizeof(int32_t) * 2 * (sd_nw + sd_ns + 1);
    const size_t fold_lds = L.esz * (2 * L.Hp + 208 + 2 * kBlock) + sizeof(int16_t) * 2 * L.Hp + sizeof(int32_t) * 208;
    L.lds_fold = fold_lds;
    L.lds_show = sd_lds;
    L.lds_bytes = std::max(sd_lds, fold_lds);
}

}  // namespace pcfr

using namespace pcfr;

namespace pcfr {
// Launch schedule of the level sweeps: workgroup size per level and phase.
// The arithmetic of each (node, hand) does not depend on it, so any schedule
// gives bitwise the same iterates.
struct Sched {
    std::vector<int> fwd_block, bwd_block;
    // runs of consecutive levels with at most this many threads (nodes x
    // Hp/4) each are swept by one level-fused launch; 0 = never
    int64_t fuse_threads = 16384;
};
}  // namespace pcfr

struct pcfr_solver {
    std::vector<Tree> trees;
    pcfr_solver_cfg cfg;
    Prepared P;
    Plan L;
    Sched sched;
    hipStream_t stream = nullptr;
    // second stream and fork/join events: terminals and exact leaves run
    // beside the network stage (a parallel branch of the captured graph)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    char* ws = nullptr;
    std::vector<double> ranges;       // [n_sub][2][1326]
    std::vector<double> pair_mass;    // [n_sub]
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    pcfr_leafnet* net = nullptr;
    IsoMap iso;                 // suit isomorphism map (suit_iso = 1)
    bool leaf_zero_sum = true;  // shift network outputs to zero-sum leaf values
    int64_t t_host = 0;     // iterations enqueued
    int32_t launch_mode = PCFR_LAUNCH_GRAPH;
    int32_t persist_grid = 0, persist_maxa = 0;   // persistent launch: resident workgroups, action bucket
    // terminal fusion (k_backward_tf): off by default (one workgroup per
    // parent runs its terminals and its backward in series, slower on turns
    // than the separate wide launches); the plan follows the level-fusion
    // schedule and is rebuilt with the graph
    bool tf_enabled = false;
    struct {
        bool on = false;
        std::vector<int64_t> tf_off, rest_off;   // per level starts into the device record arrays
        int64_t n_fold = 0, n_show = 0;          // terminals left to k_terminal
        size_t lds = 0, val_off = 0;             // dynamic LDS of k_backward_tf, offset of its value rows
    } tf;
    template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
    ~pcfr_solver() {
        if (stream && ws) (void)hipStreamSynchronize(stream);
        if (aux) { (void)hipStreamSynchronize(aux); (void)hipStreamDestroy(aux); }
        if (graph) (void)hipGraphExecDestroy(graph);
        if (graph_def) (void)hipGraphDestroy(graph_def);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
    }
};

namespace pcfr {

// One sweep: forward, terminals and leaves, backward.  upd: the player whose
// regrets and average strategy are updated (-1: both); begin: this sweep
// starts a new iteration (advances t).
template <typename T, int MODE>
static int32_t enqueue_sweep(pcfr_solver* s, hipStream_t stream, LaunchTimer* tm = nullptr, int upd = -1,
                             bool begin = true) {
    const Plan& L = s->L;
    const Prepared& P = s->P;
    const int Hp = (int)L.Hp;
    const int groups = Hp / 4;
    DNode* nodes = s->at<DNode>(L.off_nodes);
    DNode* fwd = s->at<DNode>(L.off_fwd);
    DNode* dec = s->at<DNode>(L.off_dec);
    T* R = s->at<T>(L.off_R);
    T* S = s->at<T>(L.off_S);
    T* reach = s->at<T>(L.off_reach);
    T* cfv = s->at<T>(L.off_cfv);
    T* Mp = s->cfg.variant == PCFR_PCFRPLUS ? s->at<T>(L.off_M) : nullptr;
    IterState* st = s->at<IterState>(L.off_state);
    // the kernels are instantiated for at most 3, 6, 8 or 12 actions; a level
    // uses the smallest that covers its nodes (fewer registers, more waves)
#define PCFR_BUCKET(KER, l, ...)                                                                      \
    do {                                                                                              \
        const int ma = P.lvl_maxa[l];                                                                 \
        if (ma <= 3) hipLaunchKernelGGL((KER<T, MODE, 3>), __VA_ARGS__);                              \
        else if (ma <= 6) hipLaunchKernelGGL((KER<T, MODE, 6>), __VA_ARGS__);                         \
        else if (ma <= 8) hipLaunchKernelGGL((KER<T, MODE, 8>), __VA_ARGS__);                         \
        else hipLaunchKernelGGL((KER<T, MODE, 12>), __VA_ARGS__);                                     \
    } while (0)
    // forward: decision nodes only; the first launch of an iteration also
    // advances t and sets the Stage-7 coefficients
#define PCFR_BUCKET_MA(KER, ma, ...)                                                                  \
    do {                                                                                              \
        if ((ma) <= 3) hipLaunchKernelGGL((KER<T, MODE, 3>), __VA_ARGS__);                            \
        else if ((ma) <= 6) hipLaunchKernelGGL((KER<T, MODE, 6>), __VA_ARGS__);                       \
        else if ((ma) <= 8) hipLaunchKernelGGL((KER<T, MODE, 8>), __VA_ARGS__);                       \
        else hipLaunchKernelGGL((KER<T, MODE, 12>), __VA_ARGS__);                                     \
    } while (0)
    const int64_t fuse = s->sched.fuse_threads;
    const dim3 fgrid((unsigned)(Hp / kFuseHands));
    auto dec_cnt = [&](int l) { return P.dec_off[l + 1] - P.dec_off[l]; };
    auto all_cnt = [&](int l) { return P.fwd_off[l + 1] - P.fwd_off[l]; };
    bool first = MODE == MODE_ITER && begin;
    // regret-based pruning flags of this sweep (iteration sweeps only): the
    // action slots' flags are cleared, the roots' stay set
    int32_t* nzs = (MODE == MODE_ITER && s->cfg.prune) ? s->at<int32_t>(L.off_nzs) : nullptr;
    if (nzs) {
        const int64_t n = L.rows;
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 2048)), dim3(256), 0, stream,
                           nzs + 2 * P.n_sub, n, 0);
    }
    // with thresholding every forward launch reads this iteration's
    // threshold (thr_st), so t advances in a launch of its own
    const IterState* thr_st = (MODE == MODE_ITER && s->cfg.threshold > 0) ? st : nullptr;
    if (first && s->cfg.threshold > 0) {
        hipLaunchKernelGGL(k_begin_iteration, dim3(1), dim3(1), 0, stream, st);
        first = false;
    }
    for (int l = 0; l < P.levels;) {
        const int64_t cnt = dec_cnt(l);
        if (!cnt) { l++; continue; }
        if (cnt * groups <= fuse) {
            int l1 = l + 1, ma = P.lvl_maxa[l];
            while (l1 < P.levels && dec_cnt(l1) * groups <= fuse) ma = std::max(ma, P.lvl_maxa[l1++]);
            if (tm) tm->before(1);
            PCFR_BUCKET_MA(k_forward_fused, ma, fgrid, dim3(kFuseBlock), 0, stream, dec, s->at<int64_t>(L.off_decoff), l,
                           l1, Hp, (int)(2 * P.n_sub), R, S, Mp, reach, first ? st : nullptr, thr_st, nzs);
            if (tm) tm->after();
            first = false;
            l = l1;
            continue;
        }
        const int bs = s->sched.fwd_block[l];
        const int64_t threads = cnt * groups;
        dim3 grid((unsigned)((threads + bs - 1) / bs));
        if (tm) tm->before(1, l);
        PCFR_BUCKET(k_forward, l, grid, dim3(bs), 0, stream, dec + P.dec_off[l], (int)cnt, Hp,
                    (int)(2 * P.n_sub), R, S, Mp, reach, first ? st : nullptr, thr_st, nzs);
        if (tm) tm->after();
        first = false;
        l++;
    }
    // terminals and exact-equity leaves do not depend on the network stage:
    // without per-launch timing they go to the second stream, joined before
    // the backward sweep
    const bool fork = !tm && s->aux && s->net && L.n_net;
    hipStream_t side = fork ? s->aux : stream;
    if (fork) {
        HIPCHK(hipEventRecord(s->ev_fork, stream));
        HIPCHK(hipStreamWaitEvent(side, s->ev_fork, 0));
    }
    // terminals: folds and showdowns in separate launches, each with the LDS it
    // needs; with terminal fusion only those whose parent does not evaluate them
    const bool tfo = MODE == MODE_ITER && s->tf.on;
    const int64_t n_fold = tfo ? s->tf.n_fold : (int64_t)P.folds.size();
    const int64_t n_show = tfo ? s->tf.n_show : (int64_t)P.shows.size();
    const int32_t* tlist = s->at<int32_t>(tfo ? L.off_tfterm : L.off_term);
    const DNode* trec = s->at<DNode>(tfo ? L.off_tftermrec : L.off_termrec);
    if (P.preflop && n_fold) {
        // folds over the hand classes (a preflop tree has no showdown)
        if (tm) tm->before(2);
        hipLaunchKernelGGL((k_fold_class<T>), dim3((unsigned)n_fold), dim3(kBlock), 0, side, nodes, tlist, Hp,
                           (int)P.H, reach, cfv, s->at<uint8_t>(L.off_ncompat), nzs);
        if (tm) tm->after();
    }
    for (int kind = 0; kind < 2 && !P.preflop; kind++) {
        const int64_t cnt = kind ? n_show : n_fold;
        if (!cnt) continue;
        if (tm) tm->before(2);
        if (kind)
            hipLaunchKernelGGL((k_terminal<T, 1>), dim3((unsigned)cnt), dim3(kBlock), L.lds_show, side,
                               trec + n_fold, Hp, reach, cfv, s->at<uint16_t>(L.off_hc), s->at<int32_t>(L.off_coff),
                               s->at<int16_t>(L.off_chands), (int)L.chand_stride, s->at<int16_t>(L.off_sd),
                               (int64_t)L.sd_stride, s->at<int32_t>(L.off_sdn), nzs);
        else
            hipLaunchKernelGGL((k_terminal<T, 0>), dim3((unsigned)cnt), dim3(kBlock), L.lds_fold, side, trec,
                               Hp, reach, cfv, s->at<uint16_t>(L.off_hc), s->at<int32_t>(L.off_coff),
                               s->at<int16_t>(L.off_chands), (int)L.chand_stride, s->at<int16_t>(L.off_sd),
                               (int64_t)L.sd_stride, s->at<int32_t>(L.off_sdn), nzs);
        if (tm) tm->after();
    }
    // depth-limit leaves: exact equity for all-in leaves (and for every leaf
    // without a network), the network for the others
    const int64_t n_eq_active = (s->net || P.preflop) ? P.n_allin : L.n_eq;
    if (n_eq_active) {
        const int64_t n_grp = s->net ? L.n_grp_allin : L.n_grp;
        dim3 grid((unsigned)((Hp + kBlock - 1) / kBlock), (unsigned)n_grp, kEqSplit);
        if (tm) tm->before(4);
        // the kernel's width must be the one the groups were built for
        constexpr int J1 = sizeof(T) == 8 ? 2 : 4, J2 = sizeof(T) == 8 ? 8 : 16;
        const int4* grp = reinterpret_cast<const int4*>(s->at<int32_t>(L.off_eqgrp));
        if (L.eq_J == J1)
            hipLaunchKernelGGL((k_equity_partial<T, J1>), grid, dim3(kBlock), 0, side, nodes, s->at<int32_t>(L.off_eq),
                               (int)n_eq_active, Hp, grp, s->at<T>(L.off_et), reach, s->at<T>(L.off_eqpart));
        else if (L.eq_J == J2)
            hipLaunchKernelGGL((k_equity_partial<T, J2>), grid, dim3(kBlock), 0, side, nodes, s->at<int32_t>(L.off_eq),
                               (int)n_eq_active, Hp, grp, s->at<T>(L.off_et), reach, s->at<T>(L.off_eqpart));
        else {
            set_error("equity group width does not match a kernel");
            return PCFR_E_STATE;
        }
        const int64_t tot = n_eq_active * 2 * (int64_t)Hp;
        hipLaunchKernelGGL((k_equity_reduce<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, side,
                           s->at<int32_t>(L.off_eq), s->at<double>(L.off_eqpay), (int)n_eq_active, Hp,
                           s->at<T>(L.off_eqpart), cfv);
        if (tm) tm->after();
    }
    if (P.preflop && L.n_net && s->net) {
        // preflop leaves: the flop-level network on the canonical flops (a
        // solver without one refuses to iterate, leaves_ready)
        pcfr_leafnet* net = s->net;
        const int64_t rows = L.n_net * L.n_next, Mp = (rows + 63) / 64 * 64;
        const int ldx = (int)net->P.pdims[0], ldy = (int)net->P.pdims[net->P.L];
        const float* Y = reinterpret_cast<const float*>(net->ws + net->P.off_y);
        // 16 flops per workgroup of the input kernel (4 per wave)
        const int fpg = 16;
        const int n_grp = (int)((L.n_next + fpg - 1) / fpg);
        if (tm) tm->before(4);
        hipLaunchKernelGGL((k_flop_leaf_input<T>), dim3((unsigned)L.n_net, (unsigned)n_grp), dim3(kBlock), 0, stream,
                           nodes, s->at<int32_t>(L.off_net), Hp, reach, s->at<int16_t>(L.off_c2h), s->at<T>(L.off_rc),
                           s->at<T>(L.off_agg), s->at<float>(L.off_spr), (int)L.n_next, fpg,
                           s->at<int8_t>(L.off_flops), ldx, reinterpret_cast<uint16_t*>(net->ws + net->P.off_x));
        if (tm) tm->after();
        int32_t rc = leafnet_forward_staged(net, Mp, stream, tm);
        if (rc) return rc;
        if (tm) tm->before(4);
        hipLaunchKernelGGL((k_flop_leaf_sums<T>), dim3((unsigned)L.n_net, (unsigned)L.n_fgrp), dim3(kBlock), 0, stream,
                           nodes, s->at<int32_t>(L.off_net), (int)L.n_next, (int)kFlopsPerGroup,
                           s->at<int8_t>(L.off_flops), s->at<int32_t>(L.off_orbit), s->at<int32_t>(L.off_hoff),
                           s->at<int16_t>(L.off_hlist), Hp, (int)L.H_leaf, Y, ldy, s->at<T>(L.off_rc),
                           s->at<T>(L.off_agg), s->leaf_zero_sum ? 1 : 0, s->at<T>(L.off_fpart));
        hipLaunchKernelGGL((k_flop_leaf_values<T>), dim3((unsigned)L.n_net, (unsigned)((2 * Hp + 63) / 64)), dim3(kBlock),
                           0, stream,
                           s->at<int32_t>(L.off_net), s->at<double>(L.off_potk), nodes, s->at<int32_t>(L.off_hoff),
                           (int)L.n_fgrp, Hp, (int)L.H_leaf, s->at<T>(L.off_fpart), cfv);
        if (tm) tm->after();
    } else if (s->net && L.n_net) {
        pcfr_leafnet* net = s->net;
        const int64_t rows = L.n_net * L.n_next, Mp = (rows + 63) / 64 * 64;
        if (tm) tm->before(4);
        const int ldx = (int)net->P.pdims[0];   // a multiple of 8, checked when the network is attached
        // about 1024 row groups per launch (at least one card per group)
        const int cpg = (int)std::min<int64_t>(L.n_next, std::max<int64_t>(1, (rows + 1023) / 1024));
        const int n_grp = (int)((L.n_next + cpg - 1) / cpg);
        hipLaunchKernelGGL((k_leaf_input<T>), dim3((unsigned)L.n_net, (unsigned)n_grp), dim3(kBlock), 0, stream, nodes,
                           s->at<int32_t>(L.off_net), Hp, reach, s->at<int16_t>(L.off_c2h), s->at<T>(L.off_rc),
                           s->at<T>(L.off_agg), s->at<float>(L.off_spr), (int)L.n_next, cpg,
                           s->at<int8_t>(L.off_next), reinterpret_cast<const int4*>(s->at<int32_t>(L.off_b4)), ldx,
                           reinterpret_cast<uint16_t*>(net->ws + net->P.off_x));
        if (tm) tm->after();
        int32_t rc = leafnet_forward_staged(net, Mp, stream, tm);
        if (rc) return rc;
        if (s->leaf_zero_sum) {
            if (tm) tm->before(4);
            hipLaunchKernelGGL((k_leaf_zerosum<T>), dim3((unsigned)rows), dim3(kBlock), 0, stream, (int)L.n_next,
                               s->at<int32_t>(L.off_nsub), s->at<int8_t>(L.off_next), s->at<T>(L.off_rc),
                               s->at<T>(L.off_agg),
                               reinterpret_cast<const float*>(net->ws + net->P.off_y), (int)net->P.pdims[net->P.L],
                               s->at<T>(L.off_zs));
            if (tm) tm->after();
        }
        if (tm) tm->before(4);
        hipLaunchKernelGGL((k_leaf_combine<T>), dim3((unsigned)L.n_net, (unsigned)((Hp + 63) / 64)),
                           dim3(kBlock), 0, stream, nodes,
                           s->at<int32_t>(L.off_net), s->at<double>(L.off_potk), (int)L.n_next,
                           s->at<int8_t>(L.off_next), Hp, (int)L.H_leaf, reach, cfv, s->at<uint16_t>(L.off_hc),
                           s->at<int16_t>(L.off_h2c), s->at<int16_t>(L.off_c2h),
                           reinterpret_cast<const float*>(net->ws + net->P.off_y),
                           (int)net->P.pdims[net->P.L], s->at<T>(L.off_agg),
                           s->leaf_zero_sum ? s->at<T>(L.off_zs) : nullptr);
        if (tm) tm->after();
    }
    if (fork) {
        HIPCHK(hipEventRecord(s->ev_join, side));
        HIPCHK(hipStreamWaitEvent(stream, s->ev_join, 0));
    }
    // backward; level 0 holds exactly the roots, whose values of this
    // iteration are also kept apart from later evaluation sweeps
    const IsoTabs iso = {s->cfg.suit_iso ? s->at<int32_t>(L.off_cmap) : nullptr,
                         s->cfg.suit_iso ? s->at<int16_t>(L.off_hmap) : nullptr};
    for (int l = P.levels - 1; l >= 0;) {
        const int64_t cnt = all_cnt(l);
        if (!cnt) { l--; continue; }
        if (cnt * groups <= fuse) {
            // a run does not climb to a level whose chance nodes read other
            // hands of their children (suit isomorphism): those children
            // must be complete for every hand, i.e. from an earlier launch
            int l0 = l, ma = P.lvl_maxa[l];
            while (l0 > 0 && all_cnt(l0 - 1) * groups <= fuse && !P.lvl_perm[l0 - 1]) ma = std::max(ma, P.lvl_maxa[--l0]);
            if (tm) tm->before(3);
            PCFR_BUCKET_MA(k_backward_fused, ma, fgrid, dim3(kFuseBlock), 0, stream,
                           fwd, s->at<int64_t>(L.off_fwdoff), l0, l + 1, Hp, R, S, Mp, reach, cfv, st,
                           s->at<uint16_t>(L.off_hc), (MODE == MODE_ITER && l0 == 0) ? s->at<T>(L.off_root) : nullptr,
                           upd, iso, nzs);
            if (tm) tm->after();
            l = l0 - 1;
            continue;
        }
        const int bs = s->sched.bwd_block[l];
        T* rootd = (MODE == MODE_ITER && l == 0) ? s->at<T>(L.off_root) : nullptr;
        const DNode* lrec = fwd + P.fwd_off[l];
        int64_t lcnt = cnt;
        if (tfo) {
            lrec = s->at<DNode>(L.off_tfrest) + s->tf.rest_off[l];
            lcnt = s->tf.rest_off[l + 1] - s->tf.rest_off[l];
            const int64_t ntf = s->tf.tf_off[l + 1] - s->tf.tf_off[l];
            if constexpr (MODE == MODE_ITER) {
                if (ntf) {
                    if (tm) tm->before(3);   // untagged: its workgroup size is fixed
                    const int ma = P.lvl_maxa[l];
#define PCFR_TF_LAUNCH(MA)                                                                                          \
    hipLaunchKernelGGL((k_backward_tf<T, MA>), dim3((unsigned)ntf), dim3(kBlock), s->tf.lds, stream,                  \
                       s->at<DNode>(L.off_tfrec) + s->tf.tf_off[l], nodes, Hp, R, S, Mp, reach, cfv, st,              \
                       s->at<uint16_t>(L.off_hc), s->at<int32_t>(L.off_coff), s->at<int16_t>(L.off_chands),           \
                       (int)L.chand_stride, s->at<int16_t>(L.off_sd), (int64_t)L.sd_stride, s->at<int32_t>(L.off_sdn), \
                       rootd, upd, nzs, (int)s->tf.val_off)
                    if (ma <= 3) PCFR_TF_LAUNCH(3);
                    else if (ma <= 6) PCFR_TF_LAUNCH(6);
                    else if (ma <= 8) PCFR_TF_LAUNCH(8);
                    else PCFR_TF_LAUNCH(12);
#undef PCFR_TF_LAUNCH
                    if (tm) tm->after();
                }
            }
        }
        if (lcnt) {
            const int64_t threads = lcnt * groups;
            dim3 grid((unsigned)((threads + bs - 1) / bs));
            if (tm) tm->before(3, 1000 + l);
            PCFR_BUCKET(k_backward, l, grid, dim3(bs), 0, stream, lrec, (int)lcnt, Hp, R, S, Mp,
                        reach, cfv, st, s->at<uint16_t>(L.off_hc), rootd, upd, iso, nzs);
            if (tm) tm->after();
        }
        l--;
    }
#undef PCFR_BUCKET_MA
#undef PCFR_BUCKET
    return hip_check(hipGetLastError(), "kernel launch");
}

// One iteration: one sweep updating both players, or with alternating
// updates a sweep for player 0 then one for player 1 (same t).
template <typename T>
static int32_t enqueue_iteration(pcfr_solver* s, hipStream_t stream, LaunchTimer* tm = nullptr) {
    if (!s->cfg.alternating) return enqueue_sweep<T, MODE_ITER>(s, stream, tm);
    int32_t rc = enqueue_sweep<T, MODE_ITER>(s, stream, tm, 0, true);
    if (rc) return rc;
    return enqueue_sweep<T, MODE_ITER>(s, stream, tm, 1, false);
}

template <int MODE>
static int32_t sweep(pcfr_solver* s, hipStream_t stream) {
    if (MODE == MODE_ITER)
        return s->cfg.dtype == PCFR_F64 ? enqueue_iteration<double>(s, stream) : enqueue_iteration<float>(s, stream);
    return s->cfg.dtype == PCFR_F64 ? enqueue_sweep<double, MODE>(s, stream) : enqueue_sweep<float, MODE>(s, stream);
}
template <int MODE>
static int32_t sweep(pcfr_solver* s) { return sweep<MODE>(s, s->stream); }

// Terminal fusion plan: every decision node at a backward level swept by
// per-node launches (not level-fused) with one or two fold or showdown
// children evaluates them itself (k_backward_tf); the other nodes of the
// level stay with k_backward and the other terminals with k_terminal.
template <typename T>
static int32_t tf_attrs(size_t lds) {
    if (lds <= 65536) return PCFR_OK;
    const void* ks[4] = {reinterpret_cast<const void*>(&k_backward_tf<T, 3>), reinterpret_cast<const void*>(&k_backward_tf<T, 6>),
                         reinterpret_cast<const void*>(&k_backward_tf<T, 8>), reinterpret_cast<const void*>(&k_backward_tf<T, 12>)};
    for (const void* k : ks) HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return PCFR_OK;
}

static int32_t make_tf_plan(pcfr_solver* s) {
    const Prepared& P = s->P;
    const Plan& L = s->L;
    auto& tf = s->tf;
    tf.on = false;
    tf.tf_off.assign(P.levels + 1, 0);
    tf.rest_off.assign(P.levels + 1, 0);
    if (!s->tf_enabled || P.preflop) return PCFR_OK;   // preflop folds run over classes (k_fold_class)
    const int64_t groups = L.Hp / 4, fuse = s->sched.fuse_threads;
    std::vector<DNode> tf_rec, rest_rec;
    std::vector<char> handled(P.nodes.size(), 0);
    for (int l = 0; l < P.levels; l++) {
        tf.tf_off[l] = (int64_t)tf_rec.size();
        tf.rest_off[l] = (int64_t)rest_rec.size();
        const bool fused = (P.fwd_off[l + 1] - P.fwd_off[l]) * groups <= fuse;
        for (int64_t k = P.fwd_off[l]; k < P.fwd_off[l + 1]; k++) {
            const DNode& d = P.fwd_rec[k];
            int nt = 0;
            if (!fused && d.type == PCFR_NODE_DECISION)
                for (int a = 0; a < d.n_child; a++) {
                    const int32_t t = P.nodes[d.first_child + a].type;
                    nt += t == PCFR_NODE_FOLD || t == PCFR_NODE_SHOWDOWN;
                }
            if (nt >= 1 && nt <= 2) {
                tf_rec.push_back(d);
                for (int a = 0; a < d.n_child; a++) handled[d.first_child + a] = 1;
            } else {
                rest_rec.push_back(d);
            }
        }
    }
    tf.tf_off[P.levels] = (int64_t)tf_rec.size();
    tf.rest_off[P.levels] = (int64_t)rest_rec.size();
    std::vector<int32_t> term;
    for (int32_t x : P.folds) if (!handled[x]) term.push_back(x);
    tf.n_fold = (int64_t)term.size();
    for (int32_t x : P.shows) if (!handled[x]) term.push_back(x);
    tf.n_show = (int64_t)term.size() - tf.n_fold;
    if (tf_rec.empty()) return PCFR_OK;
    tf.val_off = (L.lds_bytes + 15) & ~(size_t)15;
    tf.lds = tf.val_off + 4 * L.Hp * L.esz;
    if (tf.lds > 160 * 1024) return PCFR_OK;   // does not fit: stay with k_terminal
    int32_t rc = L.esz == 8 ? tf_attrs<double>(tf.lds) : tf_attrs<float>(tf.lds);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(s->ws + L.off_tfrec, tf_rec.data(), sizeof(DNode) * tf_rec.size(), hipMemcpyHostToDevice, s->stream));
    if (!rest_rec.empty())
        HIPCHK(hipMemcpyAsync(s->ws + L.off_tfrest, rest_rec.data(), sizeof(DNode) * rest_rec.size(), hipMemcpyHostToDevice,
                              s->stream));
    std::vector<DNode> term_rec;
    for (int32_t x : term) term_rec.push_back(P.nodes[x]);
    if (!term.empty()) {
        HIPCHK(hipMemcpyAsync(s->ws + L.off_tfterm, term.data(), sizeof(int32_t) * term.size(), hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(s->ws + L.off_tftermrec, term_rec.data(), sizeof(DNode) * term_rec.size(),
                              hipMemcpyHostToDevice, s->stream));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    tf.on = true;
    return PCFR_OK;
}

// One iteration's launch sequence, captured once on a private stream (the
// caller's may be the legacy default stream, which cannot be captured) and
// replayed on the caller's stream.
static int32_t build_graph(pcfr_solver* s) {
    int32_t rc0 = make_tf_plan(s);
    if (rc0) return rc0;
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { (void)hipStreamDestroy(cs); return hip_check(e, "hipStreamBeginCapture"); }
    int32_t rc = sweep<MODE_ITER>(s, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc != PCFR_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    HIPCHK(e);
    s->graph_def = g;
    HIPCHK(hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0));
    return PCFR_OK;
}

// Copy a [rows][Hp] device block (solver dtype) of subgame g into host doubles [rows][1326].
static int32_t fetch_hands(pcfr_solver* s, const void* dev, int rows, double* out, int32_t g = 0) {
    const Plan& L = s->L;
    std::vector<char> buf(L.esz * rows * L.Hp);
    HIPCHK(hipMemcpyAsync(buf.data(), dev, buf.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int r = 0; r < rows; r++)
        for (int k = 0; k < kCombos; k++) {
            int h = s->P.combo_hand[g][k];
            double v = 0;
            if (h >= 0) {
                size_t i = (size_t)r * L.Hp + h;
                v = L.esz == 8 ? reinterpret_cast<double*>(buf.data())[i] : (double)reinterpret_cast<float*>(buf.data())[i];
            }
            out[(size_t)r * kCombos + k] = v;
        }
    return PCFR_OK;
}

}  // namespace pcfr

namespace pcfr {

// ------------------------------------------------------------ schedules
// Tuned workgroup sizes are cached per size bucket: (phase, dtype, action
// bucket, floor(log2(threads of the launch))).  A new solver takes the cached
// size of each of its launches' buckets, 256 where none was tuned.
static std::mutex g_sched_mu;
static std::map<std::tuple<int, int, int, int>, int> g_sched_cache;

static int log2_bucket(int64_t x) {
    int b = 0;
    while (b < 62 && (int64_t(1) << (b + 1)) <= x) b++;
    return b;
}
static int action_bucket(int ma) { return ma <= 3 ? 3 : ma <= 6 ? 6 : ma <= 8 ? 8 : 12; }

static std::tuple<int, int, int, int> sched_key(const pcfr_solver* s, int phase, int l) {
    const Prepared& P = s->P;
    const int64_t cnt = phase == 0 ? P.dec_off[l + 1] - P.dec_off[l] : P.fwd_off[l + 1] - P.fwd_off[l];
    return std::make_tuple(phase, (int)s->L.esz, action_bucket(P.lvl_maxa[l]), log2_bucket(cnt * (s->L.Hp / 4)));
}

static void init_sched(pcfr_solver* s) {
    const int levels = s->P.levels;
    s->sched.fwd_block.assign(levels, 256);
    s->sched.bwd_block.assign(levels, 256);
    std::lock_guard<std::mutex> lk(g_sched_mu);
    for (int l = 0; l < levels; l++) {
        auto f = g_sched_cache.find(sched_key(s, 0, l));
        if (f != g_sched_cache.end()) s->sched.fwd_block[l] = f->second;
        auto b = g_sched_cache.find(sched_key(s, 1, l));
        if (b != g_sched_cache.end()) s->sched.bwd_block[l] = b->second;
    }
}

static int32_t check_cfg(const pcfr_solver_cfg* cfg) {
    if (cfg->dtype != PCFR_F32 && cfg->dtype != PCFR_F64) { set_error("dtype must be PCFR_F32 or PCFR_F64"); return PCFR_E_INVALID_ARG; }
    if (cfg->variant != PCFR_DCFR && cfg->variant != PCFR_CFRPLUS && cfg->variant != PCFR_PCFRPLUS) {
        set_error("variant must be PCFR_DCFR, PCFR_CFRPLUS or PCFR_PCFRPLUS");
        return PCFR_E_INVALID_ARG;
    }
    if (cfg->alternating != 0 && cfg->alternating != 1) { set_error("alternating must be 0 or 1"); return PCFR_E_INVALID_ARG; }
    if (cfg->suit_iso != 0 && cfg->suit_iso != 1) { set_error("suit_iso must be 0 or 1"); return PCFR_E_INVALID_ARG; }
    if (!std::isfinite(cfg->alpha) || !std::isfinite(cfg->beta) || !std::isfinite(cfg->gamma)) {
        set_error("alpha, beta, gamma must be finite");
        return PCFR_E_INVALID_ARG;
    }
    if (!(cfg->threshold >= 0.0 && cfg->threshold < 1.0 / 12)) {
        set_error("threshold must lie in [0, 1/12)");
        return PCFR_E_INVALID_ARG;
    }
    if (cfg->prune != 0 && cfg->prune != 1) { set_error("prune must be 0 or 1"); return PCFR_E_INVALID_ARG; }
    return PCFR_OK;
}

static int32_t workspace_for(const pcfr_tree* const* trees, int32_t n, const pcfr_solver_cfg* cfg, size_t* bytes) {
    if (!trees || n < 1 || !cfg || !bytes) { set_error("null argument or empty batch"); return PCFR_E_INVALID_ARG; }
    int32_t rc = check_cfg(cfg);
    if (rc) return rc;
    std::vector<const Tree*> tv;
    int64_t rows = 0;
    for (int32_t i = 0; i < n; i++) {
        if (!trees[i]) { set_error("null tree"); return PCFR_E_INVALID_ARG; }
        tv.push_back(&trees[i]->t);
        rows += trees[i]->t.rows;
    }
    Prepared P;
    try { rc = prepare(tv, P); } catch (const std::bad_alloc&) { set_error("out of host memory"); return PCFR_E_OUT_OF_MEMORY; }
    if (rc != PCFR_OK) return rc;
    Plan L;
    make_plan(P, rows, cfg->dtype, cfg->variant, cfg->suit_iso != 0, L);
    *bytes = L.total;
    return PCFR_OK;
}

static int32_t create_impl(const pcfr_tree* const* trees, int32_t n, const pcfr_solver_cfg* cfg, const double* ranges,
                           void* workspace, size_t workspace_bytes, void* stream, pcfr_solver** out) {
    if (!trees || n < 1 || !cfg || !ranges || !workspace || !out) { set_error("null argument or empty batch"); return PCFR_E_INVALID_ARG; }
    int32_t rc = check_cfg(cfg);
    if (rc) return rc;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) { set_error("workspace must be 256-byte aligned"); return PCFR_E_INVALID_ARG; }
    pcfr_solver* s = new (std::nothrow) pcfr_solver;
    if (!s) { set_error("out of host memory"); return PCFR_E_OUT_OF_MEMORY; }
    std::unique_ptr<pcfr_solver> guard(s);
    int64_t rows = 0;
    try {
        for (int32_t i = 0; i < n; i++) {
            if (!trees[i]) { set_error("null tree"); return PCFR_E_INVALID_ARG; }
            s->trees.push_back(trees[i]->t);
            rows += trees[i]->t.rows;
        }
        std::vector<const Tree*> tv;
        for (auto& t : s->trees) tv.push_back(&t);
        if (cfg->suit_iso) {
            for (const Tree* t : tv)
                if (t->root_mask == 0) {
                    set_error("preflop roots are solved over hand classes already; suit_iso is for boards");
                    return PCFR_E_UNSUPPORTED;
                }
            rc = suit_iso_map(tv, ranges, s->iso);
            if (rc != PCFR_OK) return rc;
        }
        rc = prepare(tv, s->P, cfg->suit_iso ? &s->iso : nullptr);
        if (rc != PCFR_OK) return rc;
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return PCFR_E_OUT_OF_MEMORY;
    }
    s->cfg = *cfg;
    make_plan(s->P, rows, cfg->dtype, cfg->variant, cfg->suit_iso != 0, s->L);
    const Plan& L = s->L;
    const Prepared& P = s->P;
    if (workspace_bytes < L.total) { set_error("workspace smaller than the size the library asked for"); return PCFR_E_OUT_OF_MEMORY; }
    if (L.lds_bytes > 160 * 1024) { set_error("hand count too large for the terminal kernel's LDS"); return PCFR_E_TOO_LARGE; }
    if (L.lds_bytes > 65536) {
        // gfx950 gives a workgroup up to 160 KB of LDS; dynamic sizes above 64 KB must be declared
        const void* ks[2] = {cfg->dtype == PCFR_F64 ? reinterpret_cast<const void*>(&k_terminal<double, 0>)
                                                    : reinterpret_cast<const void*>(&k_terminal<float, 0>),
                             cfg->dtype == PCFR_F64 ? reinterpret_cast<const void*>(&k_terminal<double, 1>)
                                                    : reinterpret_cast<const void*>(&k_terminal<float, 1>)};
        for (const void* k : ks) {
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
            if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
        }
    }
    // ranges and the joint mass of compatible pairs: r0 . (total1 - per-card sums + r1)
    const ComboTable& cc = combos();
    s->ranges.assign((size_t)n * 2 * kCombos, 0.0);
    s->pair_mass.assign(n, 0.0);
    for (int32_t g = 0; g < n; g++) {
        double mass[2] = {0, 0};
        double* rg = &s->ranges[(size_t)g * 2 * kCombos];
        for (int p = 0; p < 2; p++)
            for (int k = 0; k < kCombos; k++) {
                double v = ranges[((size_t)g * 2 + p) * kCombos + k];
                if (!std::isfinite(v) || v < 0) { set_error("ranges must be finite and >= 0"); return PCFR_E_INVALID_ARG; }
                if (P.combo_hand[g][k] < 0 && v != 0) { set_error("range mass on a combo blocked by the board"); return PCFR_E_INVALID_ARG; }
                rg[p * kCombos + k] = v;
                mass[p] += v;
            }
        double card1[52] = {0};
        for (int k = 0; k < kCombos; k++) { card1[cc.hi[k]] += rg[kCombos + k]; card1[cc.lo[k]] += rg[kCombos + k]; }
        double z = 0;
        for (int k = 0; k < kCombos; k++) {
            if (rg[k] == 0) continue;
            z += rg[k] * (mass[1] - card1[cc.hi[k]] - card1[cc.lo[k]] + rg[kCombos + k]);
        }
        s->pair_mass[g] = z;
        if (!(z > 0)) { set_error("no compatible pair of hands carries mass"); return PCFR_E_INVALID_ARG; }
        if (P.preflop)
            for (int p = 0; p < 2; p++)
                for (int k = 0; k < kCombos; k++)
                    if (rg[p * kCombos + k] != rg[p * kCombos + P.hand_combo[g][P.combo_hand[g][k]]]) {
                        set_error("a preflop root needs suit-symmetric ranges (equal on the combos of each hand class)");
                        return PCFR_E_INVALID_ARG;
                    }
    }
    s->stream = reinterpret_cast<hipStream_t>(stream);
    s->ws = reinterpret_cast<char*>(workspace);
    HIPCHK(hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    auto up = [&](size_t off, const void* src, size_t bytes) -> int32_t {
        if (!bytes) return PCFR_OK;
        return hip_check(hipMemcpyAsync(s->ws + off, src, bytes, hipMemcpyHostToDevice, s->stream), "upload");
    };
    if ((rc = up(L.off_nodes, P.nodes.data(), sizeof(DNode) * P.nodes.size()))) return rc;
    if ((rc = up(L.off_fwd, P.fwd_rec.data(), sizeof(DNode) * P.fwd_rec.size()))) return rc;
    if ((rc = up(L.off_dec, P.dec_rec.data(), sizeof(DNode) * P.dec_rec.size()))) return rc;
    if ((rc = up(L.off_fwdoff, P.fwd_off.data(), sizeof(int64_t) * P.fwd_off.size()))) return rc;
    if ((rc = up(L.off_decoff, P.dec_off.data(), sizeof(int64_t) * P.dec_off.size()))) return rc;
    if ((rc = up(L.off_term, P.term.data(), sizeof(int32_t) * P.term.size()))) return rc;
    {
        std::vector<DNode> tr;
        for (int32_t x : P.term) tr.push_back(P.nodes[x]);
        if ((rc = up(L.off_termrec, tr.data(), sizeof(DNode) * tr.size()))) return rc;
    }
    if ((rc = up(L.off_hc, P.hcards.data(), sizeof(uint16_t) * P.hcards.size()))) return rc;
    if ((rc = up(L.off_coff, P.coff.data(), sizeof(int32_t) * P.coff.size()))) return rc;
    if ((rc = up(L.off_chands, P.chands.data(), sizeof(int16_t) * P.chands.size()))) return rc;
    if ((rc = up(L.off_sd, P.sd.data(), sizeof(int16_t) * L.n_boards * L.sd_stride))) return rc;
    if ((rc = up(L.off_sdn, P.sdn.data(), sizeof(int32_t) * L.n_boards))) return rc;
    std::vector<int32_t> roots(n);
    for (int32_t g = 0; g < n; g++) roots[g] = (int32_t)P.root_node[g];
    if ((rc = up(L.off_roots, roots.data(), sizeof(int32_t) * n))) return rc;
    if (cfg->suit_iso) {
        std::vector<int32_t> cmap(2 * (size_t)L.N);
        for (int64_t i = 0; i < L.N; i++) { cmap[2 * i] = s->iso.src[i]; cmap[2 * i + 1] = s->iso.perm[i]; }
        std::vector<int16_t> hmap((size_t)24 * L.Hp * n);
        for (int32_t g = 0; g < n; g++)
            suit_hand_maps(P.hand_combo[g], P.combo_hand[g], s->iso.group[g], L.Hp, hmap.data() + (size_t)g * 24 * L.Hp);
        if ((rc = up(L.off_cmap, cmap.data(), sizeof(int32_t) * cmap.size()))) return rc;
        if ((rc = up(L.off_hmap, hmap.data(), sizeof(int16_t) * hmap.size()))) return rc;
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    {
        // per-subgame tables of the leaf-network sample builder
        std::vector<float> ps(2 * n);
        std::vector<uint8_t> boards((size_t)n * 52, 0);
        std::vector<int16_t> c2h((size_t)n * kCombos);
        for (int32_t g = 0; g < n; g++) {
            const pcfr_tree_spec& sp = s->trees[g].spec;
            const int64_t eff = std::min(sp.stack[0], sp.stack[1]);
            ps[2 * g] = (float)sp.pot;
            ps[2 * g + 1] = (float)((double)eff / (double)sp.pot);
            for (int c = 0; c < 52; c++) boards[(size_t)g * 52 + c] = (P.root_mask[g] >> c & 1ull) ? 1 : 0;
            for (int k = 0; k < kCombos; k++) c2h[(size_t)g * kCombos + k] = (int16_t)P.combo_hand[g][k];
        }
        const size_t o1 = align256(sizeof(float) * 2 * n), o2 = o1 + align256((size_t)n * 52);
        if ((rc = up(L.off_samp, ps.data(), sizeof(float) * ps.size()))) return rc;
        if ((rc = up(L.off_samp + o1, boards.data(), boards.size()))) return rc;
        if ((rc = up(L.off_samp + o2, c2h.data(), sizeof(int16_t) * c2h.size()))) return rc;
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    {
        // per subgame: combo -> hand, hand -> combo, next cards, root board
        std::vector<int16_t> c2h((size_t)n * kComboPad, -1), h2c((size_t)n * L.Hp, -1);
        for (int32_t g = 0; g < n; g++) {
            for (int k = 0; k < kCombos; k++) c2h[(size_t)g * kComboPad + k] = (int16_t)P.combo_hand[g][k];
            for (int64_t h = 0; h < P.Hs[g]; h++) h2c[(size_t)g * L.Hp + h] = (int16_t)P.hand_combo[g][h];
        }
        std::vector<int32_t> grp;
        int64_t n_grp_allin = 0;
        equity_groups(P, L.eq_J, grp, n_grp_allin);
        if ((rc = up(L.off_c2h, c2h.data(), sizeof(int16_t) * c2h.size()))) return rc;
        if ((rc = up(L.off_h2c, h2c.data(), sizeof(int16_t) * h2c.size()))) return rc;
        if ((rc = up(L.off_next, P.next_all.data(), P.next_all.size()))) return rc;
        if ((rc = up(L.off_b4, P.board4s.data(), sizeof(int32_t) * P.board4s.size()))) return rc;
        if ((rc = up(L.off_eqgrp, grp.data(), sizeof(int32_t) * grp.size()))) return rc;
        if ((rc = up(L.off_nsub, P.net_sub.data(), sizeof(int32_t) * P.net_sub.size()))) return rc;
        if ((rc = up(L.off_eq, P.eq_leaves.data(), sizeof(int32_t) * P.eq_leaves.size()))) return rc;
        if ((rc = up(L.off_eqpay, P.eq_pay.data(), sizeof(double) * P.eq_pay.size()))) return rc;
        if ((rc = up(L.off_net, P.net_leaves.data(), sizeof(int32_t) * P.net_leaves.size()))) return rc;
        if ((rc = up(L.off_spr, P.net_spr.data(), sizeof(float) * P.net_spr.size()))) return rc;
        if ((rc = up(L.off_potk, P.net_potk.data(), sizeof(double) * P.net_potk.size()))) return rc;
        if ((rc = up(L.off_hoff, P.hoff.data(), sizeof(int32_t) * P.hoff.size()))) return rc;
        if ((rc = up(L.off_hlist, P.hlist.data(), sizeof(int16_t) * P.hlist.size()))) return rc;
        if (P.preflop) {
            if ((rc = up(L.off_ncompat, P.ncompat.data(), P.ncompat.size()))) return rc;
            if ((rc = up(L.off_flops, P.flops.data(), P.flops.size()))) return rc;
            if ((rc = up(L.off_orbit, P.flop_orbit.data(), sizeof(int32_t) * P.flop_orbit.size()))) return rc;
        }
        HIPCHK(hipStreamSynchronize(s->stream));
        // pairwise equity table of each subgame holding depth-limit leaves
        for (int32_t g = 0; g < n; g++) {
            if (P.et_slot[g] < 0) continue;
            const int64_t Hg = P.Hs[g];
            std::vector<double> E;
            std::vector<char> et;
            try {
                equity_matrix(P.root_mask[g], P.hand_combo[g], E);
                et.assign(L.esz * L.Hp * L.Hp, 0);
            } catch (const std::bad_alloc&) {
                set_error("out of host memory for the equity table");
                return PCFR_E_OUT_OF_MEMORY;
            }
            for (int64_t h = 0; h < Hg; h++)
                for (int64_t o = 0; o < Hg; o++) {
                    const double v = E[(size_t)h * Hg + o];
                    const size_t i = (size_t)o * L.Hp + h;   // transposed
                    if (L.esz == 8) reinterpret_cast<double*>(et.data())[i] = v;
                    else reinterpret_cast<float*>(et.data())[i] = (float)v;
                }
            if ((rc = up(L.off_et + L.esz * L.Hp * L.Hp * (size_t)P.et_slot[g], et.data(), et.size()))) return rc;
            HIPCHK(hipStreamSynchronize(s->stream));
        }
    }
    {
        IterState st{};
        st.variant = cfg->variant;
        st.alpha = cfg->alpha;
        st.beta = cfg->beta;
        st.gamma = cfg->gamma;
        st.thr0 = cfg->threshold;
        if ((rc = up(L.off_state, &st, sizeof(st)))) return rc;
        // pruning flags: the roots' reach slots hold the ranges, set once
        std::vector<int32_t> nzs(2 * (size_t)P.n_sub + L.rows, 0);
        for (int64_t i = 0; i < 2 * (int64_t)P.n_sub; i++) nzs[i] = 1;
        if ((rc = up(L.off_nzs, nzs.data(), sizeof(int32_t) * nzs.size()))) return rc;
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    HIPCHK(hipMemsetAsync(s->ws + L.off_R, 0, L.esz * L.rows * L.Hp, s->stream));
    HIPCHK(hipMemsetAsync(s->ws + L.off_S, 0, L.esz * L.rows * L.Hp, s->stream));
    if (cfg->variant == PCFR_PCFRPLUS) HIPCHK(hipMemsetAsync(s->ws + L.off_M, 0, L.esz * L.rows * L.Hp, s->stream));
    HIPCHK(hipMemsetAsync(s->ws + L.off_reach, 0, L.esz * L.slots * L.Hp, s->stream));
    HIPCHK(hipMemsetAsync(s->ws + L.off_cfv, 0, L.esz * L.N * 2 * L.Hp, s->stream));
    HIPCHK(hipMemsetAsync(s->ws + L.off_root, 0, L.esz * 2 * L.Hp * n, s->stream));
    // root reach = ranges in hand order, slots 2g and 2g + 1 (never written again)
    {
        std::vector<char> rr(L.esz * 2 * L.Hp * n, 0);
        for (int32_t g = 0; g < n; g++)
            for (int p = 0; p < 2; p++)
                for (int64_t h = 0; h < P.Hs[g]; h++) {
                    double v = s->ranges[((size_t)g * 2 + p) * kCombos + P.hand_combo[g][h]];
                    size_t i = ((size_t)g * 2 + p) * L.Hp + h;
                    if (L.esz == 8) reinterpret_cast<double*>(rr.data())[i] = v;
                    else reinterpret_cast<float*>(rr.data())[i] = (float)v;
                }
        if ((rc = up(L.off_reach, rr.data(), rr.size()))) return rc;
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    init_sched(s);
    if ((rc = build_graph(s))) return rc;
    *out = guard.release();
    return PCFR_OK;
}

static int32_t strategy_impl(pcfr_solver* s, int32_t g, int32_t node, int32_t which, double* out) {
    if (!s || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if (which != PCFR_AVG && which != PCFR_CURRENT) { set_error("which must be PCFR_AVG or PCFR_CURRENT"); return PCFR_E_INVALID_ARG; }
    if (g < 0 || g >= s->P.n_sub) { set_error("subgame index out of range"); return PCFR_E_INVALID_ARG; }
    const int64_t nn = (int64_t)s->trees[g].nodes.size();
    if (node < 0 || node >= nn || s->trees[g].nodes[node].type != PCFR_NODE_DECISION) {
        set_error("node is not a decision node");
        return PCFR_E_INVALID_ARG;
    }
    // a node skipped by suit isomorphism: its representative's strategy with
    // hands relabelled, sigma_n(h) = sigma_rep(Pi^-1 h), Pi composed along
    // the chain of representatives
    int64_t gn = s->P.node_base[g] + node;
    int Pi = 0;
    while (!s->iso.skip.empty() && s->iso.skip[gn]) {
        if (s->iso.corr[gn] < 0 || s->iso.cperm[gn] < 0) {
            set_error("internal: a node skipped by suit isomorphism has no representative");
            return PCFR_E_STATE;
        }
        Pi = suit_perm_compose(Pi, s->iso.cperm[gn]);
        gn = s->iso.corr[gn];
    }
    const DNode& d = s->P.nodes[gn];
    const Plan& L = s->L;
    void* stage = s->ws + L.off_stage;
    dim3 grid((unsigned)((L.Hp + 255) / 256));
    if (L.esz == 8)
        hipLaunchKernelGGL((k_strategy<double>), grid, dim3(256), 0, s->stream,
                           s->at<double>(which == PCFR_AVG ? L.off_S : L.off_R),
                           (which == PCFR_CURRENT && s->cfg.variant == PCFR_PCFRPLUS) ? s->at<double>(L.off_M) : nullptr,
                           d.rs, d.n_child, (int)L.Hp,
                           which == PCFR_CURRENT ? 1 : 0, s->at<IterState>(L.off_state), (double*)stage);
    else
        hipLaunchKernelGGL((k_strategy<float>), grid, dim3(256), 0, s->stream,
                           s->at<float>(which == PCFR_AVG ? L.off_S : L.off_R),
                           (which == PCFR_CURRENT && s->cfg.variant == PCFR_PCFRPLUS) ? s->at<float>(L.off_M) : nullptr,
                           d.rs, d.n_child, (int)L.Hp,
                           which == PCFR_CURRENT ? 1 : 0, s->at<IterState>(L.off_state), (float*)stage);
    HIPCHK(hipGetLastError());
    int32_t rc = fetch_hands(s, stage, d.n_child, out, g);
    if (rc) return rc;
    for (int a = 0; a < d.n_child; a++)
        for (int k = 0; k < kCombos; k++)
            if (s->P.combo_hand[g][k] < 0) out[(size_t)a * kCombos + k] = 0;
    if (Pi != 0) {
        // out[a][k] = rep[a][Pi^-1 k]: combo Pi(j) takes the representative's combo j
        const ComboTable& cc = combos();
        std::vector<double> rep(out, out + (size_t)d.n_child * kCombos);
        for (int j = 0; j < kCombos; j++) {
            const int k = combo_of(suit_perm_card(Pi, cc.hi[j]), suit_perm_card(Pi, cc.lo[j]));
            for (int a = 0; a < d.n_child; a++) out[(size_t)a * kCombos + k] = rep[(size_t)a * kCombos + j];
        }
    }
    return PCFR_OK;
}

// A preflop tree's leaves have no exact value: iterating and evaluating need
// the flop-level network.
static int32_t leaves_ready(const pcfr_solver* s) {
    if (s->P.preflop && s->L.n_net && !s->net) {
        set_error("leaves at the flop deal need a leaf network (pcfr_solver_attach_leafnet)");
        return PCFR_E_STATE;
    }
    return PCFR_OK;
}

static int32_t root_cfv_impl(pcfr_solver* s, int32_t g, int32_t which, double* out, bool sweep_first) {
    if (!s || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if (g < 0 || g >= s->P.n_sub) { set_error("subgame index out of range"); return PCFR_E_INVALID_ARG; }
    const Plan& L = s->L;
    if (which == PCFR_CURRENT) return fetch_hands(s, s->ws + L.off_root + L.esz * 2 * L.Hp * (size_t)g, 2, out, g);
    if (which != PCFR_AVG) { set_error("which must be PCFR_AVG or PCFR_CURRENT"); return PCFR_E_INVALID_ARG; }
    if (sweep_first) {
        int32_t rc = leaves_ready(s);
        if (rc) return rc;
        rc = sweep<MODE_EV>(s);
        if (rc) return rc;
    }
    return fetch_hands(s, s->ws + L.off_cfv + L.esz * 2 * L.Hp * (size_t)s->P.root_node[g], 2, out, g);
}

// Counterfactual values of every node of one subgame, combo-indexed (zero on
// combos the root board blocks): out[(node * 2 + p) * 1326 + k].
template <typename T>
__global__ void k_node_values(const T* __restrict__ cfv, int64_t node0, int Hp, const int16_t* __restrict__ c2h,
                              double* __restrict__ out) {
    const int64_t row = blockIdx.x;   // node * 2 + player within the subgame
    const T* src = cfv + (node0 * 2 + row) * Hp;
    for (int k = threadIdx.x; k < kCombos; k += blockDim.x) {
        const int h = c2h[k];
        out[row * kCombos + k] = h >= 0 ? (double)src[h] : 0.0;
    }
}

// Values of every node of subgame g under the average strategy profile, into
// device memory [n_nodes][2][1326].
static int32_t node_values_impl(pcfr_solver* s, int32_t g, double* out) {
    if (!s || !out) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if (g < 0 || g >= s->P.n_sub) { set_error("subgame index out of range"); return PCFR_E_INVALID_ARG; }
    if (s->cfg.suit_iso) { set_error("node values are not kept for subtrees solved through suit isomorphism"); return PCFR_E_UNSUPPORTED; }
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, out) != hipSuccess) {
        (void)hipGetLastError();
        set_error("out must be device memory");
        return PCFR_E_INVALID_ARG;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) { set_error("out must be device memory"); return PCFR_E_INVALID_ARG; }
    const Plan& L = s->L;
    const int64_t n0 = s->P.node_base[g];
    const int64_t nn = (g + 1 < s->P.n_sub ? s->P.node_base[g + 1] : (int64_t)s->P.nodes.size()) - n0;
    int32_t rc = sweep<MODE_EV>(s);
    if (rc) return rc;
    std::vector<int16_t> c2h(kCombos);
    for (int k = 0; k < kCombos; k++) c2h[k] = (int16_t)s->P.combo_hand[g][k];
    void* dc = nullptr;
    HIPCHK(hipMalloc(&dc, sizeof(int16_t) * kCombos));
    hipError_t e = hipMemcpyAsync(dc, c2h.data(), sizeof(int16_t) * kCombos, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && nn > 0) {
        if (L.esz == 8)
            hipLaunchKernelGGL((k_node_values<double>), dim3((unsigned)(2 * nn)), dim3(256), 0, s->stream,
                               s->at<double>(L.off_cfv), n0, (int)L.Hp, (const int16_t*)dc, out);
        else
            hipLaunchKernelGGL((k_node_values<float>), dim3((unsigned)(2 * nn)), dim3(256), 0, s->stream,
                               s->at<float>(L.off_cfv), n0, (int)L.Hp, (const int16_t*)dc, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(dc);
    return e == hipSuccess ? PCFR_OK : hip_check(e, "node values");
}

// Best-response sweep for every subgame, then per subgame
// (BR_0 + BR_1) / 2 per unit of joint pair mass.
static int32_t exploitability_impl(pcfr_solver* s, double* chips, double* br) {
    int32_t rc = leaves_ready(s);
    if (rc) return rc;
    rc = sweep<MODE_BR>(s);
    if (rc) return rc;
    const int32_t n = s->P.n_sub;
    std::vector<double> v(2 * kCombos);
    for (int32_t g = 0; g < n; g++) {
        if ((rc = root_cfv_impl(s, g, PCFR_AVG, v.data(), false))) return rc;
        const double* rg = &s->ranges[(size_t)g * 2 * kCombos];
        double b[2] = {0, 0};
        for (int p = 0; p < 2; p++)
            for (int k = 0; k < kCombos; k++) b[p] += rg[p * kCombos + k] * v[(size_t)p * kCombos + k];
        b[0] /= s->pair_mass[g];
        b[1] /= s->pair_mass[g];
        if (!std::isfinite(b[0]) || !std::isfinite(b[1])) { set_error("non-finite best-response value"); return PCFR_E_NUMERIC; }
        chips[g] = 0.5 * (b[0] + b[1]);
        if (br) { br[2 * g] = b[0]; br[2 * g + 1] = b[1]; }
    }
    return PCFR_OK;
}

static int32_t rebuild_graph(pcfr_solver* s) {
    if (s->graph) { (void)hipGraphExecDestroy(s->graph); s->graph = nullptr; }
    if (s->graph_def) { (void)hipGraphDestroy(s->graph_def); s->graph_def = nullptr; }
    return build_graph(s);
}

// Zero the iterate (t, R, S, m, stored root values): the state of a new solver.
static int32_t reset_state(pcfr_solver* s) {
    const Plan& L = s->L;
    const int64_t t0 = 0;
    HIPCHK(hipMemcpyAsync(s->ws + L.off_state + offsetof(IterState, t), &t0, sizeof(t0), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemsetAsync(s->ws + L.off_R, 0, L.esz * L.rows * L.Hp, s->stream));
    HIPCHK(hipMemsetAsync(s->ws + L.off_S, 0, L.esz * L.rows * L.Hp, s->stream));
    if (s->cfg.variant == PCFR_PCFRPLUS) HIPCHK(hipMemsetAsync(s->ws + L.off_M, 0, L.esz * L.rows * L.Hp, s->stream));
    HIPCHK(hipMemsetAsync(s->ws + L.off_root, 0, L.esz * 2 * L.Hp * s->P.n_sub, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->t_host = 0;
    return PCFR_OK;
}

// Average ms per iteration of n graph replays (after one untimed replay).
static int32_t time_replays(pcfr_solver* s, int32_t n, double* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipGraphLaunch(s->graph, s->stream));
    HIPCHK(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) { (void)hipEventDestroy(a); return hip_check(e, "hipEventCreate"); }
    e = hipEventRecord(a, s->stream);
    for (int32_t i = 0; i < n && e == hipSuccess; i++) e = hipGraphLaunch(s->graph, s->stream);
    if (e == hipSuccess) e = hipEventRecord(b, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    HIPCHK(e);
    *ms = (double)t / std::max(n, 1);
    return PCFR_OK;
}

// Autotuner of the level sweeps: every level's forward and backward launch is
// timed at each candidate workgroup size over `reps` iterations (per-launch
// events), the fastest size per launch is kept and cached for its size
// bucket, the graph is captured again, and the state is reset to t = 0.
// Persistent launch (k_iterate_persistent): n iterations in one cooperative launch.
template <typename T, int MAXA>
static const void* persist_kernel() {
    return reinterpret_cast<const void*>(&k_iterate_persistent<T, MAXA>);
}
static const void* persist_kernel_for(int dtype, int maxa) {
    const bool d = dtype == PCFR_F64;
    if (maxa <= 3) return d ? persist_kernel<double, 3>() : persist_kernel<float, 3>();
    if (maxa <= 6) return d ? persist_kernel<double, 6>() : persist_kernel<float, 6>();
    if (maxa <= 8) return d ? persist_kernel<double, 8>() : persist_kernel<float, 8>();
    return d ? persist_kernel<double, 12>() : persist_kernel<float, 12>();
}

static int32_t set_launch_impl(pcfr_solver* s, int32_t mode) {
    if (mode == PCFR_LAUNCH_GRAPH) { s->launch_mode = mode; return PCFR_OK; }
    if (mode != PCFR_LAUNCH_PERSISTENT) { set_error("unknown launch mode"); return PCFR_E_INVALID_ARG; }
    const Plan& L = s->L;
    if (L.n_eq || L.n_net || s->net) { set_error("the persistent launch serves trees without depth-limit leaves"); return PCFR_E_UNSUPPORTED; }
    if (s->cfg.alternating || s->cfg.suit_iso) {
        set_error("the persistent launch runs simultaneous updates without suit isomorphism");
        return PCFR_E_UNSUPPORTED;
    }
    int maxa = 1;
    for (int32_t v : s->P.lvl_maxa) maxa = std::max(maxa, v);
    const void* k = persist_kernel_for(s->cfg.dtype, maxa);
    if (L.lds_bytes > 65536)
        HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes));
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) { set_error("the device does not support cooperative launches"); return PCFR_E_UNSUPPORTED; }
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, L.lds_bytes));
    if (per_cu < 1 || cus < 1) { set_error("the persistent kernel does not fit a compute unit"); return PCFR_E_UNSUPPORTED; }
    s->persist_grid = per_cu * cus;
    s->persist_maxa = maxa;
    s->launch_mode = mode;
    return PCFR_OK;
}

template <typename T>
static int32_t persist_launch(pcfr_solver* s, int32_t iters) {
    const Plan& L = s->L;
    const Prepared& P = s->P;
    PersistArgs a{};
    a.nodes = s->at<DNode>(L.off_nodes);
    a.dec_rec = s->at<DNode>(L.off_dec);
    a.fwd_rec = s->at<DNode>(L.off_fwd);
    a.dec_off = s->at<int64_t>(L.off_decoff);
    a.fwd_off = s->at<int64_t>(L.off_fwdoff);
    a.term = s->at<int32_t>(L.off_term);
    a.hcards = s->at<uint16_t>(L.off_hc);
    a.coff = s->at<int32_t>(L.off_coff);
    a.chands = s->at<int16_t>(L.off_chands);
    a.sd = s->at<int16_t>(L.off_sd);
    a.sdn = s->at<int32_t>(L.off_sdn);
    a.R = s->at<T>(L.off_R);
    a.S = s->at<T>(L.off_S);
    a.Mp = s->cfg.variant == PCFR_PCFRPLUS ? s->at<T>(L.off_M) : nullptr;
    a.reach = s->at<T>(L.off_reach);
    a.cfv = s->at<T>(L.off_cfv);
    a.root = s->at<T>(L.off_root);
    a.st = s->at<IterState>(L.off_state);
    a.nzs = s->cfg.prune ? s->at<int32_t>(L.off_nzs) : nullptr;
    a.n_slots = (int32_t)(2 * P.n_sub + L.rows);
    a.sd_stride = (int64_t)L.sd_stride;
    a.levels = P.levels;
    a.Hp = (int32_t)L.Hp;
    a.cbase = 2 * P.n_sub;
    a.n_term = (int32_t)(P.folds.size() + P.shows.size());
    a.chand_stride = (int32_t)L.chand_stride;
    a.iters = iters;
    void* params[] = {&a};
    const void* k = persist_kernel_for(s->cfg.dtype, s->persist_maxa);
    HIPCHK(hipLaunchCooperativeKernel(k, dim3((unsigned)s->persist_grid), dim3(kBlock), params, (unsigned)L.lds_bytes,
                                      s->stream));
    return PCFR_OK;
}

static int32_t autotune_impl(pcfr_solver* s, int32_t reps, double* ms_before, double* ms_after) {
    if (!s || reps < 1 || !ms_before || !ms_after) { set_error("null argument or reps < 1"); return PCFR_E_INVALID_ARG; }
    int64_t t = 0;
    {
        IterState st;
        HIPCHK(hipMemcpyAsync(&st, s->ws + s->L.off_state, sizeof(st), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        t = st.t;
    }
    if (t != 0 || s->t_host != 0) { set_error("autotune needs a solver that has not iterated yet"); return PCFR_E_STATE; }
    int32_t rc = time_replays(s, reps, ms_before);
    if (rc) return rc;
    // level fusion threshold, by whole-iteration replays
    {
        const int64_t fcand[5] = {0, 4096, 16384, 65536, 262144};
        double best = 1e30;
        int64_t pick = s->sched.fuse_threads;
        for (int64_t f : fcand) {
            s->sched.fuse_threads = f;
            double ms = 0;
            if ((rc = rebuild_graph(s)) || (rc = time_replays(s, reps, &ms))) return rc;
            if (ms < best) { best = ms; pick = f; }
        }
        s->sched.fuse_threads = pick;
    }
    const int levels = s->P.levels;
    const int cand[4] = {64, 128, 256, 512};
    std::vector<double> best_f(levels, 1e30), best_b(levels, 1e30);
    std::vector<int> pick_f(levels, 256), pick_b(levels, 256);
    for (int c : cand) {
        s->sched.fwd_block.assign(levels, c);
        s->sched.bwd_block.assign(levels, c);
        std::vector<double> tf(levels, 0.0), tb(levels, 0.0);
        for (int32_t r = 0; r <= reps; r++) {
            LaunchTimer tm;
            tm.stream = s->stream;
            rc = s->cfg.dtype == PCFR_F64 ? enqueue_iteration<double>(s, s->stream, &tm)
                                          : enqueue_iteration<float>(s, s->stream, &tm);
            hipError_t e = hipStreamSynchronize(s->stream);
            for (size_t k = 0; k < tm.tag.size(); k++) {
                float ms = 0;
                if (r > 0 && rc == PCFR_OK && e == hipSuccess && tm.tag[k] >= 0) {
                    (void)hipEventElapsedTime(&ms, tm.ev[2 * k], tm.ev[2 * k + 1]);
                    if (tm.tag[k] >= 1000) tb[tm.tag[k] - 1000] += ms;
                    else tf[tm.tag[k]] += ms;
                }
            }
            for (auto ev : tm.ev) (void)hipEventDestroy(ev);
            if (rc) return rc;
            HIPCHK(e);
        }
        for (int l = 0; l < levels; l++) {
            if (tf[l] > 0 && tf[l] < best_f[l]) { best_f[l] = tf[l]; pick_f[l] = c; }
            if (tb[l] > 0 && tb[l] < best_b[l]) { best_b[l] = tb[l]; pick_b[l] = c; }
        }
    }
    s->sched.fwd_block = pick_f;
    s->sched.bwd_block = pick_b;
    if (s->net && s->L.n_net) {
        double nb = 0, na = 0;
        const int64_t rows = (s->L.n_net * s->L.n_next + 63) / 64 * 64;
        if ((rc = leafnet_autotune(s->net, rows, reps, &nb, &na))) return rc;
    }
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        // only launches that ran on their own (not inside a fused run) were timed
        for (int l = 0; l < levels; l++) {
            if (best_f[l] < 1e30) g_sched_cache[sched_key(s, 0, l)] = pick_f[l];
            if (best_b[l] < 1e30) g_sched_cache[sched_key(s, 1, l)] = pick_b[l];
        }
    }
    if ((rc = rebuild_graph(s))) return rc;
    if ((rc = time_replays(s, reps, ms_after))) return rc;
    return reset_state(s);
}

}  // namespace pcfr

extern "C" {

int32_t pcfr_autotune(pcfr_solver* s, int32_t reps, double* ms_before, double* ms_after) {
    if (s) if (const int32_t rc = leaves_ready(s)) return rc;
    return autotune_impl(s, reps, ms_before, ms_after);
}

int32_t pcfr_batch_autotune(pcfr_solver* s, int32_t budget_ms) {
    if (!s || budget_ms <= 0) { set_error("null solver or non-positive budget"); return PCFR_E_INVALID_ARG; }
    if (const int32_t rc = leaves_ready(s)) return rc;
    {
        int64_t t = 0;
        int32_t rc = pcfr_iteration(s, &t);
        if (rc) return rc;
        if (t != 0 || s->t_host != 0) { set_error("autotune needs a solver that has not iterated yet"); return PCFR_E_STATE; }
    }
    // the tuner runs about 12 trials of reps iterations (5 fusion thresholds,
    // 4 workgroup sizes, before/after); one replay estimates an iteration
    double ms = 0;
    int32_t rc = time_replays(s, 1, &ms);
    if (rc) return rc;
    if ((rc = reset_state(s))) return rc;
    const int32_t reps = (int32_t)std::max(1.0, std::min(50.0, budget_ms / (12.0 * std::max(ms, 1e-3))));
    double before = 0, after = 0;
    return autotune_impl(s, reps, &before, &after);
}

int32_t pcfr_solver_workspace_bytes(const pcfr_tree* tree, const pcfr_solver_cfg* cfg, size_t* bytes) {
    const pcfr_tree* t[1] = {tree};
    return workspace_for(t, 1, cfg, bytes);
}

int32_t pcfr_solver_create(const pcfr_tree* tree, const pcfr_solver_cfg* cfg, const double* ranges, void* workspace,
                           size_t workspace_bytes, void* stream, pcfr_solver** out) {
    const pcfr_tree* t[1] = {tree};
    return create_impl(t, 1, cfg, ranges, workspace, workspace_bytes, stream, out);
}

int32_t pcfr_batch_workspace_bytes(const pcfr_tree* const* trees, int32_t n, const pcfr_solver_cfg* cfg, size_t* bytes) {
    return workspace_for(trees, n, cfg, bytes);
}

int32_t pcfr_batch_create(const pcfr_tree* const* trees, int32_t n, const pcfr_solver_cfg* cfg, const double* ranges,
                          void* workspace, size_t workspace_bytes, void* stream, pcfr_solver** out) {
    return create_impl(trees, n, cfg, ranges, workspace, workspace_bytes, stream, out);
}

int32_t pcfr_batch_size(const pcfr_solver* s, int32_t* n) {
    if (!s || !n) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    *n = s->P.n_sub;
    return PCFR_OK;
}

int32_t pcfr_solver_attach_leafnet(pcfr_solver* s, pcfr_leafnet* net) {
    if (!s) { set_error("null solver"); return PCFR_E_INVALID_ARG; }
    if (net) {
        const LeafNetPlan& N = net->P;
        if (N.dims[0] != 2 * kCombos + 53 || N.dims[N.L] != 2 * kCombos) {
            set_error("leaf network must map 2*1326 + 53 inputs to 2*1326 outputs");
            return PCFR_E_INVALID_ARG;
        }
        if (s->L.n_net * s->L.n_next > N.Mp) { set_error("leaf network max_batch below leaves x next cards"); return PCFR_E_INVALID_ARG; }
        if (N.pdims[0] % 8) { set_error("leaf network input rows must be padded to 8 columns"); return PCFR_E_INVALID_ARG; }
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    s->net = net;
    if (s->graph) { (void)hipGraphExecDestroy(s->graph); s->graph = nullptr; }
    if (s->graph_def) { (void)hipGraphDestroy(s->graph_def); s->graph_def = nullptr; }
    return build_graph(s);
}

int32_t pcfr_solver_set_leaf_zero_sum(pcfr_solver* s, int32_t on) {
    if (!s || (on != 0 && on != 1)) { set_error("null solver or flag not 0/1"); return PCFR_E_INVALID_ARG; }
    HIPCHK(hipStreamSynchronize(s->stream));
    s->leaf_zero_sum = on != 0;
    if (s->graph) { (void)hipGraphExecDestroy(s->graph); s->graph = nullptr; }
    if (s->graph_def) { (void)hipGraphDestroy(s->graph_def); s->graph_def = nullptr; }
    return build_graph(s);
}

int32_t pcfr_leaf_rows(pcfr_solver* s, int32_t* n_leaves, int32_t* n_next) {
    if (!s || !n_leaves || !n_next) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    *n_leaves = (int32_t)s->L.n_net;
    *n_next = (int32_t)s->L.n_next;
    return PCFR_OK;
}

int32_t pcfr_solver_free(pcfr_solver* s) {
    delete s;   // the destructor waits for the streams and releases graph, stream and events
    return PCFR_OK;
}

int32_t pcfr_cfr_iterate(pcfr_solver* s, int32_t n) {
    if (!s || n < 0) { set_error("null solver or negative count"); return PCFR_E_INVALID_ARG; }
    if (const int32_t rc = leaves_ready(s)) return rc;
    if (s->launch_mode == PCFR_LAUNCH_PERSISTENT) {
        if (n > 0) {
            const int32_t rc = s->cfg.dtype == PCFR_F64 ? persist_launch<double>(s, n) : persist_launch<float>(s, n);
            if (rc) return rc;
        }
        s->t_host += n;
        return PCFR_OK;
    }
    for (int32_t i = 0; i < n; i++) HIPCHK(hipGraphLaunch(s->graph, s->stream));
    s->t_host += n;
    return PCFR_OK;
}

int32_t pcfr_profile_iterations(pcfr_solver* s, int32_t n, double* ms, int64_t* launches) {
    if (!s || n < 0 || !ms || !launches) { set_error("null argument or negative count"); return PCFR_E_INVALID_ARG; }
    if (const int32_t rc = leaves_ready(s)) return rc;
    for (int k = 0; k < 8; k++) { ms[k] = 0; launches[k] = 0; }
    for (int32_t i = 0; i < n; i++) {
        LaunchTimer tm;
        tm.stream = s->stream;
        int32_t rc = s->cfg.dtype == PCFR_F64 ? enqueue_iteration<double>(s, s->stream, &tm)
                                              : enqueue_iteration<float>(s, s->stream, &tm);
        hipError_t e = hipStreamSynchronize(s->stream);
        for (size_t k = 0; k < tm.cls.size(); k++) {
            float t = 0;
            if (e == hipSuccess && rc == PCFR_OK) (void)hipEventElapsedTime(&t, tm.ev[2 * k], tm.ev[2 * k + 1]);
            ms[tm.cls[k]] += t;
            launches[tm.cls[k]]++;
        }
        for (auto ev : tm.ev) (void)hipEventDestroy(ev);
        if (rc) return rc;
        HIPCHK(e);
    }
    s->t_host += n;
    return PCFR_OK;
}

int32_t pcfr_solver_unreached_nodes(pcfr_solver* s, int64_t* n) {
    if (!s || !n) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if (!s->cfg.prune) { set_error("the solver was created without pruning"); return PCFR_E_STATE; }
    const Plan& L = s->L;
    std::vector<int32_t> nzs(2 * (size_t)s->P.n_sub + L.rows);
    HIPCHK(hipMemcpyAsync(nzs.data(), s->ws + L.off_nzs, sizeof(int32_t) * nzs.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    int64_t cnt = 0;
    for (const DNode& d : s->P.nodes)
        if (nzs[d.slot[0]] == 0 && nzs[d.slot[1]] == 0) cnt++;
    *n = cnt;
    return PCFR_OK;
}

int32_t pcfr_solver_set_terminal_fusion(pcfr_solver* s, int32_t on) {
    if (!s || (on != 0 && on != 1)) { set_error("null solver or flag not 0/1"); return PCFR_E_INVALID_ARG; }
    s->tf_enabled = on != 0;
    return rebuild_graph(s);
}

int32_t pcfr_solver_set_launch(pcfr_solver* s, int32_t mode) {
    if (!s) { set_error("null solver"); return PCFR_E_INVALID_ARG; }
    return set_launch_impl(s, mode);
}

int32_t pcfr_synchronize(pcfr_solver* s) {
    if (!s) { set_error("null solver"); return PCFR_E_INVALID_ARG; }
    HIPCHK(hipStreamSynchronize(s->stream));
    return PCFR_OK;
}

int32_t pcfr_iteration(pcfr_solver* s, int64_t* t) {
    if (!s || !t) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    IterState st;
    HIPCHK(hipMemcpyAsync(&st, s->ws + s->L.off_state, sizeof(st), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    *t = st.t;
    return PCFR_OK;
}

int32_t pcfr_get_strategy(pcfr_solver* s, int32_t node, int32_t which, double* out) {
    return strategy_impl(s, 0, node, which, out);
}

int32_t pcfr_solver_swept_nodes(pcfr_solver* s, int64_t* n) {
    if (!s || !n) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    *n = (int64_t)(s->P.fwd.size() + s->P.term.size());
    return PCFR_OK;
}

int32_t pcfr_batch_get_strategy(pcfr_solver* s, int32_t sub, int32_t node, int32_t which, double* out) {
    return strategy_impl(s, sub, node, which, out);
}

int32_t pcfr_get_root_cfv(pcfr_solver* s, int32_t which, double* out) { return root_cfv_impl(s, 0, which, out, true); }

int32_t pcfr_batch_get_root_cfv(pcfr_solver* s, int32_t sub, int32_t which, double* out) {
    return root_cfv_impl(s, sub, which, out, true);
}

int32_t pcfr_node_values(pcfr_solver* s, int32_t sub, double* out) { return node_values_impl(s, sub, out); }

int32_t pcfr_exploitability(pcfr_solver* s, double* chips_per_hand, double* br) {
    if (!s || !chips_per_hand) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    std::vector<double> e(s->P.n_sub), b(2 * s->P.n_sub);
    int32_t rc = exploitability_impl(s, e.data(), b.data());
    if (rc) return rc;
    *chips_per_hand = e[0];
    if (br) { br[0] = b[0]; br[1] = b[1]; }
    return PCFR_OK;
}

int32_t pcfr_batch_exploitability(pcfr_solver* s, double* chips_per_hand, double* br) {
    if (!s || !chips_per_hand) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    return exploitability_impl(s, chips_per_hand, br);
}

int32_t pcfr_state_bytes(pcfr_solver* s, size_t* bytes) {
    if (!s || !bytes) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    *bytes = 16 + (s->cfg.variant == PCFR_PCFRPLUS ? 3 : 2) * s->L.esz * s->L.rows * s->L.Hp;
    return PCFR_OK;
}

int32_t pcfr_save_state(pcfr_solver* s, void* buf, size_t bytes) {
    size_t need;
    if (!s || !buf) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    pcfr_state_bytes(s, &need);
    if (bytes < need) { set_error("state buffer too small"); return PCFR_E_INVALID_ARG; }
    const Plan& L = s->L;
    IterState st;
    char* b = reinterpret_cast<char*>(buf);
    size_t rb = L.esz * L.rows * L.Hp;
    HIPCHK(hipMemcpyAsync(&st, s->ws + L.off_state, sizeof(st), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(b + 16, s->ws + L.off_R, rb, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(b + 16 + rb, s->ws + L.off_S, rb, hipMemcpyDeviceToHost, s->stream));
    if (s->cfg.variant == PCFR_PCFRPLUS)
        HIPCHK(hipMemcpyAsync(b + 16 + 2 * rb, s->ws + L.off_M, rb, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    int64_t hdr[2] = {st.t, (int64_t)L.esz + 16 * s->cfg.variant};
    std::memcpy(b, hdr, 16);
    return PCFR_OK;
}

int32_t pcfr_load_state(pcfr_solver* s, const void* buf, size_t bytes) {
    size_t need;
    if (!s || !buf) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    pcfr_state_bytes(s, &need);
    if (bytes < need) { set_error("state buffer too small"); return PCFR_E_INVALID_ARG; }
    const Plan& L = s->L;
    const char* b = reinterpret_cast<const char*>(buf);
    int64_t hdr[2];
    std::memcpy(hdr, b, 16);
    if (hdr[1] != (int64_t)L.esz + 16 * s->cfg.variant || hdr[0] < 0) {
        set_error("state was saved with another dtype or variant");
        return PCFR_E_INVALID_ARG;
    }
    size_t rb = L.esz * L.rows * L.Hp;
    const int64_t t = hdr[0];
    HIPCHK(hipMemcpyAsync(s->ws + L.off_state + offsetof(IterState, t), &t, sizeof(t), hipMemcpyHostToDevice, s->stream));
    if (s->cfg.variant == PCFR_PCFRPLUS)
        HIPCHK(hipMemcpyAsync(s->ws + L.off_M, b + 16 + 2 * rb, rb, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + L.off_R, b + 16, rb, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + L.off_S, b + 16 + rb, rb, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return PCFR_OK;
}

int32_t pcfr_batch_leaf_samples(pcfr_solver* s, float* x, int32_t ldx, float* y, float* mask, int32_t ldy) {
    if (!s || !x || !y || !mask) { set_error("null argument"); return PCFR_E_INVALID_ARG; }
    if (ldx < 2 * kCombos + 53 || ldy < 2 * kCombos) { set_error("row strides too small"); return PCFR_E_INVALID_ARG; }
    const Plan& L = s->L;
    const int32_t n = s->P.n_sub;
    const float* dps = s->at<float>(L.off_samp);
    const uint8_t* dboards = s->at<uint8_t>(L.off_samp + align256(sizeof(float) * 2 * n));
    const int16_t* dc2h = s->at<int16_t>(L.off_samp + align256(sizeof(float) * 2 * n) + align256((size_t)n * 52));
    int32_t rc = sweep<MODE_EV>(s);
    if (rc) return rc;
    if (L.esz == 8)
        hipLaunchKernelGGL((k_samples<double>), dim3(n), dim3(kBlock), 0, s->stream, s->at<int32_t>(L.off_roots), dps,
                           dboards, (int)L.Hp, s->at<double>(L.off_reach), s->at<double>(L.off_cfv),
                           s->at<uint16_t>(L.off_hc), dc2h, s->at<int32_t>(L.off_coff), s->at<int16_t>(L.off_chands),
                           (int)L.chand_stride, x, ldx, y, mask, ldy);
    else
        hipLaunchKernelGGL((k_samples<float>), dim3(n), dim3(kBlock), 0, s->stream, s->at<int32_t>(L.off_roots), dps,
                           dboards, (int)L.Hp, s->at<float>(L.off_reach), s->at<float>(L.off_cfv),
                           s->at<uint16_t>(L.off_hc), dc2h, s->at<int32_t>(L.off_coff), s->at<int16_t>(L.off_chands),
                           (int)L.chand_stride, x, ldx, y, mask, ldy);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return PCFR_OK;
}

}  // extern "C"
