/*
 * pcfr.h -- C ABI of the MI355X (gfx950) discounted-CFR library for heads-up
 * no-limit hold'em public subgames.
 *
 * The operation is one CFR iteration over a public tree whose every node
 * carries a range vector per player over the 1326 hole-card combos (Li &
 * Huang, "Real-Time Parallel Counterfactual Regret Minimization", Sec. 4:
 * the seven stages of Table 1 -- forward reach, aggregation, opponent reach,
 * showdown, leaf evaluation, backward counterfactual values, regret update).
 * Every stage runs in HIP kernels on the GPU; the host only builds the tree
 * and its lookup tables once.
 *
 * Conventions shared with callers:
 *   card  = 4*rank + suit, rank 0..12 = 2..A, suit 0..3;
 *   combo = a(a-1)/2 + b for cards a > b, 0 <= combo < 1326;
 *   chips are integers; each player has put pot/2 in at the root.
 *
 * Errors: every call returns an int32 status.  Out-parameters are written
 * only on PCFR_OK.  pcfr_last_error() returns a message for the calling
 * thread's most recent failure.  No C++ exception crosses this boundary.
 *
 * Threading: a handle is not thread-safe; distinct handles are independent.
 * Device work of a solver is ordered on the stream given at creation.
 */
#ifndef PCFR_H
#define PCFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCFR_ABI_VERSION 2
#define PCFR_NCOMBO 1326

enum {
    PCFR_OK = 0,
    PCFR_E_INVALID_ARG = 1,   /* bad pointer, size, card, range, node or enum */
    PCFR_E_OUT_OF_MEMORY = 2, /* host allocation failed or workspace too small */
    PCFR_E_DEVICE = 3,        /* a HIP runtime call failed */
    PCFR_E_STATE = 4,         /* call not valid in the handle's current state */
    PCFR_E_UNSUPPORTED = 5,   /* option not implemented */
    PCFR_E_NUMERIC = 6,       /* non-finite value detected */
    PCFR_E_TOO_LARGE = 7      /* tree exceeds an internal limit */
};

enum { PCFR_F32 = 0, PCFR_F64 = 1 };             /* solver arithmetic */
enum { PCFR_AVG = 0, PCFR_CURRENT = 1 };         /* which strategy / values */
enum { PCFR_DCFR = 0, PCFR_CFRPLUS = 1, PCFR_PCFRPLUS = 2 }; /* Stage-7 rule */

/* Node types in exported trees. */
enum {
    PCFR_NODE_DECISION = 0,
    PCFR_NODE_FOLD = 1,
    PCFR_NODE_SHOWDOWN = 2,
    PCFR_NODE_CHANCE = 3,
    PCFR_NODE_LEAF = 4,       /* depth-limit leaf, valued by the leaf model */
    PCFR_NODE_ALLIN_LEAF = 5  /* depth-limit leaf with a player all in: exact runout equity */
};

/* Betting abstraction of a subgame (Sec. 5 "Game": fixed action
 * abstraction, stack-to-pot ratio, number of raise sizes).
 *   n_board      3, 4 or 5 public cards in board[0..n_board); or 0, a
 *                preflop root: then depth_limit must be 1 (the leaves sit at
 *                the flop deal) and no betting line may put a player all in
 *                (else PCFR_E_UNSUPPORTED).  A preflop root is solved over
 *                the 169 hand classes (pairs, suited and offsuit rank
 *                pairs; lossless suit abstraction, Sec. 4.5): its ranges
 *                must be equal on the combos of each class
 *                (PCFR_E_INVALID_ARG otherwise), suit_iso does not apply
 *                (PCFR_E_UNSUPPORTED), a batch holds preflop roots only,
 *                and per-hand outputs repeat a class's value on its combos.
 *   pot          chips in the pot at the root; even, > 0
 *   stack[2]     chips behind per player; the smaller one caps every bet
 *   size_pct     n_sizes (<= 8) bet sizes as integer percent of the pot after
 *                calling; a bet puts in to_call + floor((pct*pot' + 50)/100)
 *   allin        1 adds an all-in action wherever bets are allowed
 *   max_raises   bets + raises allowed per street, the opening bet included
 *   depth_limit  0: play to showdown; 1: stop at the end of the root street
 *                with depth-limit leaves.
 * Player 0 acts first on every street. */
typedef struct pcfr_tree_spec {
    int32_t n_board;
    int32_t board[5];
    int64_t pot;
    int64_t stack[2];
    int32_t n_sizes;
    int32_t size_pct[8];
    int32_t allin;
    int32_t max_raises;
    int32_t depth_limit;
} pcfr_tree_spec;

/* Solver options.  DCFR discounting (the paper's default CFR variant,
 * Sec. 5 "Baselines", after Brown & Sandholm 2019): after adding the
 * iteration-t regret, a positive cumulative regret is scaled by
 * t^alpha/(t^alpha+1), a non-positive one by t^beta/(t^beta+1), and the
 * average-strategy sum by (t/(t+1))^gamma.  alternating = 0: both players
 * are updated from the same strategies (simultaneous updates, one sweep per
 * iteration); 1: player 0 is updated first, then player 1 against player 0's
 * new strategy, both with iteration t's coefficients (two sweeps per
 * iteration); other values are PCFR_E_INVALID_ARG.  suit_iso = 1: lossless
 * suit isomorphism (Sec. 4.5, information abstraction).  The suit
 * permutations that map a subgame's root board onto itself and leave both
 * root ranges exactly unchanged form its symmetry group; below each chance
 * node only one child per orbit of the dealt card (under the permutations
 * that also fix the cards dealt above the node) is swept, and the node reads
 * the other children's values through the hand permutation.  Results equal
 * those of suit_iso = 0 up to rounding order; ranges without symmetry change
 * nothing.  Strategies inside a skipped subtree are not stored;
 * pcfr_get_strategy returns the representative's with the hands relabelled
 * by the permutation.
 *
 * threshold = thr0 > 0: dynamic thresholding (cited in Sec. 2 among the
 * pruning methods: low-probability actions are dropped on the fly).  In
 * iteration t, after regret matching, every action whose probability is
 * below thr0 / sqrt(t) is set to 0 and the others are renormalised (the
 * threshold shrinks as the regret-matching error bound does, so the average
 * strategy still converges); PCFR_CURRENT strategies are those of the next
 * iteration.  prune = 1: regret-based pruning as Sec. 2 describes it --
 * subtrees unreachable under the current strategy profile are skipped.  A
 * node whose reach is zero for every hand of both players contributes exact
 * zeros (every value in its subtree is weighted by the other player's
 * reach); the iteration does not load its regrets or evaluate its terminals,
 * and only applies the Stage-7 discount to its regret and average rows, so
 * the iterates are bitwise those of prune = 0.  Thresholding makes such
 * subtrees common. */
typedef struct pcfr_solver_cfg {
    int32_t dtype;        /* PCFR_F32 or PCFR_F64 */
    int32_t variant;      /* PCFR_DCFR, PCFR_CFRPLUS or PCFR_PCFRPLUS */
    double alpha, beta, gamma;
    int32_t alternating;  /* 0 or 1 */
    int32_t suit_iso;     /* 0 or 1: lossless suit isomorphism at chance nodes */
    double threshold;     /* dynamic thresholding: 0 (off) or thr0 in (0, 1/12) */
    int32_t prune;        /* 0 or 1: skip subtrees no hand of either player reaches */
} pcfr_solver_cfg;

typedef struct pcfr_tree pcfr_tree;
typedef struct pcfr_solver pcfr_solver;

int32_t pcfr_abi_version(void);
const char* pcfr_last_error(void);

/* ---------------------------------------------------------------- tree
 * Build the public tree of a subgame on the host (Sec. 3, depth-limited
 * solving: the tree ends at showdown or at the depth limit).  Node ids are
 * breadth-first from the root; children follow action order (fold, call or
 * check, then bets ascending) and chance children ascend by card.  The
 * library owns *out; release with pcfr_tree_free. */
int32_t pcfr_build_tree(const pcfr_tree_spec* spec, pcfr_tree** out);
int32_t pcfr_tree_free(pcfr_tree* tree);

/* out[16]: nodes, decision, fold, showdown, chance, leaf, allin-leaf,
 * levels, action rows (sum of actions over decision nodes), hands the
 * solver sweeps (board-compatible combos; the 169 hand classes of a preflop
 * root), those padded to 64, then zeros. */
int32_t pcfr_tree_info(const pcfr_tree* tree, int64_t* out);

/* Node arrays, each of length nodes (contrib: 2 per node), caller-owned
 * host buffers.  player: actor of a decision, folder of a fold, else -1.
 * parent/action: -1 at the root.  chance_card: card dealt on the edge into
 * the node, else -1.  first_child: -1 for nodes without children. */
int32_t pcfr_tree_export(const pcfr_tree* tree, int32_t* type, int32_t* player, int32_t* parent,
                         int32_t* action, int32_t* depth, int64_t* contrib, int32_t* chance_card,
                         int32_t* first_child, int32_t* n_child);

/* Lossless suit isomorphism of one subgame (host only; what a solver with
 * suit_iso = 1 uses).  ranges: [2][1326] host doubles, as for
 * pcfr_solver_create.  group: bit q set when suit permutation q (the q-th
 * permutation of (0, 1, 2, 3) in lexicographic order, suit s -> perm[s])
 * maps the root board and both ranges onto themselves.  Per node (caller
 * buffers of length nodes): src, for a chance child, the child whose values
 * stand for it (itself for a representative, the smallest card of its
 * orbit), else -1; perm, for a mapped child, the permutation taking the
 * representative's card to its own, else -1; skip, 1 inside subtrees that
 * are not swept. */
int32_t pcfr_suit_iso_map(const pcfr_tree* tree, const double* ranges, uint32_t* group, int32_t* src,
                          int32_t* perm, int8_t* skip);

/* Online pruning (Sec. 5, "Online Pruning"): dominated actions are removed
 * once, before any iteration, and every later iteration sweeps the smaller
 * tree.
 *
 * pcfr_prune_dominated runs the dominance test on the GPU, one workgroup per
 * decision node (the decisions at the information sets are independent).
 * lo, hi: device doubles [nodes][1326], row n = lower and upper bounds on the
 * value to the actor of the action leading to node n (rows of nodes that no
 * decision leads to are not read), per combo, on any scale shared by the
 * siblings of one node (counterfactual values, or values given the node is
 * reached).  ranges: host [2][1326], as for pcfr_solver_create.  Action a of
 * a node is dominated for hand h when hi[a][h] < lo[b][h] for some sibling b;
 * removed[n] (host, length nodes) becomes 1 when the action into n is
 * dominated for every hand h of the actor's range (range > 0) that the
 * node's board does not block, else 0 (so a node where the actor holds no
 * such hand removes nothing).  With lo <= hi the action holding the largest
 * lower bound of some hand survives, so no node loses every action.
 * Synchronises the device's null stream; the bounds must be complete before
 * the call.
 *
 * pcfr_tree_prune builds the reduced tree (host only): the actions flagged
 * in removed (a flag on a child of a decision node drops that action and its
 * subtree) are gone, kept nodes keep their breadth-first order and their
 * children's order, and a child's action index becomes its position among
 * the kept siblings.  new_id (caller buffer of length nodes, may be NULL)
 * receives each node's id in the reduced tree, -1 when dropped.  Fails with
 * PCFR_E_INVALID_ARG when a flag sits on a node no decision leads to or a
 * decision node would keep no action.  The library owns *out; release with
 * pcfr_tree_free. */
int32_t pcfr_prune_dominated(const pcfr_tree* tree, const double* ranges, const double* lo, const double* hi,
                             uint8_t* removed);
int32_t pcfr_tree_prune(const pcfr_tree* tree, const uint8_t* removed, pcfr_tree** out, int32_t* new_id);

/* pcfr_prune_dominated without any device allocation, for callers that
 * cannot allocate (serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, checks and result as pcfr_prune_dominated; the node list,
 * combo masks, ranges and flags live in a static device array of the
 * library (about 1.9 MB per GPU, held until the process ends), reached
 * through the current device's symbol address.  Trees with more than 65536
 * decision nodes or 262144 nodes give PCFR_E_TOO_LARGE.  Work runs on the
 * device's null stream and the call returns after the flags are copied
 * back.  Every call on one GPU shares that array, so calls that overlap on
 * one GPU (from several host threads) race; each call clears the flags it
 * uses. */
int32_t pcfr_prune_dominated_noalloc(const pcfr_tree* tree, const double* ranges, const double* lo,
                                     const double* hi, uint8_t* removed);

/* Seven-card hand values, host side (used to order hands at showdown,
 * Sec. 4.3 Stage 4).  cards: n*7 card ids; out: n values.  Value layout:
 * category (0 high card .. 8 straight flush) in bits 20..23 and the
 * tie-breaking ranks in bits 16..19 down to 0..3. */
int32_t pcfr_eval7_batch(const int32_t* cards, int64_t n, int32_t* out);

/* Pairwise check-down equity on the tree's root board (3 or 4 cards): out
 * [1326][1326] host doubles, out[h][o] = mean over every completion of the
 * board by cards neither hand holds of sign(value(h) - value(o)); 0 for
 * pairs sharing a card or touching the board.  This is the exact value per
 * chip of contribution of an all-in depth-limit leaf (Sec. 3, depth-limited
 * solving: leaves where nothing is left to decide are valued exactly). */
int32_t pcfr_equity_table(const pcfr_tree* tree, double* out);

/* ---------------------------------------------------------------- solver
 * Device memory is the caller's: ask for the size, allocate it, keep it alive
 * until pcfr_solver_free.  The solver copies the tree, so the tree may be
 * freed after creation. */
int32_t pcfr_solver_workspace_bytes(const pcfr_tree* tree, const pcfr_solver_cfg* cfg, size_t* bytes);

/* ranges: host [2][1326] reach of each player's hands at the root; finite,
 * >= 0, zero on combos that share a card with the board, and some compatible
 * pair of hands must carry mass.  workspace: device pointer of at least
 * pcfr_solver_workspace_bytes bytes, 256-byte aligned.  stream: a hipStream_t
 * (NULL = default stream).  The solver starts at iteration 0 with zero
 * regrets and zero average-strategy sums. */
int32_t pcfr_solver_create(const pcfr_tree* tree, const pcfr_solver_cfg* cfg, const double* ranges,
                           void* workspace, size_t workspace_bytes, void* stream, pcfr_solver** out);
int32_t pcfr_solver_free(pcfr_solver* s);

/* Enqueue n >= 0 DCFR iterations on the solver's stream (asynchronous).
 * The per-iteration launch sequence is captured once in a HIP graph and
 * replayed; the iteration counter lives on the device. */
int32_t pcfr_cfr_iterate(pcfr_solver* s, int32_t n);
int32_t pcfr_synchronize(pcfr_solver* s);

/* How pcfr_cfr_iterate runs the iterations of a solver or batch.
 * PCFR_LAUNCH_GRAPH (the default): each iteration is a replay of the
 * captured HIP graph of per-level launches.  PCFR_LAUNCH_PERSISTENT: one
 * cooperative launch of a resident grid runs all n iterations, the level
 * sweeps and terminals separated by grid barriers (the batching workload of
 * many subgames in one persistent launch); for solvers whose subgames are
 * played to showdown (no depth-limit leaves), with simultaneous updates and
 * without suit isomorphism, else PCFR_E_UNSUPPORTED.  Both modes compute
 * bitwise the same iterates; other calls (strategies, values,
 * exploitability, autotuning, profiling) are unaffected. */
enum { PCFR_LAUNCH_GRAPH = 0, PCFR_LAUNCH_PERSISTENT = 1 };
int32_t pcfr_solver_set_launch(pcfr_solver* s, int32_t mode);

/* Terminal fusion of the graph launches, on (1) or off (0, the default).
 * On: every decision node at a backward level swept by per-node launches
 * that has one or two fold or showdown children evaluates them in its own
 * workgroup (LDS) and reads their values there, instead of a separate
 * terminal launch writing them to memory for the backward launch to read
 * back.  The arithmetic is the same, so the iterates are bitwise equal
 * either way.  Re-captures the iteration graph. */
int32_t pcfr_solver_set_terminal_fusion(pcfr_solver* s, int32_t on);

/* Nodes (over all subgames) that the last iteration found unreachable and
 * skipped, for a solver created with prune = 1 (else PCFR_E_STATE); with
 * alternating updates, those of the second half-step.  Synchronises. */
int32_t pcfr_solver_unreached_nodes(pcfr_solver* s, int64_t* n);

/* Run n iterations like pcfr_cfr_iterate, but launch by launch with HIP
 * events around every kernel on the solver's stream, and return the summed
 * device time and launch count per kernel class: [0] iteration bookkeeping,
 * [1] forward reach sweep, [2] fold/showdown terminals, [3] backward value
 * and regret sweep, [4] depth-limit leaves (exact equity, network input and
 * combine), [5] leaf-network hidden-layer GEMMs (bias + ReLU), [6] its output
 * layer GEMM, [7] unused.  ms and launches are host arrays of 8.
 * Synchronises. */
int32_t pcfr_profile_iterations(pcfr_solver* s, int32_t n, double* ms, int64_t* launches);
int32_t pcfr_iteration(pcfr_solver* s, int64_t* t);   /* synchronises */

/* Strategy at a decision node: PCFR_AVG = average strategy (sum of
 * reach-weighted strategies, normalised; uniform where the sum is 0),
 * PCFR_CURRENT = regret matching of the cumulative regrets (eq. rm; uniform
 * where no regret is positive).  out: host [A][1326] doubles, A = the node's
 * action count; combos blocked by the board get 0.  Synchronises. */
int32_t pcfr_get_strategy(pcfr_solver* s, int32_t node, int32_t which, double* out);
/* Nodes the sweeps visit (decision, chance and terminal nodes outside the
 * subtrees suit isomorphism skips), over all subgames. */
int32_t pcfr_solver_swept_nodes(pcfr_solver* s, int64_t* n);

/* Root counterfactual values in chips (eq. cfv: each hand's value summed over
 * compatible opponent hands weighted by their reach).  PCFR_CURRENT: from the
 * last iteration, under the strategy it used; PCFR_AVG: under the average
 * strategies of both players.  out: host [2][1326]; blocked combos get 0. */
int32_t pcfr_get_root_cfv(pcfr_solver* s, int32_t which, double* out);

/* Counterfactual values of every node of subgame sub (0 for a single
 * subgame) under the average strategies of both players, as
 * pcfr_get_root_cfv with PCFR_AVG gives them at the root.  out: device
 * doubles [nodes of the subgame][2][1326] (player 0 row, then player 1);
 * combos blocked by the root board get 0, combos blocked by cards dealt
 * above a node carry no meaning.  Not available with suit_iso.
 * Synchronises. */
int32_t pcfr_node_values(pcfr_solver* s, int32_t sub, double* out);

/* Exploitability of the average strategy in chips per hand:
 * (BR_0 + BR_1) / 2, BR_i = best-response value of player i against the
 * other's average strategy, per unit of joint mass of compatible hand pairs.
 * br may be NULL.  Synchronises. */
int32_t pcfr_exploitability(pcfr_solver* s, double* chips_per_hand, double* br);

/* Checkpoint: iteration counter, cumulative regrets and average-strategy
 * sums in the solver's dtype.  pcfr_state_bytes gives the buffer size; buf is
 * host memory.  The blob is the solver's own state, for pcfr_load_state on a
 * solver of the same trees and configuration, not a table of the paper's
 * quantities: the chance probability 1/K is applied once at each chance node
 * (to the values passed up), so the regrets of rows below chance nodes hold
 * the paper's cumulative regrets times the product of the divisors K above
 * them (regret matching and every update rule are invariant under that
 * per-row scale, so the strategies are the paper's); the average-strategy
 * sums, weighted by the player's own reach, are not scaled. */
int32_t pcfr_state_bytes(pcfr_solver* s, size_t* bytes);
int32_t pcfr_save_state(pcfr_solver* s, void* buf, size_t bytes);
int32_t pcfr_load_state(pcfr_solver* s, const void* buf, size_t bytes);

/* ---------------------------------------------------------------- batches
 * Many independent subgames (river and turn, uneven sizes) solved together:
 * their trees form one forest whose levels are swept by the same launches,
 * so one graph replay advances every subgame by one iteration.  The handle is
 * a pcfr_solver; the single-subgame calls act on subgame 0, the batch calls
 * take a subgame index.  ranges: host [n][2][1326].  Depth-limited trees
 * batch too (their leaves are evaluated together: one equity table per
 * subgame, and with a leaf network one input row per leaf and next card of
 * every subgame in the same GEMMs); the subgames holding depth-limit leaves
 * must have boards of one size, else PCFR_E_UNSUPPORTED.  Results are bitwise
 * identical to solving each subgame alone (with a network, when its layers
 * use the same GEMM tiles in both). */
int32_t pcfr_batch_workspace_bytes(const pcfr_tree* const* trees, int32_t n, const pcfr_solver_cfg* cfg,
                                   size_t* bytes);
int32_t pcfr_batch_create(const pcfr_tree* const* trees, int32_t n, const pcfr_solver_cfg* cfg,
                          const double* ranges, void* workspace, size_t workspace_bytes, void* stream,
                          pcfr_solver** out);
int32_t pcfr_batch_size(const pcfr_solver* s, int32_t* n);
int32_t pcfr_batch_get_strategy(pcfr_solver* s, int32_t sub, int32_t node, int32_t which, double* out);
int32_t pcfr_batch_get_root_cfv(pcfr_solver* s, int32_t sub, int32_t which, double* out);
/* chips_per_hand: host [n]; br: host [n][2] or NULL.  Synchronises. */
int32_t pcfr_batch_exploitability(pcfr_solver* s, double* chips_per_hand, double* br);

/* Launch-schedule autotuner for a solver or batch that has not iterated yet
 * (else PCFR_E_STATE).  First the level-fusion threshold: runs of
 * consecutive levels with at most that many threads (nodes x padded hands /
 * 4) are swept by one launch in which each workgroup owns a slice of hands
 * and steps through the levels with workgroup barriers (candidates 0, 4096,
 * 16384 (the default), 65536, 262144; whole-iteration replays decide).  Then
 * each remaining level's forward and backward launch is
 * timed at workgroup sizes 64, 128, 256 and 512 over reps >= 1 iterations;
 * the fastest size per launch is kept, cached for the launch's size bucket
 * (phase, dtype, action-count bucket, log2 of its thread count) so that
 * solvers created later in the process start from it, and the iteration is
 * captured again.  ms_before / ms_after: host doubles, ms per iteration of
 * the captured iteration before and after tuning.  The sweep schedule
 * changes no arithmetic: without a network, iterates stay bitwise identical.
 * When a leaf network is attached, its forward GEMM tiles are tuned too (as
 * pcfr_leafnet_autotune for the solver's network rows; that choice can move
 * network outputs in the last bits).  The state is reset to iteration 0 on
 * return.  Synchronises. */
int32_t pcfr_autotune(pcfr_solver* s, int32_t reps, double* ms_before, double* ms_after);

/* pcfr_autotune with the trial length chosen to spend about budget_ms > 0 of
 * device time (at least one iteration per trial, at most 50).  Same
 * preconditions and effects. */
int32_t pcfr_batch_autotune(pcfr_solver* s, int32_t budget_ms);

/* ---------------------------------------------------------------- leaf network
 * The value network f_theta of depth-limited solving (Sec. 3): a ReLU MLP
 * d_in -> width x depth -> d_out evaluated for all leaves of an iteration in
 * one batch (Sec. 4.3, Stage 5) with bfloat16 MFMA GEMMs accumulating in
 * FP32.  FP32 master parameters; host layout for set/get: for each layer l
 * in order, W_l [out][in] row-major, then b_l [out].  Device memory is the
 * caller's workspace (256-byte aligned), work is ordered on `stream`.
 * max_batch bounds the rows of forward/train calls.  Parameters start at 0. */
typedef struct pcfr_leafnet pcfr_leafnet;

int32_t pcfr_leafnet_workspace_bytes(int32_t d_in, int32_t width, int32_t depth, int32_t d_out,
                                     int32_t max_batch, size_t* bytes);
int32_t pcfr_leafnet_create(int32_t d_in, int32_t width, int32_t depth, int32_t d_out, int32_t max_batch,
                            void* workspace, size_t workspace_bytes, void* stream, pcfr_leafnet** out);
int32_t pcfr_leafnet_free(pcfr_leafnet* net);
int32_t pcfr_leafnet_num_params(const pcfr_leafnet* net, int64_t* count);
/* Host FP32 parameters in, all finite; resets the Adam state.  Synchronises. */
int32_t pcfr_leafnet_set_params(pcfr_leafnet* net, const float* host);
int32_t pcfr_leafnet_get_params(pcfr_leafnet* net, float* host);
/* Gradients of the last train step, same layout.  Synchronises. */
int32_t pcfr_leafnet_get_grads(pcfr_leafnet* net, float* host);

/* y[m][d_out] = f(x[m][d_in]); x and y device FP32 (x is rounded to bf16
 * on the device).  Asynchronous. */
int32_t pcfr_leafnet_forward(pcfr_leafnet* net, const float* x, int32_t m, float* y);

/* Tile autotuner of the forward GEMMs for batches of m rows: every layer is
 * timed over reps >= 1 launches with each workgroup tile (PCFR_TILE_*
 * below) that divides its output width, and the
 * fastest is kept for all later forward calls (including the solver's leaf
 * stage).  Tiles group the FP32 partial sums differently, so outputs may
 * change in the last bits; for a fixed choice they are deterministic.  ms_before /
 * ms_after: host doubles, ms per forward pass before and after.  Clobbers
 * the staged activations.  Synchronises. */
int32_t pcfr_leafnet_autotune(pcfr_leafnet* net, int32_t m, int32_t reps, double* ms_before, double* ms_after);

/* Forward GEMM tile per layer (count = depth + 1 layers): PCFR_TILE_DEFAULT
 * (-1, chosen from the shape), PCFR_TILE_64x64, PCFR_TILE_128x64,
 * PCFR_TILE_64x128, PCFR_TILE_128x128 (rows x columns, 4 waves),
 * PCFR_TILE_64x64_K2, PCFR_TILE_64x128_K2 (two 4-wave groups that split
 * the K loop and add their partial sums), or PCFR_TILE_64x64_P4,
 * PCFR_TILE_64x128_P4 (4 waves, global loads four K stages ahead instead
 * of two), or PCFR_TILE_DIRECT, PCFR_TILE_DIRECT_K2, PCFR_TILE_DIRECT_K4
 * (one wave per 64 x 64 output tile, two or four with _K2 or _K4 splitting
 * K, both operands read straight into registers from copies in an
 * MFMA-ready layout, no LDS stage; only for
 * layers after the first whose input width is 1536, and every layer after a
 * direct layer must be direct too, since a direct layer's input is written
 * in that layout by the layer before).  The column count must divide the
 * layer's output width padded to 64; a tile that does not fit the layer
 * gives PCFR_E_INVALID_ARG.  Training steps run direct layers with the
 * default tile.  get returns the current choice.  Every tile spreads its
 * workgroups over the GPU's XCDs so that each XCD's L2 serves one block of
 * output rows x columns; that placement changes no arithmetic. */
enum {
    PCFR_TILE_DEFAULT = -1, PCFR_TILE_64x64 = 0, PCFR_TILE_128x64 = 1, PCFR_TILE_64x128 = 2, PCFR_TILE_128x128 = 3,
    PCFR_TILE_64x64_K2 = 4, PCFR_TILE_64x128_K2 = 5, PCFR_TILE_64x64_P4 = 6, PCFR_TILE_64x128_P4 = 7,
    PCFR_TILE_DIRECT = 8, PCFR_TILE_DIRECT_K2 = 9, PCFR_TILE_DIRECT_K4 = 10
};
int32_t pcfr_leafnet_set_tiles(pcfr_leafnet* net, const int32_t* tiles, int32_t count);
int32_t pcfr_leafnet_get_tiles(pcfr_leafnet* net, int32_t* tiles, int32_t count);

/* One Adam step (beta 0.9/0.999, eps 1e-8, learning rate lr) on the Huber
 * loss (delta 1) between f(x) and target over entries where mask != 0,
 * averaged over the mask's sum.  x [m][d_in], target and mask [m][d_out]
 * device FP32.  loss (host, may be NULL) receives the batch loss before the
 * step, which synchronises. */
int32_t pcfr_leafnet_train_step(pcfr_leafnet* net, const float* x, const float* target, const float* mask,
                                int32_t m, float lr, float* loss);

/* Value the solver's depth-limit leaves with net (NULL: exact check-down
 * equity, the stub model).  The net must map 2*1326 + 53 inputs (both
 * normalised ranges after each next card, the board one-hot, the
 * stack-to-pot ratio) to 2*1326 outputs (each hand's value per pot unit and
 * per unit of compatible opponent reach) and hold leaves x next-cards rows.
 * All-in leaves stay exact.  The net must outlive the attachment.
 *
 * Preflop leaves (Sec. 4.3's leaf model at the flop deal): one row per
 * (leaf, canonical flop) -- the 1755 flops that no suit permutation maps to a
 * smaller card mask, by their sorted cards in lexicographic order -- with
 * the ranges cleared of the flop's cards and the flop's three cards one-hot.
 * A hand class's leaf value is pot / C(48,3) / |class| times the sum over
 * the canonical flops of (flops in the orbit) x the sum over the class's
 * combos clear of the flop of EV x the opponent's reach clear of combo and
 * flop (exact for the suit-symmetric reach of a preflop root).  These leaves
 * have no exact model: without a net, iterating and evaluating return
 * PCFR_E_STATE. */
int32_t pcfr_solver_attach_leafnet(pcfr_solver* s, pcfr_leafnet* net);

/* Zero-sum correction of network leaf values, on (1, the default) or off (0).
 * For each (leaf, next card c) row, both players' outputs EV_i(h | c) are
 * shifted by the same d = e / (2 z), e = sum_h r0(h) M1(h|c) EV0(h|c) +
 * sum_h r1(h) M0(h|c) EV1(h|c), z = sum_h r0(h) M1(h|c) (hands holding c
 * excluded), so that the row's values sum to zero over both players as
 * solved values do.  The paper does not say how leaf values are kept
 * consistent; this is a reading.  Re-captures the iteration graph. */
int32_t pcfr_solver_set_leaf_zero_sum(pcfr_solver* s, int32_t on);
/* Training samples for the leaf network from a solved batch (the paper's
 * depth-limited method, Sec. 3: the network is trained on subgames the
 * solver itself solves).  Row g of x (device fp32 [n][ldx], ldx >= 2705):
 * subgame g's root ranges normalised to sum 1 over the 1326 combos, its board
 * one-hot, its stack-to-pot ratio.  Row g of y and mask (device fp32
 * [n][ldy], ldy >= 2652): each hand's root value under both average
 * strategies divided by (pot * the opponent's root reach compatible with the
 * hand), mask 1 where that reach is positive, else 0.  Runs one value sweep
 * under the average strategies.  Synchronises. */
int32_t pcfr_batch_leaf_samples(pcfr_solver* s, float* x, int32_t ldx, float* y, float* mask, int32_t ldy);

/* Network leaves and next cards per leaf (rows = product); for a batch, the
 * leaves of every subgame (the network's max_batch must hold all rows). */
int32_t pcfr_leaf_rows(pcfr_solver* s, int32_t* n_leaves, int32_t* n_next);

#ifdef __cplusplus
}
#endif
#endif /* PCFR_H */
