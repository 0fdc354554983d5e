/*
 * oracle.c -- plain, slow, FP64 reference for discounted CFR on heads-up
 * no-limit hold'em public subgames, plus Kuhn poker behind the same engine.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the product path never
 * does.  It shares no code, header, table or generator with the GPU library.
 *
 * What it computes, and where the paper defines it (Li & Huang, "Real-Time
 * Parallel Counterfactual Regret Minimization"):
 *   - counterfactual value of an information set, Sec. 3 eq. (cfv): computed
 *     history by history, summing over the opponent's private hand with its
 *     reach probability as the weight;
 *   - instantaneous regret r = v(sigma_{I->a}) - v(sigma), Sec. 3;
 *   - regret matching, Sec. 3 eq. (rm), uniform when no positive regret;
 *   - the average strategy as the output policy, Sec. 3;
 *   - the DCFR update of Stage 7 (Sec. 4.4, Table 1) with the discounting of
 *     Brown & Sandholm (2019), which the paper cites for its default variant
 *     (Sec. 2 and Sec. 5 "Baselines");
 *   - the "computationally exact" contract of Sec. 4 and the correctness
 *     guarantee of Sec. 4.5: the pipeline must reproduce a serial CFR, which
 *     is what this file is.
 * Readings where the paper is silent (payoff convention, betting rules,
 * chance weights, card encoding) are listed in the design notes; each is
 * restated where it is used below.
 *
 * Parallelism: OpenMP over the traverser's private hand only.  Each thread
 * owns the regret and value entries of its own hand, so no two threads write
 * the same address.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define NCOMBO 1326
#define MAXDEPTH 64

/* ------------------------------------------------------------------ cards */
/* card = 4*rank + suit, rank 0..12 stands for 2..A.
 * combo {a > b} has index a(a-1)/2 + b. */

static int combo_index(int a, int b) {
    if (a < b) { int t = a; a = b; b = t; }
    return a * (a - 1) / 2 + b;
}

/* Five-card hand value.  Category in bits 20..23 (0 high card, 1 pair,
 * 2 two pair, 3 trips, 4 straight, 5 flush, 6 full house, 7 quads,
 * 8 straight flush); the ranks that break ties, most significant first, in
 * bits 16..19, 12..15, 8..11, 4..7, 0..3, unused positions zero.  A wheel
 * (A-2-3-4-5) is a straight with high card "5" (rank 3). */
int ora_eval5(const int* c) {
    int cnt[13] = {0};
    int r[5], s[5];
    for (int i = 0; i < 5; i++) { r[i] = c[i] >> 2; s[i] = c[i] & 3; cnt[r[i]]++; }
    int flush = (s[0] == s[1] && s[1] == s[2] && s[2] == s[3] && s[3] == s[4]);
    /* distinct ranks, descending */
    int distinct = 0, hi = -1, lo = 13;
    for (int k = 0; k < 13; k++) if (cnt[k]) { distinct++; if (k > hi) hi = k; if (k < lo) lo = k; }
    int straight = 0, shigh = -1;
    if (distinct == 5) {
        if (hi - lo == 4) { straight = 1; shigh = hi; }
        else if (cnt[12] && cnt[0] && cnt[1] && cnt[2] && cnt[3]) { straight = 1; shigh = 3; }
    }
    int cat, k[5] = {0, 0, 0, 0, 0};
    if (straight && flush) { cat = 8; k[0] = shigh; }
    else if (straight)     { cat = 4; k[0] = shigh; }
    else {
        /* order ranks by (multiplicity desc, rank desc) */
        int ord[5], n = 0;
        for (int m = 4; m >= 1; m--)
            for (int q = 12; q >= 0; q--)
                if (cnt[q] == m) ord[n++] = q;
        int m0 = cnt[ord[0]], m1 = n > 1 ? cnt[ord[1]] : 0;
        if (m0 == 4)                 { cat = 7; k[0] = ord[0]; k[1] = ord[1]; }
        else if (m0 == 3 && m1 == 2) { cat = 6; k[0] = ord[0]; k[1] = ord[1]; }
        else if (flush)              { cat = 5; for (int i = 0; i < 5; i++) k[i] = ord[i]; }
        else if (m0 == 3)            { cat = 3; k[0] = ord[0]; k[1] = ord[1]; k[2] = ord[2]; }
        else if (m0 == 2 && m1 == 2) { cat = 2; k[0] = ord[0]; k[1] = ord[1]; k[2] = ord[2]; }
        else if (m0 == 2)            { cat = 1; for (int i = 0; i < 4; i++) k[i] = ord[i]; }
        else                         { cat = 0; for (int i = 0; i < 5; i++) k[i] = ord[i]; }
    }
    return (cat << 20) | (k[0] << 16) | (k[1] << 12) | (k[2] << 8) | (k[3] << 4) | k[4];
}

/* Seven-card value: the best of the 21 five-card subsets. */
int ora_eval7(const int* c) {
    int best = -1, sub[5];
    for (int x = 0; x < 7; x++)
        for (int y = x + 1; y < 7; y++) {
            int n = 0;
            for (int i = 0; i < 7; i++) if (i != x && i != y) sub[n++] = c[i];
            int v = ora_eval5(sub);
            if (v > best) best = v;
        }
    return best;
}

/* Category histogram over every n-card hand from the 52-card deck
 * (n = 5 or 7).  Used to pin the evaluator to the published counts. */
void ora_category_counts(int n, int64_t* out9) {
    int64_t tot[9] = {0};
    #pragma omp parallel
    {
        int64_t loc[9] = {0};
        int c[7];
        #pragma omp for schedule(dynamic)
        for (int a = 0; a < 52; a++) {
            c[0] = a;
            for (int b = a + 1; b < 52; b++) { c[1] = b;
            for (int d = b + 1; d < 52; d++) { c[2] = d;
            for (int e = d + 1; e < 52; e++) { c[3] = e;
            for (int f = e + 1; f < 52; f++) { c[4] = f;
                if (n == 5) { loc[ora_eval5(c) >> 20]++; continue; }
                for (int g = f + 1; g < 52; g++) { c[5] = g;
                for (int h = g + 1; h < 52; h++) { c[6] = h;
                    loc[ora_eval7(c) >> 20]++;
                }}
            }}}}
        }
        #pragma omp critical
        for (int i = 0; i < 9; i++) tot[i] += loc[i];
    }
    memcpy(out9, tot, sizeof(tot));
}

/* Number of distinct five-card values (7462 classes expected). */
int ora_distinct5(void) {
    const int N = 1 << 24;
    unsigned char* seen = calloc(N, 1);
    int c[5], cnt = 0;
    for (c[0] = 0; c[0] < 52; c[0]++)
    for (c[1] = c[0] + 1; c[1] < 52; c[1]++)
    for (c[2] = c[1] + 1; c[2] < 52; c[2]++)
    for (c[3] = c[2] + 1; c[3] < 52; c[3]++)
    for (c[4] = c[3] + 1; c[4] < 52; c[4]++) {
        int v = ora_eval5(c);
        if (!seen[v]) { seen[v] = 1; cnt++; }
    }
    free(seen);
    return cnt;
}

void ora_eval7_batch(const int32_t* cards, int64_t n, int32_t* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int c[7];
        for (int j = 0; j < 7; j++) c[j] = cards[i * 7 + j];
        out[i] = ora_eval7(c);
    }
}

/* ------------------------------------------------------------- game tree */
enum { T_DEC = 0, T_FOLD = 1, T_SHOW = 2, T_CHANCE = 3, T_LEAF = 4, T_ALLIN = 5 };

typedef struct {
    int type, player, depth, chance_card;
    int64_t c[2];
    int nb, board[5];
    int nch, chcap, *ch;      /* children during construction (pool ids) */
} tnode;

typedef struct {
    /* rules */
    int kuhn;
    int64_t pot, cap;         /* cap = pot/2 + effective stack (max contribution) */
    int n_sizes, size_pct[8], allin, max_raises, depth_limit;
    int err;                  /* set when the spec asks for something the builder does not support */
    /* pool */
    int n, capn;
    tnode* v;
} builder;

static int b_new(builder* b, int type, int player, int depth, const int64_t c[2],
                 int nb, const int* board, int chance_card) {
    if (b->n == b->capn) {
        b->capn = b->capn ? 2 * b->capn : 1024;
        b->v = realloc(b->v, sizeof(tnode) * b->capn);
    }
    tnode* t = &b->v[b->n];
    memset(t, 0, sizeof(*t));
    t->type = type; t->player = player; t->depth = depth; t->chance_card = chance_card;
    t->c[0] = c[0]; t->c[1] = c[1];
    t->nb = nb;
    for (int i = 0; i < nb; i++) t->board[i] = board[i];
    return b->n++;
}

static void b_addch(builder* b, int parent, int child) {
    tnode* t = &b->v[parent];
    if (t->nch == t->chcap) {
        t->chcap = t->chcap ? 2 * t->chcap : 8;
        t->ch = realloc(t->ch, sizeof(int) * t->chcap);
    }
    t->ch[t->nch++] = child;
}

typedef struct { int nb, board[5]; int64_t c[2]; int p, nraises, depth, chance_card; } bstate;

static int b_decision(builder* b, bstate s);

/* The betting round is over (check-check or a call).  River: showdown.
 * Someone all in: deal the rest of the board, then showdown (or an exact
 * all-in leaf when the tree is depth-limited).  Otherwise: a leaf when the
 * tree stops at this round, else a chance node dealing the next card. */
static int b_street_end(builder* b, bstate s) {
    if (b->kuhn || s.nb == 5)
        return b_new(b, T_SHOW, -1, s.depth, s.c, s.nb, s.board, s.chance_card);
    int allin = (s.c[0] >= b->cap || s.c[1] >= b->cap);
    /* Preflop (no board): only depth-limited trees whose betting never puts a
     * player all in are built; their leaves sit at the flop deal. */
    if (s.nb == 0 && (allin || !b->depth_limit)) {
        b->err = 1;
        return b_new(b, T_LEAF, -1, s.depth, s.c, s.nb, s.board, s.chance_card);
    }
    if (b->depth_limit)
        return b_new(b, allin ? T_ALLIN : T_LEAF, -1, s.depth, s.c, s.nb, s.board, s.chance_card);
    int id = b_new(b, T_CHANCE, -1, s.depth, s.c, s.nb, s.board, s.chance_card);
    uint64_t used = 0;
    for (int i = 0; i < s.nb; i++) used |= 1ULL << s.board[i];
    for (int card = 0; card < 52; card++) {
        if (used >> card & 1) continue;
        bstate t = s;
        t.board[t.nb++] = card;
        t.depth = s.depth + 1;
        t.chance_card = card;
        int ch;
        if (allin) ch = b_street_end(b, t);
        else { t.p = 0; t.nraises = 0; ch = b_decision(b, t); }
        b_addch(b, id, ch);
    }
    return id;
}

static int cmp64(const void* x, const void* y) {
    int64_t a = *(const int64_t*)x, c = *(const int64_t*)y;
    return (a > c) - (a < c);
}

/* A betting decision.  Facing a bet: fold, call, then raises; otherwise
 * check, then bets.  A sized bet or raise of pct% puts in the amount to call
 * plus pct% of the pot after that call (integer chips, half rounded up),
 * capped at the stack.  Bets and raises are counted per street, the opening
 * bet included, and allowed while the count is below max_raises and the
 * opponent still has chips behind. */
static int b_decision(builder* b, bstate s) {
    int p = s.p, o = 1 - p;
    int id = b_new(b, T_DEC, p, s.depth, s.c, s.nb, s.board, s.chance_card);
    int64_t to_call = s.c[o] - s.c[p];
    bstate base = s;
    base.depth = s.depth + 1;
    base.chance_card = -1;
    if (to_call > 0) {
        int f = b_new(b, T_FOLD, p, base.depth, s.c, s.nb, s.board, -1);
        b_addch(b, id, f);
        bstate t = base;
        t.c[p] = s.c[o];
        b_addch(b, id, b_street_end(b, t));
    } else {
        bstate t = base;
        int ch;
        if (p == 1) ch = b_street_end(b, t);
        else { t.p = 1; ch = b_decision(b, t); }
        b_addch(b, id, ch);
    }
    if (s.nraises < b->max_raises && s.c[o] < b->cap) {
        int64_t cand[10];
        int nc = 0;
        int64_t pot_after_call = s.c[0] + s.c[1] + to_call;
        for (int k = 0; k < b->n_sizes; k++) {
            int64_t put = to_call + (b->size_pct[k] * pot_after_call + 50) / 100;
            int64_t tgt = s.c[p] + put;
            if (tgt > b->cap) tgt = b->cap;
            cand[nc++] = tgt;
        }
        if (b->allin) cand[nc++] = b->cap;
        qsort(cand, nc, sizeof(int64_t), cmp64);
        int64_t last = -1;
        for (int k = 0; k < nc; k++) {
            if (cand[k] <= s.c[o] || cand[k] == last) continue;
            last = cand[k];
            bstate t = base;
            t.c[p] = cand[k];
            t.nraises = s.nraises + 1;
            t.p = o;
            b_addch(b, id, b_decision(b, t));
        }
    }
    return id;
}

/* ------------------------------------------------------------- the game */
typedef struct {
    int type, player, parent, action, depth, chance_card;
    int first_child, n_child;
    int64_t c[2];
    int nb, board[5];
    uint64_t bmask;
    int bid;     /* index into the rank tables (showdown / leaf boards) */
    int rs;      /* first regret row (decision nodes), else -1 */
} onode;

typedef struct {
    int kuhn;
    int n;
    onode* nd;
    int nh;                       /* number of private hands (1326, or 3 for Kuhn) */
    uint64_t hmask[NCOMBO];
    int hvalid[NCOMBO];
    int nrows;                    /* total regret rows = sum of actions */
    int nboards;
    uint64_t* bmasks;
    int32_t* rank;                /* [nboards][nh] */
    int counts[6];
    int n_levels;
    double** eq;                  /* per board: [nh][nh] check-down equity, or NULL */
} ogame;

static void game_free(ogame* g) {
    if (!g) return;
    if (g->eq) for (int i = 0; i < g->nboards; i++) free(g->eq[i]);
    free(g->nd); free(g->bmasks); free(g->rank); free(g->eq); free(g);
}

static int board_id(ogame* g, uint64_t m) {
    for (int i = 0; i < g->nboards; i++) if (g->bmasks[i] == m) return i;
    g->bmasks = realloc(g->bmasks, sizeof(uint64_t) * (g->nboards + 1));
    g->bmasks[g->nboards] = m;
    return g->nboards++;
}

static ogame* game_from_builder(builder* b, int kuhn, const int* root_board, int root_nb) {
    ogame* g = calloc(1, sizeof(ogame));
    g->kuhn = kuhn;
    g->n = b->n;
    g->nd = calloc(b->n, sizeof(onode));
    /* breadth-first renumbering from the root (pool id 0) */
    int* order = malloc(sizeof(int) * b->n);
    int* newid = malloc(sizeof(int) * b->n);
    int* par = malloc(sizeof(int) * b->n);
    int* act = malloc(sizeof(int) * b->n);
    int head = 0, tail = 0;
    order[tail++] = 0; par[0] = -1; act[0] = -1;
    while (head < tail) {
        int u = order[head++];
        for (int k = 0; k < b->v[u].nch; k++) {
            int w = b->v[u].ch[k];
            par[w] = u; act[w] = k;
            order[tail++] = w;
        }
    }
    for (int i = 0; i < b->n; i++) newid[order[i]] = i;
    int rows = 0;
    for (int i = 0; i < b->n; i++) {
        tnode* t = &b->v[order[i]];
        onode* o = &g->nd[i];
        o->type = t->type; o->player = t->player; o->depth = t->depth;
        o->chance_card = t->chance_card;
        o->c[0] = t->c[0]; o->c[1] = t->c[1];
        o->nb = t->nb;
        o->bmask = 0;
        for (int k = 0; k < t->nb; k++) { o->board[k] = t->board[k]; o->bmask |= 1ULL << t->board[k]; }
        o->parent = par[order[i]] < 0 ? -1 : newid[par[order[i]]];
        o->action = act[order[i]];
        o->n_child = t->nch;
        o->first_child = t->nch ? newid[t->ch[0]] : -1;
        for (int k = 1; k < t->nch; k++)
            if (newid[t->ch[k]] != o->first_child + k) abort();   /* BFS keeps siblings adjacent */
        o->rs = -1;
        if (o->type == T_DEC) { o->rs = rows; rows += o->n_child; }
        if (o->depth + 1 > g->n_levels) g->n_levels = o->depth + 1;
        g->counts[o->type]++;
    }
    g->nrows = rows;
    free(order); free(newid); free(par); free(act);
    for (int i = 0; i < b->n; i++) free(b->v[i].ch);
    free(b->v);

    /* private hands */
    uint64_t rootmask = 0;
    for (int i = 0; i < root_nb; i++) rootmask |= 1ULL << root_board[i];
    if (kuhn) {
        g->nh = 3;
        for (int h = 0; h < 3; h++) { g->hmask[h] = 1ULL << h; g->hvalid[h] = 1; }
    } else {
        g->nh = NCOMBO;
        for (int a = 1; a < 52; a++)
            for (int c = 0; c < a; c++) {
                int h = combo_index(a, c);
                g->hmask[h] = (1ULL << a) | (1ULL << c);
                g->hvalid[h] = (g->hmask[h] & rootmask) == 0;
            }
    }
    /* rank tables for every board that ends in a showdown or a leaf */
    for (int i = 0; i < g->n; i++) {
        onode* o = &g->nd[i];
        o->bid = -1;
        if (o->type == T_SHOW || o->type == T_LEAF || o->type == T_ALLIN) o->bid = board_id(g, o->bmask);
    }
    g->rank = malloc(sizeof(int32_t) * (size_t)(g->nboards ? g->nboards : 1) * g->nh);
    for (int bi = 0; bi < g->nboards; bi++) {
        for (int h = 0; h < g->nh; h++) {
            int32_t v = -1;
            if (kuhn) v = h;
            else if ((g->hmask[h] & g->bmasks[bi]) == 0 && __builtin_popcountll(g->bmasks[bi]) == 5) {
                int c[7], n = 0;
                for (int k = 0; k < 52; k++) if ((g->hmask[h] | g->bmasks[bi]) >> k & 1) c[n++] = k;
                v = ora_eval7(c);
            }
            g->rank[(size_t)bi * g->nh + h] = v;
        }
    }
    return g;
}

/* Pairwise check-down equity on a board of 3 or 4 cards: the mean over every
 * completion of the board by cards held by neither player of
 * sign(value(h) - value(o)).  This is the exact value of an all-in leaf per
 * unit contribution, and the stub leaf used for depth-limited parity. */
static double* game_eq(ogame* g, int bi) {
    size_t nh = g->nh;
    if (!g->eq) g->eq = calloc(g->nboards, sizeof(double*));
    if (g->eq[bi]) return g->eq[bi];
    double* E = calloc(nh * nh, sizeof(double));
    g->eq[bi] = E;
    uint64_t bm = g->bmasks[bi];
    int nb = __builtin_popcountll(bm);
    int need = 5 - nb;
    int rest[52], nr = 0;
    for (int k = 0; k < 52; k++) if (!(bm >> k & 1)) rest[nr++] = k;
    int nrun = need == 1 ? nr : nr * (nr - 1) / 2;
    /* ranks per completion */
    int32_t* rk = malloc(sizeof(int32_t) * nrun * nh);
    uint64_t* rm = malloc(sizeof(uint64_t) * nrun);
    int q = 0;
    for (int x = 0; x < nr; x++)
        for (int y = (need == 1 ? x : x + 1); y < (need == 1 ? x + 1 : nr); y++) {
            uint64_t m = bm | (1ULL << rest[x]) | (1ULL << rest[y]);
            rm[q] = m;
            q++;
        }
    #pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < nrun; r++) {
        for (size_t h = 0; h < nh; h++) {
            int32_t v = -1;
            if (g->hvalid[h] && !(g->hmask[h] & rm[r])) {
                int c[7], n = 0;
                uint64_t all = g->hmask[h] | rm[r];
                for (int k = 0; k < 52; k++) if (all >> k & 1) c[n++] = k;
                v = ora_eval7(c);
            }
            rk[(size_t)r * nh + h] = v;
        }
    }
    #pragma omp parallel for schedule(dynamic)
    for (size_t h = 0; h < nh; h++) {
        if (!g->hvalid[h]) continue;
        for (size_t o = 0; o < nh; o++) {
            if (!g->hvalid[o] || (g->hmask[h] & g->hmask[o])) continue;
            double s = 0; int cnt = 0;
            for (int r = 0; r < nrun; r++) {
                if (rm[r] & (g->hmask[h] | g->hmask[o])) continue;
                int32_t a = rk[(size_t)r * nh + h], c = rk[(size_t)r * nh + o];
                s += (a > c) - (a < c);
                cnt++;
            }
            E[h * nh + o] = s / cnt;
        }
    }
    free(rk); free(rm);
    return E;
}

/* Equity tables are built before any parallel walk reads them. */
static void game_prepare_leaves(ogame* g) {
    for (int i = 0; i < g->n; i++)
        if ((g->nd[i].type == T_LEAF || g->nd[i].type == T_ALLIN) && g->nd[i].nb > 0) game_eq(g, g->nd[i].bid);
}

/* Build a hold'em subgame.  Returns NULL on invalid input. */
ogame* ora_build_tree(int n_board, const int32_t* board, int64_t pot, int64_t stack0, int64_t stack1,
                      int n_sizes, const int32_t* size_pct, int allin, int max_raises, int depth_limit) {
    if ((n_board != 0 && n_board < 3) || n_board > 5 || pot <= 0 || (pot & 1) || stack0 < 0 || stack1 < 0)
        return NULL;
    if (n_sizes < 0 || n_sizes > 8 || max_raises < 0) return NULL;
    uint64_t m = 0;
    for (int i = 0; i < n_board; i++) {
        if (board[i] < 0 || board[i] >= 52 || (m >> board[i] & 1)) return NULL;
        m |= 1ULL << board[i];
    }
    builder b;
    memset(&b, 0, sizeof(b));
    b.pot = pot;
    b.cap = pot / 2 + (stack0 < stack1 ? stack0 : stack1);
    b.n_sizes = n_sizes;
    for (int i = 0; i < n_sizes; i++) b.size_pct[i] = size_pct[i];
    b.allin = allin; b.max_raises = max_raises; b.depth_limit = depth_limit;
    bstate s;
    memset(&s, 0, sizeof(s));
    s.nb = n_board;
    for (int i = 0; i < n_board; i++) s.board[i] = board[i];
    s.c[0] = s.c[1] = pot / 2;
    s.p = 0; s.nraises = 0; s.depth = 0; s.chance_card = -1;
    b_decision(&b, s);
    if (b.err) {
        for (int i = 0; i < b.n; i++) free(b.v[i].ch);
        free(b.v);
        return NULL;
    }
    return game_from_builder(&b, 0, board, n_board);
}

/* Kuhn poker (Kuhn 1950) on the same engine: a 3-card deck J<Q<K, one card
 * each, ante 1 each, one bet of 1 chip and no raise.  Private "hands" are the
 * single cards; showdown compares them. */
ogame* ora_build_kuhn(void) {
    builder b;
    memset(&b, 0, sizeof(b));
    b.kuhn = 1; b.pot = 2; b.cap = 2;
    b.n_sizes = 1; b.size_pct[0] = 50; b.allin = 0; b.max_raises = 1; b.depth_limit = 0;
    bstate s;
    memset(&s, 0, sizeof(s));
    s.c[0] = s.c[1] = 1; s.chance_card = -1;
    b_decision(&b, s);
    return game_from_builder(&b, 1, NULL, 0);
}

/* Online pruning (Sec. 5, "Online Pruning"): actions removed before the
 * iterations begin.  removed[n] != 0 on a child of a decision node drops the
 * action leading to n together with n's whole subtree; every other node is
 * copied as it is, its children kept in their order, and the reduced game is
 * renumbered breadth-first like any built tree.  Returns NULL when a flag
 * sits on a node whose parent is not a decision node, or when a decision
 * node would keep no action. */
ogame* ora_tree_prune(const ogame* g, const unsigned char* removed) {
    builder b;
    memset(&b, 0, sizeof(b));
    b.kuhn = g->kuhn;
    int* pool = malloc(sizeof(int) * g->n);
    int bad = 0;
    for (int i = 0; i < g->n && !bad; i++) {
        const onode* o = &g->nd[i];
        if (removed[i] && (o->parent < 0 || g->nd[o->parent].type != T_DEC)) { bad = 1; break; }
        if (removed[i] || (o->parent >= 0 && pool[o->parent] < 0)) { pool[i] = -1; continue; }
        pool[i] = b_new(&b, o->type, o->player, o->depth, o->c, o->nb, o->board, o->chance_card);
        if (o->parent >= 0) b_addch(&b, pool[o->parent], pool[i]);
    }
    for (int i = 0; i < g->n && !bad; i++)
        if (pool[i] >= 0 && g->nd[i].type == T_DEC && b.v[pool[i]].nch == 0) bad = 1;
    free(pool);
    if (bad) {
        for (int i = 0; i < b.n; i++) free(b.v[i].ch);
        free(b.v);
        return NULL;
    }
    return game_from_builder(&b, g->kuhn, g->kuhn ? NULL : g->nd[0].board, g->kuhn ? 0 : g->nd[0].nb);
}

/* Dominance test of online pruning (Sec. 5): at a decision node of player p
 * an action a is dominated for hand h when its optimistic value hi[a][h]
 * lies below the pessimistic value lo[b][h] of one of its siblings b.  The
 * action is removed from the public tree when it is dominated for every hand
 * h of p's range (r_p(h) > 0) that the node's board does not block; a node
 * where p holds no such hand removes nothing.  lo, hi: [n][nh], row = the
 * child node the action leads to; removed: [n]. */
void ora_prune_dominated(const ogame* g, const double* ranges, const double* lo, const double* hi,
                         unsigned char* removed) {
    int nh = g->nh;
    memset(removed, 0, (size_t)g->n);
    for (int i = 0; i < g->n; i++) {
        const onode* o = &g->nd[i];
        if (o->type != T_DEC) continue;
        int p = o->player, fc = o->first_child, A = o->n_child;
        for (int a = 0; a < A; a++) {
            int any = 0, all = 1;
            for (int h = 0; h < nh && all; h++) {
                if (!g->hvalid[h] || !(ranges[p * nh + h] > 0) || (g->hmask[h] & o->bmask)) continue;
                any = 1;
                int dom = 0;
                for (int b = 0; b < A && !dom; b++)
                    if (b != a && hi[(size_t)(fc + a) * nh + h] < lo[(size_t)(fc + b) * nh + h]) dom = 1;
                if (!dom) all = 0;
            }
            removed[fc + a] = (unsigned char)(any && all);
        }
    }
}

void ora_tree_free(ogame* g) { game_free(g); }

/* counts: nodes, decision, fold, showdown, chance, leaf, allin-leaf, levels, rows */
void ora_tree_info(const ogame* g, int64_t* out) {
    out[0] = g->n;
    for (int k = 0; k < 6; k++) out[1 + k] = g->counts[k];
    out[7] = g->n_levels;
    out[8] = g->nrows;
}

void ora_tree_export(const ogame* g, int32_t* type, int32_t* player, int32_t* parent, int32_t* action,
                     int32_t* depth, int64_t* contrib, int32_t* chance_card, int32_t* first_child,
                     int32_t* n_child) {
    for (int i = 0; i < g->n; i++) {
        const onode* o = &g->nd[i];
        type[i] = o->type; player[i] = o->player; parent[i] = o->parent; action[i] = o->action;
        depth[i] = o->depth; contrib[2 * i] = o->c[0]; contrib[2 * i + 1] = o->c[1];
        chance_card[i] = o->chance_card; first_child[i] = o->first_child; n_child[i] = o->n_child;
    }
}

/* ------------------------------------------------------------- solver */
enum { LEAF_EQUITY = 0, LEAF_TABLE = 1, LEAF_FLOP = 2 };

/* Stage-7 update rules (Sec. 4.4: the CFR variant only changes Stage 7).
 *   DCFR  (Brown & Sandholm 2019): discounted regrets and average, see
 *         iterate_once.
 *   CFR+  (Tammelin 2014): cumulative regrets floored at zero after every
 *         update; the average strategy weights iteration t by t.
 *   PCFR+ (Farina, Kroer & Sandholm 2021): predictive regret matching -- the
 *         strategy of iteration t matches [R^{t-1} + m^t]^+ with the
 *         prediction m^t = r^{t-1}, the last instantaneous regret; regrets
 *         floored at zero; the average weights iteration t by t^2. */
enum { V_DCFR = 0, V_CFRPLUS = 1, V_PCFRPLUS = 2 };

/* Relative size below which an instantaneous regret counts as an exact tie. */
#define TIE_REL 1e-10

typedef struct {
    ogame* g;
    double alpha, beta, gamma;
    int variant;
    double rng[2][NCOMBO];
    double *R, *S, *sig, *rinst, *sadd, *pred;
    double* cva;          /* per row and hand: the counterfactual value of the row's action (this half-step) */
    double cfv[2][NCOMBO];
    int64_t t;
    int support_only;
    int alternating;       /* 0: both players from the same strategies; 1: player 0, then player 1 */
    double thr0;           /* dynamic threshold of iteration t: thr0 / sqrt(t); 0 = off */
    unsigned char* row_player;  /* [nrows]: the player acting at the row's node */
    unsigned char* tmask;  /* optional [2][nh]: traverser hands to evaluate (NULL = all) */
    int leaf_kind;
    double* leaf_ev;      /* LEAF_TABLE: [leaf node][player][card][nh] expected value per pot */
    /* LEAF_FLOP (preflop leaves): per leaf and player, sums of the expected
     * value E(h | g) over the flops g that share no card with h -- in all
     * (A[nh]), holding card x (B[nh][52]), holding both cards of combo xy
     * (D[nh][nh]) -- so that a history's mean over the flops clear of both
     * hands follows by inclusion-exclusion */
    double *flopA, *flopB, *flopD;
    int* leaf_slot;       /* node -> leaf slot */
    int nleaf;
} osolver;

static int compat(const ogame* g, int a, int b) { return (g->hmask[a] & g->hmask[b]) == 0; }

osolver* ora_solver_create(ogame* g, const double* ranges, double alpha, double beta, double gamma,
                           int support_only) {
    osolver* s = calloc(1, sizeof(osolver));
    s->g = g; s->alpha = alpha; s->beta = beta; s->gamma = gamma;
    s->support_only = support_only;
    for (int p = 0; p < 2; p++)
        for (int h = 0; h < g->nh; h++) s->rng[p][h] = g->hvalid[h] ? ranges[p * g->nh + h] : 0.0;
    size_t n = (size_t)g->nrows * g->nh;
    s->R = calloc(n, sizeof(double)); s->S = calloc(n, sizeof(double));
    s->sig = calloc(n, sizeof(double)); s->rinst = calloc(n, sizeof(double));
    s->sadd = calloc(n, sizeof(double));
    s->cva = calloc(n, sizeof(double));
    s->pred = calloc(n, sizeof(double));
    s->row_player = calloc(g->nrows > 0 ? g->nrows : 1, 1);
    for (int i = 0; i < g->n; i++)
        if (g->nd[i].type == T_DEC)
            for (int a = 0; a < g->nd[i].n_child; a++) s->row_player[g->nd[i].rs + a] = (unsigned char)g->nd[i].player;
    s->leaf_slot = malloc(sizeof(int) * g->n);
    for (int i = 0; i < g->n; i++) {
        s->leaf_slot[i] = -1;
        if (g->nd[i].type == T_LEAF) s->leaf_slot[i] = s->nleaf++;
    }
    game_prepare_leaves(g);
    return s;
}

void ora_solver_free(osolver* s) {
    if (!s) return;
    free(s->R); free(s->S); free(s->sig); free(s->rinst); free(s->sadd); free(s->pred); free(s->cva);
    free(s->leaf_ev); free(s->leaf_slot); free(s->tmask); free(s->row_player);
    free(s->flopA); free(s->flopB); free(s->flopD); free(s);
}

/* Restrict the traverser's hands whose values and regrets are computed (the
 * opponent's range is always used in full).  Regrets of the skipped hands
 * stay zero, so this is only meaningful for a single iteration from the
 * initial state or for hands whose rows are compared alone. */
void ora_set_traverser_hands(osolver* s, const unsigned char* mask) {
    size_t n = (size_t)2 * s->g->nh;
    if (!s->tmask) s->tmask = malloc(n);
    memcpy(s->tmask, mask, n);
}

/* Threshold of iteration t (t >= 1): thr0 / sqrt(t). */
static double threshold_at(const osolver* s, int64_t t) {
    return s->thr0 > 0 && t > 0 ? s->thr0 / sqrt((double)t) : 0.0;
}
static const double* matched_regrets(const osolver* s, double* tmp);

/* Regret matching (eq. rm): positive part normalised, uniform if none.
 * With a threshold thr > 0 (dynamic thresholding, cited in Sec. 2): every
 * action whose probability is below thr is set to 0 and the remaining ones
 * are renormalised (the largest is at least 1/A > thr, so one stays). */
static void regret_match(const double* R, double* out, int A, int nh, int h, double thr) {
    double den = 0;
    for (int a = 0; a < A; a++) { double x = R[(size_t)a * nh + h]; if (x > 0) den += x; }
    for (int a = 0; a < A; a++) {
        double x = R[(size_t)a * nh + h];
        out[(size_t)a * nh + h] = den > 0 ? (x > 0 ? x / den : 0.0) : 1.0 / A;
    }
    if (thr > 0) {
        double keep = 0;
        for (int a = 0; a < A; a++) {
            double* q = &out[(size_t)a * nh + h];
            if (*q < thr) *q = 0.0;
            keep += *q;
        }
        for (int a = 0; a < A; a++) out[(size_t)a * nh + h] /= keep;
    }
}

static void strategy_rows(const ogame* g, const double* src, double* dst, int normalise_sum, double thr) {
    /* normalise_sum = 0: regret matching of src (threshold thr); 1: src / sum(src), uniform if zero */
    for (int i = 0; i < g->n; i++) {
        const onode* o = &g->nd[i];
        if (o->type != T_DEC) continue;
        int A = o->n_child;
        const double* x = src + (size_t)o->rs * g->nh;
        double* y = dst + (size_t)o->rs * g->nh;
        for (int h = 0; h < g->nh; h++) {
            if (!normalise_sum) { regret_match(x, y, A, g->nh, h, thr); continue; }
            double den = 0;
            for (int a = 0; a < A; a++) den += x[(size_t)a * g->nh + h];
            for (int a = 0; a < A; a++)
                y[(size_t)a * g->nh + h] = den > 0 ? x[(size_t)a * g->nh + h] / den : 1.0 / A;
        }
    }
}

/* Leaf value of one history (hi for player i, ho for the opponent), per
 * history and in chips. */
static double leaf_value(osolver* s, int n, int i, int hi, int ho) {
    ogame* g = s->g;
    const onode* o = &g->nd[n];
    if (o->type == T_ALLIN || s->leaf_kind == LEAF_EQUITY) {
        double* E = g->eq[o->bid];
        return (double)o->c[0] * E[(size_t)hi * g->nh + ho];
    }
    int slot = s->leaf_slot[n];
    double pot = (double)(o->c[0] + o->c[1]);
    if (o->nb == 0) {
        /* preflop leaf: mean over the C(48, 3) flops that neither hand touches
         * of pot * E_i(hi | flop); flops holding a card x or y of the
         * opponent's hand are taken out of the sum over all flops clear of hi
         * by inclusion-exclusion (a flop holding both is removed twice) */
        if (s->leaf_kind != LEAF_FLOP) abort();   /* refused before iterating */
        size_t k = (size_t)slot * 2 + i, nh = g->nh;
        int x = -1, y = -1;
        for (int c = 0; c < 52; c++)
            if (g->hmask[ho] >> c & 1) { if (y < 0) y = c; else x = c; }
        double acc = s->flopA[k * nh + hi] - s->flopB[(k * nh + hi) * 52 + x] - s->flopB[(k * nh + hi) * 52 + y] +
                     s->flopD[(k * nh + hi) * nh + combo_index(x, y)];
        return pot * acc / 17296.0;
    }
    /* LEAF_TABLE: the value network's expected value (per unit of pot) of
     * hand hi for player i after next card c, averaged over the cards that
     * neither hand holds: mean_c pot * EV_i(hi | c). */
    double acc = 0; int cnt = 0;
    uint64_t used = o->bmask | g->hmask[hi] | g->hmask[ho];
    for (int c = 0; c < 52; c++) {
        if (used >> c & 1) continue;
        acc += s->leaf_ev[(((size_t)slot * 2 + i) * 52 + c) * g->nh + hi];
        cnt++;
    }
    return pot * acc / cnt;
}

/* Value of one history below node n for traverser i holding hi against an
 * opponent holding ho; w is the opponent-and-chance reach of the history.
 * At the traverser's nodes the instantaneous regrets of its information set
 * (node n, hand hi) gain w * (v(child a) - v(n)). */
static double walk(osolver* s, int n, int i, int hi, int ho, double w) {
    ogame* g = s->g;
    const onode* o = &g->nd[n];
    switch (o->type) {
    case T_FOLD: {
        /* zero-sum: the folder loses what it has put in, the other wins it */
        double cf = (double)o->c[o->player];
        return o->player == i ? -cf : cf;
    }
    case T_SHOW: {
        int32_t a = g->rank[(size_t)o->bid * g->nh + hi], b = g->rank[(size_t)o->bid * g->nh + ho];
        return (double)o->c[0] * ((a > b) - (a < b));
    }
    case T_LEAF: case T_ALLIN:
        return leaf_value(s, n, i, hi, ho);
    case T_CHANCE: {
        uint64_t used = o->bmask | g->hmask[hi] | g->hmask[ho];
        int K = 0;
        for (int k = 0; k < o->n_child; k++) if (!(used >> g->nd[o->first_child + k].chance_card & 1)) K++;
        double v = 0;
        for (int k = 0; k < o->n_child; k++) {
            int ch = o->first_child + k;
            if (used >> g->nd[ch].chance_card & 1) continue;
            v += walk(s, ch, i, hi, ho, w / K) / K;
        }
        return v;
    }
    default: break;
    }
    int A = o->n_child;
    const double* sg = s->sig + (size_t)o->rs * g->nh;
    if (o->player == i) {
        double va[64], v = 0;
        for (int a = 0; a < A; a++) {
            va[a] = walk(s, o->first_child + a, i, hi, ho, w);
            v += sg[(size_t)a * g->nh + hi] * va[a];
        }
        /* instantaneous regret v(I.a) - v(I), written as sum_b sigma_b (v_a - v_b):
         * the same quantity (the sigma_b sum to one), but actions whose values are
         * exactly tied get exactly zero regret whatever the summation order, so
         * regret matching does not flip on the sign of a rounding residue */
        double* ri = s->rinst + (size_t)o->rs * g->nh;
        double* cv = s->cva + (size_t)o->rs * g->nh;
        for (int a = 0; a < A; a++) {
            double r = 0;
            for (int b = 0; b < A; b++) r += sg[(size_t)b * g->nh + hi] * (va[a] - va[b]);
            ri[(size_t)a * g->nh + hi] += w * r;
            cv[(size_t)a * g->nh + hi] += w * va[a];
        }
        return v;
    }
    double v = 0;
    for (int a = 0; a < A; a++) {
        double p = sg[(size_t)a * g->nh + ho];
        if (p == 0) continue;
        v += p * walk(s, o->first_child + a, i, hi, ho, w * p);
    }
    return v;
}

/* Own reach of hand h for player p (Stage 1): product of p's own action
 * probabilities from the root, starting at the root range.  At p's decision
 * nodes the reach-weighted strategy is added to the average-strategy
 * increment once per information set. */
static void own_reach(osolver* s, int n, int p, int h, double pi) {
    ogame* g = s->g;
    const onode* o = &g->nd[n];
    if (o->type == T_CHANCE) {
        for (int k = 0; k < o->n_child; k++) {
            int ch = o->first_child + k;
            if (g->hmask[h] >> g->nd[ch].chance_card & 1) continue;
            own_reach(s, ch, p, h, pi);
        }
        return;
    }
    if (o->type != T_DEC) return;
    int A = o->n_child;
    const double* sg = s->sig + (size_t)o->rs * g->nh;
    if (o->player == p) {
        double* sa = s->sadd + (size_t)o->rs * g->nh;
        for (int a = 0; a < A; a++) {
            double q = sg[(size_t)a * g->nh + h];
            sa[(size_t)a * g->nh + h] += pi * q;
            own_reach(s, o->first_child + a, p, h, pi * q);
        }
    } else {
        for (int a = 0; a < A; a++) own_reach(s, o->first_child + a, p, h, pi);
    }
}

void ora_set_variant(osolver* s, int variant) { s->variant = variant; }
void ora_set_alternating(osolver* s, int on) { s->alternating = on; }
void ora_set_threshold(osolver* s, double thr0) { s->thr0 = thr0; }

/* Regrets the next strategy is matched on: R, or R + m for PCFR+. */
static const double* matched_regrets(const osolver* s, double* tmp) {
    if (s->variant != V_PCFRPLUS) return s->R;
    size_t n = (size_t)s->g->nrows * s->g->nh;
    for (size_t k = 0; k < n; k++) tmp[k] = s->R[k] + s->pred[k];
    return tmp;
}

/* One iteration.  Simultaneous updates: both players' regrets and averages
 * from the same strategies sigma^t.  Alternating updates: player 0 is
 * updated first; player 1 then traverses against player 0's new strategy
 * (matched on the just-updated regrets); both halves use iteration t's
 * discounts, and each updates only its own player's rows. */
static void half_step(osolver* s, int upd, double t);

static void iterate_once(osolver* s) {
    s->t++;
    double t = (double)s->t;
    if (!s->alternating) {
        half_step(s, -1, t);
    } else {
        half_step(s, 0, t);
        half_step(s, 1, t);
    }
}

/* Traverse for the players in {upd} (both when upd < 0) and update their rows. */
static void half_step(osolver* s, int upd, double t) {
    ogame* g = s->g;
    int nh = g->nh;
    double ta = pow(t, s->alpha), tb = pow(t, s->beta);
    double dpos = ta / (ta + 1.0), dneg = tb / (tb + 1.0);
    double davg = pow(t / (t + 1.0), s->gamma);
    size_t n = (size_t)g->nrows * nh;
    strategy_rows(g, matched_regrets(s, s->rinst), s->sig, 0, threshold_at(s, (int64_t)t));
    memset(s->rinst, 0, n * sizeof(double));
    memset(s->sadd, 0, n * sizeof(double));
    memset(s->cva, 0, n * sizeof(double));
    for (int i = 0; i < 2; i++) {
        if (upd >= 0 && i != upd) continue;
        int op = 1 - i;
        int* olist = malloc(sizeof(int) * nh);
        int no = 0;
        for (int h = 0; h < nh; h++) if (g->hvalid[h] && s->rng[op][h] > 0) olist[no++] = h;
        #pragma omp parallel for schedule(dynamic)
        for (int hi = 0; hi < nh; hi++) {
            s->cfv[i][hi] = 0;
            if (!g->hvalid[hi]) continue;
            if (s->support_only && !(s->rng[i][hi] > 0)) continue;
            if (s->tmask && !s->tmask[i * nh + hi]) continue;
            double acc = 0;
            for (int k = 0; k < no; k++) {
                int ho = olist[k];
                if (!compat(g, hi, ho)) continue;
                double w = s->rng[op][ho];
                acc += w * walk(s, 0, i, hi, ho, w);
            }
            s->cfv[i][hi] = acc;
        }
        free(olist);
    }
    for (int p = 0; p < 2; p++) {
        if (upd >= 0 && p != upd) continue;
        #pragma omp parallel for schedule(dynamic)
        for (int h = 0; h < nh; h++)
            if (g->hvalid[h]) own_reach(s, 0, p, h, s->rng[p][h]);
    }
    /* Ties: an information set's instantaneous regret whose magnitude is at
     * most TIE_REL of the largest counterfactual value of its actions is an
     * exact tie (zero).  Regrets that vanish in exact arithmetic come out of
     * any summation order as residues of either sign, and regret matching
     * would follow that sign. */
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < g->n; i++) {
        const onode* o = &g->nd[i];
        if (o->type != T_DEC || (upd >= 0 && o->player != upd)) continue;
        const int A = o->n_child;
        for (int h = 0; h < nh; h++) {
            double mx = 0;
            for (int a = 0; a < A; a++) {
                const double c = fabs(s->cva[((size_t)o->rs + a) * nh + h]);
                if (c > mx) mx = c;
            }
            for (int a = 0; a < A; a++) {
                double* ri = &s->rinst[((size_t)o->rs + a) * nh + h];
                if (fabs(*ri) <= TIE_REL * mx) *ri = 0.0;
            }
        }
    }
    #pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; k++) {
        if (upd >= 0 && s->row_player[k / nh] != upd) continue;
        double r = s->R[k] + s->rinst[k];
        if (s->variant == V_DCFR) {
            s->R[k] = r * (r > 0 ? dpos : dneg);
            s->S[k] = (s->S[k] + s->sadd[k]) * davg;
        } else {
            s->R[k] = r > 0 ? r : 0.0;
            s->S[k] += (s->variant == V_CFRPLUS ? t : t * t) * s->sadd[k];
            s->pred[k] = s->rinst[k];
        }
    }
}

int ora_max_threads(void) { return omp_get_max_threads(); }

void ora_iterate(osolver* s, int n_iter, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    for (int k = 0; k < n_iter; k++) iterate_once(s);
}

int64_t ora_iteration(const osolver* s) { return s->t; }

/* which: 0 = average strategy S / sum S, 1 = current strategy RM(R).
 * out: [A][nh]; invalid hands get 0. */
int ora_get_strategy(const osolver* s, int node, int which, double* out) {
    const ogame* g = s->g;
    if (node < 0 || node >= g->n || g->nd[node].type != T_DEC) return 1;
    const onode* o = &g->nd[node];
    int A = o->n_child, nh = g->nh;
    double cur[64];
    const double* src = (which == 0 ? s->S : s->R) + (size_t)o->rs * nh;
    for (int h = 0; h < nh; h++) {
        if (!g->hvalid[h]) { for (int a = 0; a < A; a++) out[(size_t)a * nh + h] = 0; continue; }
        if (which == 1) {
            for (int a = 0; a < A; a++)
                cur[a] = src[(size_t)a * nh + h] + (s->variant == V_PCFRPLUS ? s->pred[((size_t)o->rs + a) * nh + h] : 0.0);
            double sg[64];
            regret_match(cur, sg, A, 1, 0, threshold_at(s, s->t + 1));
            for (int a = 0; a < A; a++) out[(size_t)a * nh + h] = sg[a];
            continue;
        }
        double den = 0;
        for (int a = 0; a < A; a++) den += src[(size_t)a * nh + h];
        for (int a = 0; a < A; a++) out[(size_t)a * nh + h] = den > 0 ? src[(size_t)a * nh + h] / den : 1.0 / A;
    }
    return 0;
}

/* which: 0 = cumulative regrets R, 1 = average-strategy sums S, 2 = the
 * last instantaneous regrets (PCFR+'s prediction; zero for other rules),
 * 3 = the last half-step's action values, 4 = its instantaneous regrets. */
void ora_get_rows(const osolver* s, int which, double* out) {
    size_t n = (size_t)s->g->nrows * s->g->nh;
    const double* src = which == 0 ? s->R : which == 1 ? s->S : which == 2 ? s->pred : which == 3 ? s->cva : s->rinst;
    memcpy(out, src, n * sizeof(double));
}

void ora_set_rows(osolver* s, const double* R, const double* S, int64_t t) {
    size_t n = (size_t)s->g->nrows * s->g->nh;
    memcpy(s->R, R, n * sizeof(double));
    memcpy(s->S, S, n * sizeof(double));
    s->t = t;
}

/* Root counterfactual values of the last iteration (under sigma^t). */
void ora_root_cfv_current(const osolver* s, double* out) {
    for (int p = 0; p < 2; p++) memcpy(out + p * s->g->nh, s->cfv[p], sizeof(double) * s->g->nh);
}

/* Value recursion for one traverser hand against a weighted opponent range.
 * w[k] is the reach of opponent hand olist[k] (opponent strategy and
 * chance).  mode 0: best response (max over own actions); mode 1: follow the
 * traverser's average strategy.  The opponent always plays the average. */
static double value_rec(osolver* s, const double* sbar, int n, int i, int hi, const int* olist, int no,
                        const double* w, double* stack, int mode) {
    ogame* g = s->g;
    const onode* o = &g->nd[n];
    int nh = g->nh;
    switch (o->type) {
    case T_FOLD: {
        double cf = (double)o->c[o->player], sgn = o->player == i ? -1.0 : 1.0, m = 0;
        for (int k = 0; k < no; k++) m += w[k];
        return sgn * cf * m;
    }
    case T_SHOW: {
        int32_t a = g->rank[(size_t)o->bid * nh + hi];
        double v = 0;
        for (int k = 0; k < no; k++) {
            int32_t b = g->rank[(size_t)o->bid * nh + olist[k]];
            v += w[k] * ((a > b) - (a < b));
        }
        return (double)o->c[0] * v;
    }
    case T_LEAF: case T_ALLIN: {
        double v = 0;
        for (int k = 0; k < no; k++) if (w[k] != 0) v += w[k] * leaf_value(s, n, i, hi, olist[k]);
        return v;
    }
    case T_CHANCE: {
        double* w2 = stack;
        double v = 0;
        for (int c = 0; c < o->n_child; c++) {
            int ch = o->first_child + c;
            int card = g->nd[ch].chance_card;
            if (g->hmask[hi] >> card & 1) continue;
            for (int k = 0; k < no; k++) {
                uint64_t used = o->bmask | g->hmask[hi] | g->hmask[olist[k]];
                int K = 52 - __builtin_popcountll(used);
                w2[k] = (g->hmask[olist[k]] >> card & 1) ? 0.0 : w[k] / K;
            }
            v += value_rec(s, sbar, ch, i, hi, olist, no, w2, stack + no, mode);
        }
        return v;
    }
    default: break;
    }
    int A = o->n_child;
    const double* sb = sbar + (size_t)o->rs * nh;
    if (o->player == i) {
        double best = -INFINITY, avg = 0;
        for (int a = 0; a < A; a++) {
            double v = value_rec(s, sbar, o->first_child + a, i, hi, olist, no, w, stack, mode);
            if (v > best) best = v;
            avg += sb[(size_t)a * nh + hi] * v;
        }
        return mode == 0 ? best : avg;
    }
    double* w2 = stack;
    double v = 0;
    for (int a = 0; a < A; a++) {
        for (int k = 0; k < no; k++) w2[k] = w[k] * sb[(size_t)a * nh + olist[k]];
        v += value_rec(s, sbar, o->first_child + a, i, hi, olist, no, w2, stack + no, mode);
    }
    return v;
}

static double* avg_strategy_all(const osolver* s) {
    size_t n = (size_t)s->g->nrows * s->g->nh;
    double* sb = malloc(n * sizeof(double));
    strategy_rows(s->g, s->S, sb, 1, 0.0);
    return sb;
}

/* Per-hand values at the root under the average strategy (mode 1) or of the
 * best response to the opponent's average strategy (mode 0).  out: [2][nh]. */
static void root_values(osolver* s, int mode, double* out) {
    ogame* g = s->g;
    int nh = g->nh;
    double* sbar = avg_strategy_all(s);
    for (int i = 0; i < 2; i++) {
        int op = 1 - i;
        #pragma omp parallel for schedule(dynamic)
        for (int hi = 0; hi < nh; hi++) {
            out[i * nh + hi] = 0;
            if (!g->hvalid[hi]) continue;
            if (s->support_only && !(s->rng[i][hi] > 0)) continue;
            int* ol = malloc(sizeof(int) * nh);
            double* w = malloc(sizeof(double) * nh);
            int no = 0;
            for (int h = 0; h < nh; h++)
                if (g->hvalid[h] && s->rng[op][h] > 0 && compat(g, hi, h)) { ol[no] = h; w[no] = s->rng[op][h]; no++; }
            double* stack = malloc(sizeof(double) * (size_t)(no + 1) * MAXDEPTH);
            out[i * nh + hi] = value_rec(s, sbar, 0, i, hi, ol, no, w, stack, mode);
            free(stack); free(ol); free(w);
        }
    }
    free(sbar);
}

void ora_root_cfv_avg(osolver* s, double* out) { root_values(s, 1, out); }

/* Joint mass of compatible hand pairs, Z = sum r0(h) r1(o). */
double ora_pair_mass(const osolver* s) {
    const ogame* g = s->g;
    double z = 0;
    for (int h = 0; h < g->nh; h++) {
        if (!g->hvalid[h] || s->rng[0][h] == 0) continue;
        for (int o = 0; o < g->nh; o++)
            if (g->hvalid[o] && compat(g, h, o)) z += s->rng[0][h] * s->rng[1][o];
    }
    return z;
}

/* Exploitability of the average strategy: (BR_0 + BR_1) / 2 in chips per
 * hand, where BR_i is player i's best-response value per unit of joint pair
 * mass.  br_out receives BR_0, BR_1. */
double ora_exploitability(osolver* s, double* br_out) {
    ogame* g = s->g;
    int nh = g->nh;
    double* v = malloc(sizeof(double) * 2 * nh);
    root_values(s, 0, v);
    double z = ora_pair_mass(s);
    double br[2] = {0, 0};
    for (int i = 0; i < 2; i++)
        for (int h = 0; h < nh; h++) br[i] += s->rng[i][h] * v[i * nh + h];
    free(v);
    br[0] /= z; br[1] /= z;
    if (br_out) { br_out[0] = br[0]; br_out[1] = br[1]; }
    return 0.5 * (br[0] + br[1]);
}

/* Leaf values given as a table of expected values per unit of pot:
 * ev[leaf][player][card][nh], leaves in node order. */
void ora_set_leaf_table(osolver* s, const double* ev) {
    size_t n = (size_t)s->nleaf * 2 * 52 * s->g->nh;
    if (!s->leaf_ev) s->leaf_ev = malloc(n * sizeof(double));
    memcpy(s->leaf_ev, ev, n * sizeof(double));
    s->leaf_kind = LEAF_TABLE;
}

int ora_num_leaves(const osolver* s) { return s->nleaf; }

/* ------------------------------------------------------------- flops at preflop leaves
 * Suit permutations act on cards as 4 r + s -> 4 r + pi(s).  A flop (3 cards,
 * as a 52-bit mask) is canonical when no permutation maps it to a smaller
 * mask; the canonical flops, listed by their sorted cards in lexicographic
 * order, stand for their orbits
 * (the lossless suit abstraction of Sec. 4.5 applied to the flop deal). */
static int PERM[24][4];
static int PERM_INV[24];
static void perms_init(void) {
    static int done = 0;
    if (done) return;
    int q = 0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            for (int c = 0; c < 4; c++)
                for (int d = 0; d < 4; d++) {
                    if (a == b || a == c || a == d || b == c || b == d || c == d) continue;
                    PERM[q][0] = a; PERM[q][1] = b; PERM[q][2] = c; PERM[q][3] = d;
                    q++;
                }
    for (q = 0; q < 24; q++)
        for (int r = 0; r < 24; r++) {
            int id = 1;
            for (int u = 0; u < 4; u++) id &= PERM[r][PERM[q][u]] == u;
            if (id) PERM_INV[q] = r;
        }
    done = 1;
}
static int perm_card(int q, int c) { return 4 * (c / 4) + PERM[q][c % 4]; }
static uint64_t perm_mask(int q, uint64_t m) {
    uint64_t out = 0;
    for (int c = 0; c < 52; c++) if (m >> c & 1) out |= 1ULL << perm_card(q, c);
    return out;
}
static uint64_t canon_mask(uint64_t m) {
    uint64_t best = m;
    for (int q = 0; q < 24; q++) { uint64_t x = perm_mask(q, m); if (x < best) best = x; }
    return best;
}

/* Canonical flops: writes up to cap entries of cards[3] (ascending) and the
 * orbit size of each; returns how many there are. */
int ora_canonical_flops(int32_t* cards, int32_t* orbit, int cap) {
    perms_init();
    static uint64_t canon[22100], mask[22100];
    int k = 0;
    for (int x = 0; x < 52; x++)
        for (int y = x + 1; y < 52; y++)
            for (int z = y + 1; z < 52; z++, k++) {
                mask[k] = (1ULL << x) | (1ULL << y) | (1ULL << z);
                canon[k] = canon_mask(mask[k]);
            }
    int n = 0;
    for (int i = 0; i < 22100; i++) {
        if (canon[i] != mask[i]) continue;
        if (n < cap) {
            int j = 0;
            for (int c = 0; c < 52; c++) if (mask[i] >> c & 1) cards[3 * n + j++] = c;
            int m = 0;
            for (int u = 0; u < 22100; u++) m += canon[u] == mask[i];
            orbit[n] = m;
        }
        n++;
    }
    return n;
}

/* Leaf values of a preflop tree from a table of expected values per unit of
 * pot on the canonical flops: ev[leaf][player][flop][nh], flops as
 * ora_canonical_flops lists them.  A flop g stands in the orbit of its
 * canonical flop f; the expected value of hand h on g is the table's value
 * on f of the hand mapped back, averaged over every permutation pi with
 * pi(f) = g: E(h | g) = mean_pi ev[f][pi^-1(h)].  Returns 0, or 1 if the
 * tree has no preflop leaf. */
int ora_set_flop_leaf_table(osolver* s, const double* ev) {
    ogame* g = s->g;
    int any = 0;
    for (int i = 0; i < g->n; i++) any |= g->nd[i].type == T_LEAF && g->nd[i].nb == 0;
    if (!any || g->nh != NCOMBO) return 1;
    perms_init();
    enum { NF = 1755 };
    static int32_t fc[NF * 3], fo[NF];
    if (ora_canonical_flops(fc, fo, NF) != NF) abort();
    /* every flop: its canonical flop and the permutations that map it there */
    int nfl = 22100;
    int32_t* fidx = malloc(sizeof(int32_t) * nfl);
    int32_t* fq = malloc(sizeof(int32_t) * nfl * 24);
    int32_t* fnq = malloc(sizeof(int32_t) * nfl);
    uint64_t* fm = malloc(sizeof(uint64_t) * nfl);
    int k = 0;
    for (int x = 0; x < 52; x++)
        for (int y = x + 1; y < 52; y++)
            for (int z = y + 1; z < 52; z++, k++) {
                uint64_t m = (1ULL << x) | (1ULL << y) | (1ULL << z);
                uint64_t cm = canon_mask(m);
                int f = -1;
                for (int j = 0; j < NF; j++)
                    if (((1ULL << fc[3 * j]) | (1ULL << fc[3 * j + 1]) | (1ULL << fc[3 * j + 2])) == cm) { f = j; break; }
                fidx[k] = f; fm[k] = m; fnq[k] = 0;
                for (int q = 0; q < 24; q++) if (perm_mask(q, cm) == m) fq[k * 24 + fnq[k]++] = q;
            }
    size_t nh = NCOMBO, L = (size_t)s->nleaf * 2;
    int hc[2 * NCOMBO];
    for (size_t h = 0; h < nh; h++) {
        int j = 0;
        for (int c = 0; c < 52; c++) if (g->hmask[h] >> c & 1) hc[2 * h + j++] = c;
    }
    free(s->flopA); free(s->flopB); free(s->flopD);
    s->flopA = calloc(L * nh, sizeof(double));
    s->flopB = calloc(L * nh * 52, sizeof(double));
    s->flopD = calloc(L * nh * nh, sizeof(double));
    #pragma omp parallel for schedule(dynamic)
    for (long li = 0; li < (long)L; li++) {
        const double* tab = ev + (size_t)li * NF * nh;
        double* A = s->flopA + li * nh;
        double* B = s->flopB + li * nh * 52;
        double* D = s->flopD + li * nh * nh;
        for (int q = 0; q < nfl; q++) {
            int c3[3], n3 = 0;
            for (int c = 0; c < 52; c++) if (fm[q] >> c & 1) c3[n3++] = c;
            const double* row = tab + (size_t)fidx[q] * nh;
            for (size_t h = 0; h < nh; h++) {
                if (g->hmask[h] & fm[q]) continue;
                double e = 0;
                for (int j = 0; j < fnq[q]; j++) {
                    int qi = PERM_INV[fq[q * 24 + j]];
                    e += row[combo_index(perm_card(qi, hc[2 * h]), perm_card(qi, hc[2 * h + 1]))];
                }
                e /= fnq[q];
                A[h] += e;
                for (int u = 0; u < 3; u++) B[h * 52 + c3[u]] += e;
                D[h * nh + combo_index(c3[1], c3[0])] += e;
                D[h * nh + combo_index(c3[2], c3[0])] += e;
                D[h * nh + combo_index(c3[2], c3[1])] += e;
            }
        }
    }
    free(fidx); free(fq); free(fnq); free(fm);
    s->leaf_kind = LEAF_FLOP;
    return 0;
}

/* Counterfactual value of every hand of player i at leaf node n against the
 * opponent reach ro[nh]: out[h] = sum over compatible ho of ro[ho] times the
 * history's leaf value.  Returns 1 if n is not a leaf. */
int ora_leaf_cfv(osolver* s, int n, int i, const double* ro, double* out) {
    ogame* g = s->g;
    if (n < 0 || n >= g->n || (g->nd[n].type != T_LEAF && g->nd[n].type != T_ALLIN)) return 1;
    for (int h = 0; h < g->nh; h++) {
        double v = 0;
        if (g->hvalid[h])
            for (int o = 0; o < g->nh; o++)
                if (g->hvalid[o] && compat(g, h, o) && ro[o] != 0) v += ro[o] * leaf_value(s, n, i, h, o);
        out[h] = v;
    }
    return 0;
}

/* 1 when the tree has leaves at the flop deal (a preflop root). */
int ora_has_flop_leaves(const ogame* g) {
    for (int i = 0; i < g->n; i++) if (g->nd[i].type == T_LEAF && g->nd[i].nb == 0) return 1;
    return 0;
}

/* Own reach of both players at every node under the current strategy
 * RM(R) (what the next iteration will use).  out: [n][2][nh]. */
static void reach_rec(const ogame* g, const double* sig, int n, const double* r0, const double* r1, double* out) {
    const onode* o = &g->nd[n];
    int nh = g->nh;
    double* me = out + (size_t)n * 2 * nh;
    memcpy(me, r0, sizeof(double) * nh);
    memcpy(me + nh, r1, sizeof(double) * nh);
    if (o->type != T_DEC && o->type != T_CHANCE) return;
    double* tmp = malloc(sizeof(double) * 2 * nh);
    for (int k = 0; k < o->n_child; k++) {
        int ch = o->first_child + k;
        memcpy(tmp, r0, sizeof(double) * nh);
        memcpy(tmp + nh, r1, sizeof(double) * nh);
        if (o->type == T_CHANCE) {
            int card = g->nd[ch].chance_card;
            for (int h = 0; h < nh; h++) if (g->hmask[h] >> card & 1) { tmp[h] = 0; tmp[nh + h] = 0; }
        } else {
            const double* sg = sig + ((size_t)o->rs + k) * nh;
            double* mine = tmp + (size_t)o->player * nh;
            for (int h = 0; h < nh; h++) mine[h] *= sg[h];
        }
        reach_rec(g, sig, ch, tmp, tmp + nh, out);
    }
    free(tmp);
}

void ora_reach_current(const osolver* s, double* out) {
    size_t n = (size_t)s->g->nrows * s->g->nh;
    double* sig = malloc(n * sizeof(double));
    double* tmp = malloc(n * sizeof(double));
    strategy_rows(s->g, matched_regrets(s, tmp), sig, 0, threshold_at(s, s->t + 1));
    reach_rec(s->g, sig, 0, s->rng[0], s->rng[1], out);
    free(tmp);
    free(sig);
}

/* Pairwise equity table of a showdown/leaf board (for the all-in leaf). */
int ora_equity_table(ogame* g, int node, double* out) {
    if (node < 0 || node >= g->n || g->nd[node].bid < 0) return 1;
    double* E = game_eq(g, g->nd[node].bid);
    memcpy(out, E, sizeof(double) * g->nh * g->nh);
    return 0;
}

int ora_node_board(const ogame* g, int node, int32_t* board) {
    const onode* o = &g->nd[node];
    for (int k = 0; k < o->nb; k++) board[k] = o->board[k];
    return o->nb;
}
