/* oracle.c -- plain, slow, single-threaded FP64 reference for CFR.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * library.
 *
 * What it computes (paper, Section 3 "Background", eqs. reach, cfv, regret,
 * rm, exploitability; Section 4.1 for the compiled arrays):
 *
 *  - or_layout: the canonical compiled arrays of a game (breadth-first node
 *    numbering, depth offsets, parent/child CSR, information sets numbered by
 *    first occurrence, slot offsets, member lists, and the chance-folded
 *    values template v_tmpl(z) = pi_c(z) u(z) of eq. (template)), written out
 *    directly from their definitions.
 *  - or_iterate: T iterations of CFR / CFR+ by textbook per-history
 *    recursion over an explicit tree with chance probabilities applied on the
 *    chance edges (NOT the folded, edge/slot formulation), with an
 *    information-set table keyed by the game's keys:
 *        sigma^t   = regret matching of R^{t-1} (uniform if no positive regret)
 *        v(h)      = expected payoff to player 1 below h under sigma^t
 *        r(I,a)    = sum_{h in I} s_i pi_{-i}(h) pi_c(h) (v(h.a) - v(h))
 *        R^t       = R^{t-1} + r      (CFR+: then R^t <- max(R^t, 0))
 *        sbar(I,a) += w_t pi_i(I) sigma^t(I,a),  w_t = t (linear) or 1
 *    Simultaneous updates: both players' regrets come from one profile.
 *    (A control option sums each node's children in reverse order: another rounding pattern.)
 *    Alternating updates: player 1's half-iteration (regret and average of
 *    player 1 only) runs first; player 2's half then sees player 1's updated
 *    strategy.
 *  - or_exploitability: NashConv/2 of the normalised average profile, eq.
 *    (exploitability), by an exact recursive best response with
 *    information-set argmax (ties to the lowest action index).
 *
 * Everything is in double precision by default.  Built with
 * -DORACLE_STATE_FLOAT, the state the paper keeps in its configured compute
 * dtype (reach, values, regrets, strategy) is float while strategy sums stay
 * double (paper, Table 'tab:memplan' and Proposition 4): a control build that
 * measures how far any FP32-state run drifts from the FP64 iterates.  The
 * public entry points take the game as plain arrays (node type, children,
 * chance probabilities, keys, payoffs).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <math.h>

enum { CH = 0, PL1 = 1, PL2 = 2, TERM = 3 };

#ifdef ORACLE_STATE_FLOAT
typedef float st_t;
#else
typedef double st_t;
#endif

typedef struct {
    int64_t key;
    int player, nA, depth;
    int64_t slot;                 /* first slot */
    int64_t first_member;         /* canonical id of the first member */
} oinfo;

typedef struct {
    /* game, in the caller's node ids */
    int64_t n, e, root;
    int8_t *type;
    int64_t *kb;                  /* child begin */
    int32_t *nk;
    int64_t *kids;
    double *prob;
    int64_t *key;
    double *payoff;
    /* canonical numbering */
    int64_t *canon;               /* caller id -> canonical id */
    int64_t *order;               /* canonical id -> caller id */
    int32_t *depth;               /* by caller id */
    int64_t *iset;                /* by caller id: infoset index, -1 if none */
    int max_depth;
    /* information sets */
    int64_t ni, na;
    oinfo *info;
    int64_t *mem_off, *mem;       /* members (canonical ids), ascending */
    /* hash table key -> infoset index */
    int64_t hcap;
    int64_t *hkey, *hval;
    /* solver state (per slot) */
    st_t *R, *sigma, *rinst, *pred;
    double *sbar;
    int64_t *avg_stamp;           /* per infoset: last (iteration, player) stamp the average was added */
    int rule, linear, alternating; /* rule: RULE_CFR, RULE_CFR_PLUS, RULE_DCFR, RULE_PCFR_PLUS */
    int reverse;                  /* control option: sum each node's children in reverse order */
    int64_t t;                    /* iterations done */
    /* scratch for BR */
    double *memo, *q;
    int *astar;
} oracle;

/* Update rules (paper Sec. 6 "Update rule and update order"; constants the paper leaves out are
 * those of the published methods):
 *   CFR    R += r;                                     average weight w_t (t or 1)
 *   CFR+   R = max(R + r, 0);                          average weight w_t
 *   DCFR   R = R + r, then times t^a/(t^a+1) where positive and t^b/(t^b+1) where not
 *          (a = 3/2, b = 0); S = (S + pi sigma) (t/(t+1))^g (g = 2)   (Brown and Sandholm 2019)
 *   PCFR+  R = max(R + r, 0); sigma^{t+1} = regret matching of R + m with the prediction
 *          m = r (the latest instantaneous regret); average weight t^2  (Farina et al. 2021) */
enum { RULE_CFR = 0, RULE_CFR_PLUS = 1, RULE_DCFR = 2, RULE_PCFR_PLUS = 3 };
#define DCFR_ALPHA 1.5
#define DCFR_BETA 0.0
#define DCFR_GAMMA 2.0

static uint64_t mix64(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdull; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ull; x ^= x >> 33;
    return x;
}

static int64_t hfind(oracle *o, int64_t key, int insert, int64_t val) {
    uint64_t h = mix64((uint64_t)key) & (uint64_t)(o->hcap - 1);
    for (;;) {
        if (o->hval[h] < 0) {
            if (!insert) return -1;
            o->hkey[h] = key; o->hval[h] = val;
            return val;
        }
        if (o->hkey[h] == key) return o->hval[h];
        h = (h + 1) & (uint64_t)(o->hcap - 1);
    }
}

static void seterr(char *err, int len, const char *m) { if (err && len > 0) snprintf(err, (size_t)len, "%s", m); }

void or_destroy(oracle *o) {
    if (!o) return;
    free(o->type); free(o->kb); free(o->nk); free(o->kids); free(o->prob); free(o->key); free(o->payoff);
    free(o->canon); free(o->order); free(o->depth); free(o->iset); free(o->info); free(o->mem_off); free(o->mem);
    free(o->hkey); free(o->hval); free(o->R); free(o->sbar); free(o->sigma); free(o->rinst); free(o->pred); free(o->avg_stamp);
    free(o->memo); free(o->q); free(o->astar);
    free(o);
}

oracle *or_create(int64_t n, int64_t root, const int8_t *type, const int64_t *child_begin, const int32_t *n_children,
                  const int64_t *children, const double *prob, const int64_t *key, const double *payoff,
                  char *err, int errlen) {
    if (n <= 0 || root < 0 || root >= n) { seterr(err, errlen, "bad node count or root"); return NULL; }
    oracle *o = (oracle *)calloc(1, sizeof(oracle));
    o->n = n; o->root = root;
    o->type = (int8_t *)malloc((size_t)n);
    o->kb = (int64_t *)malloc((size_t)n * 8);
    o->nk = (int32_t *)malloc((size_t)n * 4);
    o->key = (int64_t *)malloc((size_t)n * 8);
    o->payoff = (double *)malloc((size_t)n * 8);
    memcpy(o->type, type, (size_t)n);
    memcpy(o->nk, n_children, (size_t)n * 4);
    memcpy(o->key, key, (size_t)n * 8);
    memcpy(o->payoff, payoff, (size_t)n * 8);
    int64_t e = 0;
    for (int64_t i = 0; i < n; i++) {
        if (n_children[i] < 0) { seterr(err, errlen, "negative child count"); or_destroy(o); return NULL; }
        e += n_children[i];
    }
    o->e = e;
    o->kids = (int64_t *)malloc((size_t)(e ? e : 1) * 8);
    o->prob = (double *)malloc((size_t)(e ? e : 1) * 8);
    /* copy children compactly (own edge numbering) */
    int64_t w = 0;
    for (int64_t i = 0; i < n; i++) {
        o->kb[i] = w;
        for (int32_t a = 0; a < n_children[i]; a++) {
            int64_t c = children[child_begin[i] + a];
            if (c < 0 || c >= n) { seterr(err, errlen, "child id out of range"); or_destroy(o); return NULL; }
            o->kids[w] = c;
            o->prob[w] = prob[child_begin[i] + a];
            w++;
        }
    }
    /* validate: types, tree shape (one parent each, all reachable), chance sums */
    int32_t *npar = (int32_t *)calloc((size_t)n, 4);
    for (int64_t i = 0; i < n; i++) {
        int ty = o->type[i];
        if (ty < 0 || ty > 3) { free(npar); seterr(err, errlen, "bad node type"); or_destroy(o); return NULL; }
        if (ty == TERM && o->nk[i] != 0) { free(npar); seterr(err, errlen, "terminal with children"); or_destroy(o); return NULL; }
        if (ty != TERM && o->nk[i] == 0) { free(npar); seterr(err, errlen, "non-terminal without children"); or_destroy(o); return NULL; }
        if ((ty == PL1 || ty == PL2) && o->nk[i] > 64) { free(npar); seterr(err, errlen, "more than 64 actions"); or_destroy(o); return NULL; }
        if (ty == CH) {
            double s = 0.0;
            for (int32_t a = 0; a < o->nk[i]; a++) {
                double p = o->prob[o->kb[i] + a];
                if (!(p >= 0.0)) { free(npar); seterr(err, errlen, "negative chance probability"); or_destroy(o); return NULL; }
                s += p;
            }
            if (fabs(s - 1.0) > 1e-9) { free(npar); seterr(err, errlen, "chance probabilities do not sum to 1"); or_destroy(o); return NULL; }
        }
        for (int32_t a = 0; a < o->nk[i]; a++) npar[o->kids[o->kb[i] + a]]++;
    }
    for (int64_t i = 0; i < n; i++) {
        int want = i == root ? 0 : 1;
        if (npar[i] != want) { free(npar); seterr(err, errlen, "not a tree"); or_destroy(o); return NULL; }
    }
    free(npar);
    /* breadth-first canonical numbering (children enqueued in action order) */
    o->canon = (int64_t *)malloc((size_t)n * 8);
    o->order = (int64_t *)malloc((size_t)n * 8);
    o->depth = (int32_t *)malloc((size_t)n * 4);
    for (int64_t i = 0; i < n; i++) o->canon[i] = -1;
    int64_t head = 0, tail = 0;
    o->order[tail++] = root; o->canon[root] = 0; o->depth[root] = 0;
    o->max_depth = 0;
    while (head < tail) {
        int64_t h = o->order[head++];
        for (int32_t a = 0; a < o->nk[h]; a++) {
            int64_t c = o->kids[o->kb[h] + a];
            if (o->canon[c] >= 0) { seterr(err, errlen, "node reached twice"); or_destroy(o); return NULL; }
            o->canon[c] = tail; o->order[tail++] = c;
            o->depth[c] = o->depth[h] + 1;
            if (o->depth[c] > o->max_depth) o->max_depth = o->depth[c];
        }
    }
    if (tail != n) { seterr(err, errlen, "unreachable nodes"); or_destroy(o); return NULL; }
    /* information sets, numbered by first occurrence in canonical order */
    o->hcap = 16;
    while (o->hcap < 2 * n + 16) o->hcap *= 2;
    o->hkey = (int64_t *)malloc((size_t)o->hcap * 8);
    o->hval = (int64_t *)malloc((size_t)o->hcap * 8);
    for (int64_t i = 0; i < o->hcap; i++) o->hval[i] = -1;
    o->iset = (int64_t *)malloc((size_t)n * 8);
    int64_t cap = 1024;
    o->info = (oinfo *)malloc((size_t)cap * sizeof(oinfo));
    o->ni = 0; o->na = 0;
    int64_t *count = NULL;
    for (int64_t k = 0; k < n; k++) {
        int64_t h = o->order[k];
        o->iset[h] = -1;
        int ty = o->type[h];
        if (ty != PL1 && ty != PL2) continue;
        int64_t idx = hfind(o, o->key[h], 1, o->ni);
        if (idx == o->ni) {
            if (o->ni == cap) { cap *= 2; o->info = (oinfo *)realloc(o->info, (size_t)cap * sizeof(oinfo)); }
            oinfo *I = &o->info[o->ni++];
            I->key = o->key[h]; I->player = ty; I->nA = o->nk[h]; I->depth = o->depth[h];
            I->slot = o->na; I->first_member = k;
            o->na += o->nk[h];
        } else {
            oinfo *I = &o->info[idx];
            if (I->player != ty) { seterr(err, errlen, "information set spans players"); or_destroy(o); return NULL; }
            if (I->nA != o->nk[h]) { seterr(err, errlen, "information set action counts differ"); or_destroy(o); return NULL; }
        }
        o->iset[h] = idx;
    }
    /* members, ascending canonical id */
    o->mem_off = (int64_t *)calloc((size_t)o->ni + 1, 8);
    count = (int64_t *)calloc((size_t)o->ni + 1, 8);
    int64_t ndec = 0;
    for (int64_t h = 0; h < n; h++) if (o->iset[h] >= 0) { o->mem_off[o->iset[h] + 1]++; ndec++; }
    for (int64_t i = 0; i < o->ni; i++) o->mem_off[i + 1] += o->mem_off[i];
    o->mem = (int64_t *)malloc((size_t)(ndec ? ndec : 1) * 8);
    for (int64_t k = 0; k < n; k++) {
        int64_t h = o->order[k];
        int64_t I = o->iset[h];
        if (I < 0) continue;
        o->mem[o->mem_off[I] + count[I]++] = k;
    }
    free(count);
    int64_t A = o->na ? o->na : 1;
    o->R = (st_t *)calloc((size_t)A, sizeof(st_t));
    o->sbar = (double *)calloc((size_t)A, 8);
    o->sigma = (st_t *)calloc((size_t)A, sizeof(st_t));
    o->rinst = (st_t *)calloc((size_t)A, sizeof(st_t));
    o->pred = (st_t *)calloc((size_t)A, sizeof(st_t));
    o->avg_stamp = (int64_t *)malloc((size_t)(o->ni ? o->ni : 1) * 8);
    for (int64_t i = 0; i < o->ni; i++) o->avg_stamp[i] = -1;
    o->memo = (double *)malloc((size_t)n * 8);
    o->q = (double *)malloc((size_t)n * 8);
    o->astar = (int *)malloc((size_t)(o->ni ? o->ni : 1) * sizeof(int));
    o->rule = RULE_CFR_PLUS; o->linear = 1; o->alternating = 0; o->t = 0;
    return o;
}

/* counts: N, E, terminals, decision nodes, infosets, slots, max depth, blocks */
void or_counts(const oracle *o, int64_t *out) {
    int64_t z = 0, d = 0;
    for (int64_t i = 0; i < o->n; i++) { if (o->type[i] == TERM) z++; else if (o->type[i] != CH) d++; }
    out[0] = o->n; out[1] = o->e; out[2] = z; out[3] = d; out[4] = o->ni; out[5] = o->na;
    out[6] = o->max_depth;
    out[7] = o->n > 1 ? o->max_depth : 0;   /* edges grouped by parent depth 0..max_depth-1 */
}

/* Canonical arrays.  Sizes: depth_off[max_depth+2], parent/child_off(N+1)/in_slot/node_infoset/type/tmpl
 * per node, slot_off/mem_off[I+1], mem_node[Ndec], iset_player[I], iset_key[I]. */
void or_layout(const oracle *o, int32_t *depth_off, int32_t *parent, int32_t *child_off, int32_t *in_slot,
               int32_t *node_infoset, int8_t *ntype, float *tmpl, int32_t *slot_off, int32_t *mem_off,
               int32_t *mem_node, int8_t *iset_player, int64_t *iset_key) {
    int64_t n = o->n;
    for (int d = 0; d <= o->max_depth + 1; d++) depth_off[d] = 0;
    for (int64_t k = 0; k < n; k++) depth_off[o->depth[o->order[k]] + 1]++;
    for (int d = 0; d <= o->max_depth; d++) depth_off[d + 1] += depth_off[d];
    double *pic = (double *)malloc((size_t)n * 8);
    parent[0] = -1; in_slot[0] = -1; pic[0] = 1.0;
    int32_t next = 1;
    for (int64_t k = 0; k < n; k++) {
        int64_t h = o->order[k];
        child_off[k] = next;
        ntype[k] = o->type[h];
        node_infoset[k] = (int32_t)o->iset[h];
        for (int32_t a = 0; a < o->nk[h]; a++) {
            int64_t c = o->kids[o->kb[h] + a];
            int64_t ck = o->canon[c];
            parent[ck] = (int32_t)k;
            if (o->type[h] == CH) { in_slot[ck] = -1; pic[ck] = pic[k] * o->prob[o->kb[h] + a]; }
            else { in_slot[ck] = (int32_t)(o->info[o->iset[h]].slot + a); pic[ck] = pic[k]; }
            next++;
        }
        tmpl[k] = o->type[h] == TERM ? (float)(pic[k] * o->payoff[h]) : 0.0f;
    }
    child_off[n] = next;
    free(pic);
    for (int64_t i = 0; i <= o->ni; i++) { mem_off[i] = (int32_t)o->mem_off[i]; }
    for (int64_t i = 0; i < o->ni; i++) {
        slot_off[i] = (int32_t)o->info[i].slot;
        iset_player[i] = (int8_t)o->info[i].player;
        iset_key[i] = o->info[i].key;
    }
    slot_off[o->ni] = (int32_t)o->na;
    for (int64_t k = 0; k < o->mem_off[o->ni]; k++) mem_node[k] = (int32_t)o->mem[k];
}

void or_set_options(oracle *o, int plus, int linear, int alternating) {
    o->rule = plus ? RULE_CFR_PLUS : RULE_CFR; o->linear = linear; o->alternating = alternating;
}

/* rule: RULE_CFR .. RULE_PCFR_PLUS (linear applies to CFR and CFR+ only) */
void or_set_rule(oracle *o, int rule) { o->rule = rule; }

/* Control option: values summed over each node's children in reverse order -- another correct
 * summation order, whose rounding differs from the default's (used to sample how far runs of one
 * precision spread; the iterates agree with the default order up to rounding). */
void or_set_reverse(oracle *o, int reverse) { o->reverse = reverse; }

void or_reset(oracle *o) {
    int64_t A = o->na;
    memset(o->R, 0, (size_t)(A ? A : 1) * sizeof(st_t));
    memset(o->sbar, 0, (size_t)(A ? A : 1) * 8);
    memset(o->pred, 0, (size_t)(A ? A : 1) * sizeof(st_t));
    for (int64_t i = 0; i < o->ni; i++) o->avg_stamp[i] = -1;
    o->t = 0;
}

/* regret matching for one infoset: proportional to positive regret, uniform if none (eq. rm) */
static void regret_match(const st_t *R, st_t *sig, int nA) {
    st_t tot = 0;
    for (int a = 0; a < nA; a++) tot += R[a] > 0 ? R[a] : 0;
    for (int a = 0; a < nA; a++) sig[a] = tot > 0 ? (R[a] > 0 ? R[a] : (st_t)0) / tot : (st_t)1 / (st_t)nA;
}

/* the strategy the next traversal plays: regret matching of R, or of R + prediction (PCFR+) */
static void current_strategy(const oracle *o, const oinfo *I, st_t *sig) {
    if (o->rule != RULE_PCFR_PLUS) { regret_match(o->R + I->slot, sig, I->nA); return; }
    st_t tmp[64];
    for (int32_t a = 0; a < I->nA; a++) tmp[a] = o->R[I->slot + a] + o->pred[I->slot + a];
    regret_match(tmp, sig, I->nA);
}

static void regret_match_player(oracle *o, int player) {
    for (int64_t i = 0; i < o->ni; i++) {
        oinfo *I = &o->info[i];
        if (player && I->player != player) continue;
        current_strategy(o, I, o->sigma + I->slot);
    }
}

/* One traversal: returns the expected payoff to player 1 below h (chance on edges).
 * pi1, pi2: players' own reach; pic: chance reach.  Regrets of `upd` players
 * (bit 1 = P1, bit 2 = P2) are accumulated into rinst and their average into
 * sbar with weight w (once per infoset and stamp). */
static st_t walk(oracle *o, int64_t h, st_t pi1, st_t pi2, st_t pic, int upd, double w, int64_t stamp) {
    int ty = o->type[h];
    if (ty == TERM) return (st_t)o->payoff[h];
    if (ty == CH) {
        st_t v = 0;
        for (int32_t k = 0; k < o->nk[h]; k++) {
            const int32_t a = o->reverse ? o->nk[h] - 1 - k : k;
            st_t p = (st_t)o->prob[o->kb[h] + a];
            v += p * walk(o, o->kids[o->kb[h] + a], pi1, pi2, pic * p, upd, w, stamp);
        }
        return v;
    }
    int64_t Ii = o->iset[h];
    oinfo *I = &o->info[Ii];
    const st_t *sig = o->sigma + I->slot;
    st_t va[64];
    st_t v = 0;
    for (int32_t k = 0; k < I->nA; k++) {
        const int32_t a = o->reverse ? I->nA - 1 - k : k;
        st_t c1 = ty == PL1 ? pi1 * sig[a] : pi1;
        st_t c2 = ty == PL2 ? pi2 * sig[a] : pi2;
        va[a] = walk(o, o->kids[o->kb[h] + a], c1, c2, pic, upd, w, stamp);
        v += sig[a] * va[a];
    }
    if (upd & ty) {
        st_t s = ty == PL1 ? 1 : -1;
        st_t cf = (ty == PL1 ? pi2 : pi1) * pic;
        for (int32_t a = 0; a < I->nA; a++) o->rinst[I->slot + a] += s * cf * (va[a] - v);
        if (o->avg_stamp[Ii] != stamp) {
            o->avg_stamp[Ii] = stamp;
            double own = ty == PL1 ? (double)pi1 : (double)pi2;
            for (int32_t a = 0; a < I->nA; a++) o->sbar[I->slot + a] += w * own * (double)sig[a];
        }
    }
    return v;
}

/* Regret update of iteration t for the sets of `player` (0: both); DCFR also discounts their
 * strategy sums, whose iteration-t contribution the traversal has just added. */
static void apply_regrets(oracle *o, int player, int64_t t) {
    const double ta = pow((double)t, DCFR_ALPHA), tb = pow((double)t, DCFR_BETA);
    const st_t pos = (st_t)(ta / (ta + 1.0)), neg = (st_t)(tb / (tb + 1.0));
    const double sdisc = pow((double)t / (double)(t + 1), DCFR_GAMMA);
    for (int64_t i = 0; i < o->ni; i++) {
        oinfo *I = &o->info[i];
        if (player && I->player != player) continue;
        for (int a = 0; a < I->nA; a++) {
            int64_t q = I->slot + a;
            o->R[q] += o->rinst[q];
            if (o->rule == RULE_CFR_PLUS || o->rule == RULE_PCFR_PLUS) {
                if (o->R[q] < 0) o->R[q] = 0;
            } else if (o->rule == RULE_DCFR) {
                o->R[q] *= o->R[q] > 0 ? pos : neg;
                o->sbar[q] *= sdisc;
            }
            if (o->rule == RULE_PCFR_PLUS) o->pred[q] = o->rinst[q];
            o->rinst[q] = 0;
        }
    }
}

/* T iterations; returns the root value of the last traversal (player-1 expected payoff under sigma^t) */
double or_iterate(oracle *o, int64_t T) {
    st_t v = 0;
    for (int64_t it = 0; it < T; it++) {
        int64_t t = o->t + 1;
        double w = o->rule == RULE_DCFR ? 1.0 : o->rule == RULE_PCFR_PLUS ? (double)t * (double)t
                 : o->linear ? (double)t : 1.0;
        if (!o->alternating) {
            regret_match_player(o, 0);
            v = walk(o, o->root, 1.0, 1.0, 1.0, 3, w, 2 * t);
            apply_regrets(o, 0, t);
        } else {
            regret_match_player(o, 0);
            v = walk(o, o->root, 1.0, 1.0, 1.0, 1, w, 2 * t);
            apply_regrets(o, 1, t);
            regret_match_player(o, 1);
            walk(o, o->root, 1.0, 1.0, 1.0, 2, w, 2 * t + 1);
            apply_regrets(o, 2, t);
        }
        o->t = t;
    }
    return (double)v;
}

int64_t or_iterations(const oracle *o) { return o->t; }

/* state in canonical slot order */
void or_get(const oracle *o, double *R, double *sbar, double *sigma_cur, double *sigma_avg) {
    for (int64_t i = 0; i < o->ni; i++) {
        const oinfo *I = &o->info[i];
        st_t tmp[64];
        if (R) for (int a = 0; a < I->nA; a++) R[I->slot + a] = (double)o->R[I->slot + a];
        if (sbar) for (int a = 0; a < I->nA; a++) sbar[I->slot + a] = o->sbar[I->slot + a];
        if (sigma_cur) {
            current_strategy(o, I, tmp);
            for (int a = 0; a < I->nA; a++) sigma_cur[I->slot + a] = (double)tmp[a];
        }
        if (sigma_avg) {
            double s = 0.0;
            for (int a = 0; a < I->nA; a++) s += o->sbar[I->slot + a];
            for (int a = 0; a < I->nA; a++) sigma_avg[I->slot + a] = s > 0.0 ? o->sbar[I->slot + a] / s : 1.0 / I->nA;
        }
    }
}

void or_set_state(oracle *o, const double *R, const double *sbar, int64_t t) {
    if (R) for (int64_t q = 0; q < o->na; q++) o->R[q] = (st_t)R[q];
    if (sbar) memcpy(o->sbar, sbar, (size_t)o->na * 8);
    memset(o->pred, 0, (size_t)(o->na ? o->na : 1) * sizeof(st_t));   /* no prediction yet */
    for (int64_t i = 0; i < o->ni; i++) o->avg_stamp[i] = -1;          /* the next iteration adds its average */
    o->t = t;
}

/* PCFR+ prediction (the latest instantaneous regret), canonical slot order */
void or_get_pred(const oracle *o, double *pred) {
    for (int64_t q = 0; q < o->na; q++) pred[q] = (double)o->pred[q];
}

void or_set_pred(oracle *o, const double *pred) {
    for (int64_t q = 0; q < o->na; q++) o->pred[q] = (st_t)pred[q];
}

/* ---------------- evaluation of a fixed profile ---------------- */

/* profile in canonical slot order */
static double value_rec(const oracle *o, int64_t h, const double *prof) {
    int ty = o->type[h];
    if (ty == TERM) return o->payoff[h];
    double v = 0.0;
    if (ty == CH) {
        for (int32_t a = 0; a < o->nk[h]; a++) v += o->prob[o->kb[h] + a] * value_rec(o, o->kids[o->kb[h] + a], prof);
        return v;
    }
    const oinfo *I = &o->info[o->iset[h]];
    for (int32_t a = 0; a < I->nA; a++) v += prof[I->slot + a] * value_rec(o, o->kids[o->kb[h] + a], prof);
    return v;
}

/* opponent-and-chance reach of every node for best responder `br` */
static void opp_reach(oracle *o, int64_t h, double q, int br, const double *prof) {
    o->q[h] = q;
    int ty = o->type[h];
    for (int32_t a = 0; a < o->nk[h]; a++) {
        double m = 1.0;
        if (ty == CH) m = o->prob[o->kb[h] + a];
        else if (ty != br) m = prof[o->info[o->iset[h]].slot + a];
        opp_reach(o, o->kids[o->kb[h] + a], q * m, br, prof);
    }
}

static double br_value(oracle *o, int64_t h, int br, const double *prof) {
    if (!isnan(o->memo[h])) return o->memo[h];
    int ty = o->type[h];
    double v = 0.0;
    if (ty == TERM) v = (br == PL1 ? 1.0 : -1.0) * o->payoff[h];
    else if (ty == CH) {
        for (int32_t a = 0; a < o->nk[h]; a++) v += o->prob[o->kb[h] + a] * br_value(o, o->kids[o->kb[h] + a], br, prof);
    } else if (ty != br) {
        const oinfo *I = &o->info[o->iset[h]];
        for (int32_t a = 0; a < I->nA; a++) v += prof[I->slot + a] * br_value(o, o->kids[o->kb[h] + a], br, prof);
    } else {
        int64_t Ii = o->iset[h];
        const oinfo *I = &o->info[Ii];
        if (o->astar[Ii] < 0) {
            int best = 0;
            double bq = -INFINITY;
            for (int32_t a = 0; a < I->nA; a++) {
                double Q = 0.0;
                for (int64_t k = o->mem_off[Ii]; k < o->mem_off[Ii + 1]; k++) {
                    int64_t m = o->order[o->mem[k]];
                    Q += o->q[m] * br_value(o, o->kids[o->kb[m] + a], br, prof);
                }
                if (Q > bq) { bq = Q; best = a; }
            }
            o->astar[Ii] = best;
        }
        v = br_value(o, o->kids[o->kb[h] + o->astar[Ii]], br, prof);
    }
    o->memo[h] = v;
    return v;
}

/* best-response value of player `br` (1 or 2) against profile prof (canonical slots);
 * astar_out (optional, per infoset) receives the chosen action of br's infosets */
double or_best_response(oracle *o, int br, const double *prof, int32_t *astar_out) {
    for (int64_t i = 0; i < o->n; i++) o->memo[i] = NAN;
    for (int64_t i = 0; i < o->ni; i++) o->astar[i] = -1;
    opp_reach(o, o->root, 1.0, br, prof);
    double v = br_value(o, o->root, br, prof);
    if (astar_out) for (int64_t i = 0; i < o->ni; i++) astar_out[i] = o->astar[i];
    return v;
}

double or_profile_value(const oracle *o, const double *prof) { return value_rec(o, o->root, prof); }

/* exploitability of the average profile = (BR_1 + BR_2) / 2 (NashConv / 2) */
double or_exploitability(oracle *o, double *br1, double *br2, double *value_avg) {
    double *prof = (double *)malloc((size_t)(o->na ? o->na : 1) * 8);
    or_get(o, NULL, NULL, NULL, prof);
    double b1 = or_best_response(o, PL1, prof, NULL);
    double b2 = or_best_response(o, PL2, prof, NULL);
    if (br1) *br1 = b1;
    if (br2) *br2 = b2;
    if (value_avg) *value_avg = value_rec(o, o->root, prof);
    free(prof);
    return 0.5 * (b1 + b2);
}

/* per-node values of a profile, both ways: textbook (expected payoff to P1
 * conditioned on reaching h, chance on edges) and chance-weighted (the same
 * times the chance reach of h).  Arrays are in canonical node order. */
static double values_rec(const oracle *o, int64_t h, double pic, const double *prof, double *vt, double *vf) {
    int ty = o->type[h];
    double v = 0.0;
    if (ty == TERM) v = o->payoff[h];
    else if (ty == CH) {
        for (int32_t a = 0; a < o->nk[h]; a++) {
            double p = o->prob[o->kb[h] + a];
            v += p * values_rec(o, o->kids[o->kb[h] + a], pic * p, prof, vt, vf);
        }
    } else {
        const oinfo *I = &o->info[o->iset[h]];
        for (int32_t a = 0; a < I->nA; a++)
            v += prof[I->slot + a] * values_rec(o, o->kids[o->kb[h] + a], pic, prof, vt, vf);
    }
    int64_t k = o->canon[h];
    vt[k] = v;
    vf[k] = pic * v;
    return v;
}

void or_node_values(const oracle *o, const double *prof, double *v_text, double *v_fold) {
    values_rec(o, o->root, 1.0, prof, v_text, v_fold);
}
