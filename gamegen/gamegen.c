/* gamegen.c -- seeded synthetic game builders (inputs only; see gamegen.h).
 *
 * Build steps: (1) construct the public tree once (betting, public card deals,
 * terminals; children of a public node are contiguous), (2) enumerate the
 * private deal, (3) emit the game tree breadth-first as the product of the
 * private deal and the public tree, dropping public cards that collide with a
 * hand.  Nodes come out in breadth-first order, so the children of a node are
 * contiguous ids, but consumers must not rely on that.
 */
#include "gamegen.h"
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <math.h>

uint64_t gg_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gg_hash_step(uint64_t h, int sym) {
    return gg_splitmix64(h ^ ((uint64_t)(sym + 1) * 0x100000001B3ull));
}

/* ------------------------------------------------------------------ */
/* public tree                                                          */

typedef struct {
    int8_t   type, term;        /* term: 0 showdown, 1 P1 folded, 2 P2 folded */
    int8_t   card;              /* card dealt on the edge into this node, -1 none */
    int8_t   sym;
    int8_t   nboard, round, depth;
    int8_t   board[4];
    int16_t  nkids;
    int32_t  kid0, parent;
    double   c1, c2, cprob;
    uint64_t hh;
} pubnode;

typedef struct {
    pubnode *v;
    int64_t n, cap;
    int err;
} pubtree;

static int64_t pub_reserve(pubtree *t, int64_t k) {
    if (t->n + k > t->cap) {
        int64_t nc = t->cap ? t->cap : 1024;
        while (nc < t->n + k) nc *= 2;
        pubnode *nv = (pubnode *)realloc(t->v, (size_t)nc * sizeof(pubnode));
        if (!nv) { t->err = 1; return -1; }
        t->v = nv; t->cap = nc;
    }
    int64_t b = t->n;
    memset(t->v + b, 0, (size_t)k * sizeof(pubnode));
    t->n += k;
    return b;
}

typedef struct {
    int round, to_act, raises, nact, cards_pending;
    double to_call, c1, c2;
    int nboard; int8_t board[4];
    uint64_t hh;
    int depth;
} bstate;

typedef struct {
    const gg_card_params *p;
    int deck;
} cardctx;

static void pub_fill_card(pubtree *t, const cardctx *cx, int64_t idx, bstate st, int8_t card, int8_t sym,
                          int32_t parent);

/* write the common fields of public node idx from state st */
static void pub_set(pubtree *t, int64_t idx, const bstate *st, int8_t card, int8_t sym, int32_t parent) {
    pubnode *n = &t->v[idx];
    n->card = card; n->sym = sym; n->parent = parent;
    n->nboard = (int8_t)st->nboard;
    for (int k = 0; k < 4; k++) n->board[k] = k < st->nboard ? st->board[k] : -1;
    n->round = (int8_t)st->round; n->depth = (int8_t)st->depth;
    n->c1 = st->c1; n->c2 = st->c2; n->hh = st->hh;
    n->kid0 = -1; n->nkids = 0;
}

static bstate round_end(const cardctx *cx, bstate s, int *is_showdown) {
    const gg_card_params *p = cx->p;
    if (s.round + 1 >= p->n_rounds) { *is_showdown = 1; return s; }
    *is_showdown = 0;
    s.round += 1; s.to_act = 1; s.raises = 0; s.nact = 0; s.to_call = 0.0;
    s.cards_pending = p->board_before[s.round];
    return s;
}

static void pub_fill_card(pubtree *t, const cardctx *cx, int64_t idx, bstate st, int8_t card, int8_t sym,
                          int32_t parent) {
    const gg_card_params *p = cx->p;
    if (t->err) return;
    pub_set(t, idx, &st, card, sym, parent);
    if (st.cards_pending > 0) {
        /* public card deal: one child per card not yet on the board */
        int cand[64], nc = 0;
        for (int c = 0; c < cx->deck; c++) {
            int used = 0;
            for (int k = 0; k < st.nboard; k++) if (st.board[k] == c) used = 1;
            if (!used) cand[nc++] = c;
        }
        t->v[idx].type = GG_CHANCE;
        int64_t b = pub_reserve(t, nc);
        if (b < 0) return;
        t->v[idx].kid0 = (int32_t)b; t->v[idx].nkids = (int16_t)nc;
        for (int k = 0; k < nc; k++) {
            bstate s = st;
            s.board[s.nboard++] = (int8_t)cand[k];
            s.cards_pending -= 1;
            s.hh = gg_hash_step(st.hh, 16 + cand[k]);
            s.depth = st.depth + 1;
            pub_fill_card(t, cx, b + k, s, (int8_t)cand[k], (int8_t)(16 + cand[k]), (int32_t)idx);
        }
        return;
    }
    /* betting node */
    t->v[idx].type = (int8_t)(st.to_act == 1 ? GG_P1 : GG_P2);
    int acts[4], na = 0;
    int can_raise = st.raises < p->raise_cap;
    if (st.to_call > 0.0) acts[na++] = 0;            /* fold */
    acts[na++] = 1;                                  /* check / call */
    if (can_raise) {
        acts[na++] = 2;                              /* raise (limit) / half pot */
        if (p->betting == GG_BET_POT) acts[na++] = 3;/* pot */
    }
    int64_t b = pub_reserve(t, na);
    if (b < 0) return;
    t->v[idx].kid0 = (int32_t)b; t->v[idx].nkids = (int16_t)na;
    for (int k = 0; k < na; k++) {
        int a = acts[k];
        bstate s = st;
        s.hh = gg_hash_step(st.hh, a);
        s.depth = st.depth + 1;
        double *mine = st.to_act == 1 ? &s.c1 : &s.c2;
        int64_t ci = b + k;
        if (a == 0) {                                /* fold: terminal */
            pub_set(t, ci, &s, -1, (int8_t)a, (int32_t)idx);
            t->v[ci].type = GG_TERMINAL;
            t->v[ci].term = (int8_t)(st.to_act == 1 ? 1 : 2);
            continue;
        }
        if (a == 1) {
            int ends = (st.to_call > 0.0) || (st.nact >= 1);
            *mine += st.to_call;
            s.to_call = 0.0;
            s.nact += 1;
            if (ends) {
                int sd;
                bstate nx = round_end(cx, s, &sd);
                if (sd) {
                    pub_set(t, ci, &s, -1, (int8_t)a, (int32_t)idx);
                    t->v[ci].type = GG_TERMINAL;
                    t->v[ci].term = 0;
                } else {
                    pub_fill_card(t, cx, ci, nx, -1, (int8_t)a, (int32_t)idx);
                }
            } else {
                s.to_act = 3 - st.to_act;
                pub_fill_card(t, cx, ci, s, -1, (int8_t)a, (int32_t)idx);
            }
            continue;
        }
        /* raise */
        double put;
        if (p->betting == GG_BET_LIMIT) {
            put = st.to_call + p->raise_size[st.round];
        } else {
            double pot_after_call = st.c1 + st.c2 + st.to_call;
            put = st.to_call + (a == 2 ? 0.5 * pot_after_call : pot_after_call);
        }
        *mine += put;
        s.to_call = put - st.to_call;
        s.raises += 1;
        s.nact += 1;
        s.to_act = 3 - st.to_act;
        pub_fill_card(t, cx, ci, s, -1, (int8_t)a, (int32_t)idx);
    }
}

/* random public tree for tests: arbitrary mixes of chance, decision and
 * terminal nodes at varying depths */
typedef struct { uint64_t s; } rng64;
static uint64_t rng_next(rng64 *r) { r->s += 0x9E3779B97F4A7C15ull; return gg_splitmix64(r->s); }
static double rng_unif(rng64 *r) { return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }

static void pub_fill_random(pubtree *t, const gg_random_params *p, rng64 *r, int64_t idx, int depth,
                            uint64_t hh, int8_t sym, int32_t parent) {
    if (t->err) return;
    pubnode *n = &t->v[idx];
    n->card = -1; n->sym = sym; n->parent = parent; n->depth = (int8_t)depth;
    n->hh = hh; n->kid0 = -1; n->nkids = 0; n->nboard = 0;
    for (int k = 0; k < 4; k++) n->board[k] = -1;
    double u = rng_unif(r);
    if (depth >= p->max_depth || (depth > 0 && u < p->p_terminal)) { n->type = GG_TERMINAL; n->term = 0; return; }
    int nk;
    int8_t ty;
    if (u < p->p_terminal + p->p_chance) { ty = GG_CHANCE; nk = 1 + (int)(rng_next(r) % (uint64_t)p->max_chance); }
    else { ty = (int8_t)(1 + (int)(rng_next(r) % 2)); nk = 1 + (int)(rng_next(r) % (uint64_t)p->max_actions); }
    n->type = ty;
    int64_t b = pub_reserve(t, nk);
    if (b < 0) return;
    t->v[idx].kid0 = (int32_t)b; t->v[idx].nkids = (int16_t)nk;
    if (ty == GG_CHANCE) {
        double w[16], tot = 0.0;
        for (int k = 0; k < nk; k++) { w[k] = 0.05 + rng_unif(r); tot += w[k]; }
        for (int k = 0; k < nk; k++) t->v[b + k].cprob = w[k] / tot;
    }
    for (int k = 0; k < nk; k++) {
        double cp = t->v[b + k].cprob;
        pub_fill_random(t, p, r, b + k, depth + 1, gg_hash_step(hh, 40 + k), (int8_t)(40 + k), (int32_t)idx);
        t->v[b + k].cprob = cp;
    }
}

/* ------------------------------------------------------------------ */
/* game emission                                                        */

typedef struct {
    gg_game *g;
    int64_t cap_nodes, cap_edges;
    int err;
} emitter;

static int grow_nodes(emitter *e, int64_t need) {
    gg_game *g = e->g;
    if (need <= e->cap_nodes) return 0;
    int64_t nc = e->cap_nodes ? e->cap_nodes : 4096;
    while (nc < need) nc = nc + nc / 2 + 1024;
#define RE(ptr, T) do { void *q = realloc(g->ptr, (size_t)nc * sizeof(T)); if (!q) return -1; g->ptr = (T *)q; } while (0)
    RE(type, int8_t); RE(child_begin, int64_t); RE(n_children, int32_t);
    RE(key, int64_t); RE(payoff, double); RE(pub, int64_t); RE(pair, int32_t);
#undef RE
    e->cap_nodes = nc;
    return 0;
}

static int grow_edges(emitter *e, int64_t need) {
    gg_game *g = e->g;
    if (need <= e->cap_edges) return 0;
    int64_t nc = e->cap_edges ? e->cap_edges : 4096;
    while (nc < need) nc = nc + nc / 2 + 1024;
    void *q = realloc(g->children, (size_t)nc * sizeof(int64_t)); if (!q) return -1; g->children = (int64_t *)q;
    q = realloc(g->prob, (size_t)nc * sizeof(double)); if (!q) return -1; g->prob = (double *)q;
    e->cap_edges = nc;
    return 0;
}

static int strength1(int card, const pubnode *s, int n_suits) {
    int r = card / n_suits;
    for (int k = 0; k < s->nboard; k++)
        if (s->board[k] / n_suits == r) return 100 + r;
    return r;
}

typedef struct {
    int n_suits, payoff_mode;
    uint64_t seed;
} payctx;

static double terminal_payoff(const payctx *pc, const pubnode *s, const gg_hand *h1, const gg_hand *h2) {
    if (pc->payoff_mode == GG_PAY_HASH) {
        uint64_t k = gg_splitmix64(pc->seed ^ (((uint64_t)(uint32_t)h1->gid << 20) | (uint64_t)(uint32_t)h2->gid));
        uint64_t z = gg_splitmix64(s->hh ^ k);
        double U = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        return 2.0 * U - 1.0;
    }
    if (s->term == 1) return -s->c1;
    if (s->term == 2) return s->c2;
    int a = strength1(h1->card[0], s, pc->n_suits), b = strength1(h2->card[0], s, pc->n_suits);
    if (a > b) return s->c2;
    if (a < b) return -s->c1;
    return 0.0;
}

static int hands_clash(const gg_hand *a, const gg_hand *b) {
    for (int x = 0; x < 2; x++)
        for (int y = 0; y < 2; y++)
            if (a->card[x] >= 0 && a->card[x] == b->card[y]) return 1;
    return 0;
}

static int hand_has(const gg_hand *a, int c) { return a->card[0] == c || a->card[1] == c; }

static int emit_game(gg_game *g, const pubtree *t, int n1, const gg_hand *H1, int n2, const gg_hand *H2,
                     int sequential, const payctx *pc) {
    emitter e = { g, 0, 0, 0 };
    /* pairs, i-major */
    int64_t npairs = 0;
    for (int i = 0; i < n1; i++) for (int j = 0; j < n2; j++) if (!hands_clash(&H1[i], &H2[j])) npairs++;
    g->n_pairs = npairs;
    if (npairs == 0) return -2;
    g->pair_h1 = (int32_t *)malloc((size_t)(npairs ? npairs : 1) * sizeof(int32_t));
    g->pair_h2 = (int32_t *)malloc((size_t)(npairs ? npairs : 1) * sizeof(int32_t));
    int64_t *pair_of = (int64_t *)malloc((size_t)n1 * n2 * sizeof(int64_t) + 8);
    if (!g->pair_h1 || !g->pair_h2 || !pair_of) { free(pair_of); return -1; }
    {
        int64_t k = 0;
        for (int i = 0; i < n1; i++) for (int j = 0; j < n2; j++) {
            if (!hands_clash(&H1[i], &H2[j])) { g->pair_h1[k] = i; g->pair_h2[k] = j; pair_of[(int64_t)i * n2 + j] = k++; }
            else pair_of[(int64_t)i * n2 + j] = -1;
        }
    }
    int KH = n1 > n2 ? n1 : n2;
    /* stage of each node is implied by its id range: root (0), P2-deal nodes (sequential only), then pair nodes */
    int64_t nn = 0, ne = 0;
    if (grow_nodes(&e, 1 + n1 + npairs + 16) < 0) goto oom;
    /* root */
    g->type[0] = GG_CHANCE; g->key[0] = -1; g->payoff[0] = 0.0; g->pub[0] = -1; g->pair[0] = -1;
    nn = 1;
    /* per node public index for pair-stage nodes is kept in pub[] */
    int64_t first_pair_node;
    {
        if (sequential) {
            double w1 = 0.0;
            for (int i = 0; i < n1; i++) w1 += H1[i].weight;
            if (grow_edges(&e, n1) < 0) goto oom;
            g->child_begin[0] = 0; g->n_children[0] = n1;
            for (int i = 0; i < n1; i++) {
                g->children[ne] = nn; g->prob[ne] = H1[i].weight / w1; ne++;
                g->type[nn] = GG_CHANCE; g->key[nn] = -1; g->payoff[nn] = 0.0; g->pub[nn] = -1; g->pair[nn] = -1;
                nn++;
            }
            for (int i = 0; i < n1; i++) {
                int64_t node = 1 + i;
                double w2 = 0.0; int cnt = 0;
                for (int j = 0; j < n2; j++) if (pair_of[(int64_t)i * n2 + j] >= 0) { w2 += H2[j].weight; cnt++; }
                if (grow_edges(&e, ne + cnt) < 0 || grow_nodes(&e, nn + cnt) < 0) goto oom;
                g->child_begin[node] = ne; g->n_children[node] = cnt;
                for (int j = 0; j < n2; j++) {
                    int64_t pk = pair_of[(int64_t)i * n2 + j];
                    if (pk < 0) continue;
                    g->children[ne] = nn; g->prob[ne] = H2[j].weight / w2; ne++;
                    g->pair[nn] = (int32_t)pk; g->pub[nn] = 0; nn++;
                }
            }
            first_pair_node = 1 + n1;
        } else {
            double w = 0.0;
            for (int64_t k = 0; k < npairs; k++) w += H1[g->pair_h1[k]].weight * H2[g->pair_h2[k]].weight;
            if (grow_edges(&e, npairs) < 0 || grow_nodes(&e, 1 + npairs) < 0) goto oom;
            g->child_begin[0] = 0; g->n_children[0] = (int32_t)npairs;
            for (int64_t k = 0; k < npairs; k++) {
                g->children[ne] = nn;
                g->prob[ne] = H1[g->pair_h1[k]].weight * H2[g->pair_h2[k]].weight / w;
                ne++;
                g->pair[nn] = (int32_t)k; g->pub[nn] = 0; nn++;
            }
            first_pair_node = 1;
        }
    }
    /* breadth-first expansion of pair-stage nodes */
    for (int64_t n = first_pair_node; n < nn; n++) {
        int64_t s = g->pub[n];
        int32_t pk = g->pair[n];
        const pubnode *ps = &t->v[s];
        const gg_hand *h1 = &H1[g->pair_h1[pk]], *h2 = &H2[g->pair_h2[pk]];
        g->type[n] = ps->type;
        g->key[n] = -1; g->payoff[n] = 0.0;
        g->child_begin[n] = ne; g->n_children[n] = 0;
        if (ps->type == GG_TERMINAL) { g->payoff[n] = terminal_payoff(pc, ps, h1, h2); continue; }
        if (ps->type == GG_P1 || ps->type == GG_P2) {
            int hand = ps->type == GG_P1 ? g->pair_h1[pk] : g->pair_h2[pk];
            g->key[n] = ((int64_t)s * KH + hand) * 2 + (ps->type - 1);
        }
        int cnt = 0;
        for (int k = 0; k < ps->nkids; k++) {
            const pubnode *c = &t->v[ps->kid0 + k];
            if (c->card >= 0 && (hand_has(h1, c->card) || hand_has(h2, c->card))) continue;
            cnt++;
        }
        if (grow_edges(&e, ne + cnt) < 0 || grow_nodes(&e, nn + cnt) < 0) goto oom;
        ps = &t->v[s];
        g->n_children[n] = cnt;
        for (int k = 0; k < ps->nkids; k++) {
            const pubnode *c = &t->v[ps->kid0 + k];
            if (c->card >= 0 && (hand_has(h1, c->card) || hand_has(h2, c->card))) continue;
            g->children[ne] = nn;
            if (ps->type == GG_CHANCE) g->prob[ne] = c->card >= 0 ? 1.0 / cnt : c->cprob;
            else g->prob[ne] = 0.0;
            ne++;
            g->pair[nn] = pk; g->pub[nn] = ps->kid0 + k; nn++;
        }
    }
    /* deal nodes have no public state */
    for (int64_t n = 0; n < first_pair_node; n++) g->pub[n] = -1;
    g->n_nodes = nn; g->n_edges = ne;
    free(pair_of);
    return 0;
oom:
    free(pair_of);
    return -1;
}

static void export_pub(gg_game *g, const pubtree *t) {
    int64_t n = t->n;
    g->n_pub = n;
    g->pub_type = (int8_t *)malloc((size_t)n);
    g->pub_c1 = (double *)malloc((size_t)n * sizeof(double));
    g->pub_c2 = (double *)malloc((size_t)n * sizeof(double));
    g->pub_round = (int8_t *)malloc((size_t)n);
    g->pub_depth = (int8_t *)malloc((size_t)n);
    g->pub_parent = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    g->pub_sym = (int8_t *)malloc((size_t)n);
    if (!g->pub_type || !g->pub_c1 || !g->pub_c2 || !g->pub_round || !g->pub_depth || !g->pub_parent || !g->pub_sym)
        return;
    for (int64_t i = 0; i < n; i++) {
        g->pub_type[i] = t->v[i].type; g->pub_c1[i] = t->v[i].c1; g->pub_c2[i] = t->v[i].c2;
        g->pub_round[i] = t->v[i].round; g->pub_depth[i] = t->v[i].depth;
        g->pub_parent[i] = t->v[i].parent; g->pub_sym[i] = t->v[i].sym;
    }
}

static void set_err(gg_game *g, const char *m) { g->error = 1; snprintf(g->msg, sizeof g->msg, "%s", m); }

int gg_build_card(const gg_card_params *p, gg_game *out) {
    memset(out, 0, sizeof *out);
    if (p->n_ranks <= 0 || p->n_suits <= 0 || p->n_ranks * p->n_suits > 60) { set_err(out, "bad deck"); return 1; }
    if (p->n_rounds < 1 || p->n_rounds > 4 || p->first_round < 0 || p->first_round >= p->n_rounds) {
        set_err(out, "bad rounds"); return 1;
    }
    if (p->n_hands1 <= 0 || p->n_hands2 <= 0) { set_err(out, "no hands"); return 1; }
    if (p->payoff_mode == GG_PAY_SHOWDOWN) {
        for (int i = 0; i < p->n_hands1; i++) if (p->hands1[i].card[1] >= 0) { set_err(out, "showdown needs 1-card hands"); return 1; }
        for (int i = 0; i < p->n_hands2; i++) if (p->hands2[i].card[1] >= 0) { set_err(out, "showdown needs 1-card hands"); return 1; }
    }
    cardctx cx = { p, p->n_ranks * p->n_suits };
    pubtree t = { 0, 0, 0, 0 };
    bstate st;
    memset(&st, 0, sizeof st);
    st.round = p->first_round; st.to_act = 1; st.c1 = p->contrib1; st.c2 = p->contrib2;
    st.cards_pending = p->board_before[p->first_round];
    st.nboard = p->n_fixed_board;
    for (int k = 0; k < p->n_fixed_board; k++) st.board[k] = p->fixed_board[k];
    st.hh = p->root_hash;
    pub_reserve(&t, 1);
    pub_fill_card(&t, &cx, 0, st, -1, -1, -1);
    if (t.err) { free(t.v); set_err(out, "out of memory (public tree)"); return 2; }
    payctx pc = { p->n_suits, p->payoff_mode, p->seed };
    /* hands colliding with the fixed board can never be dealt */
    for (int i = 0; i < p->n_hands1; i++) for (int k = 0; k < p->n_fixed_board; k++)
        if (hand_has(&p->hands1[i], p->fixed_board[k])) { free(t.v); set_err(out, "hand collides with board"); return 1; }
    for (int i = 0; i < p->n_hands2; i++) for (int k = 0; k < p->n_fixed_board; k++)
        if (hand_has(&p->hands2[i], p->fixed_board[k])) { free(t.v); set_err(out, "hand collides with board"); return 1; }
    int rc = emit_game(out, &t, p->n_hands1, p->hands1, p->n_hands2, p->hands2, p->sequential_deal, &pc);
    out->pot_at_root = p->contrib1 + p->contrib2;
    export_pub(out, &t);
    free(t.v);
    if (rc == -2) { set_err(out, "no compatible pair of hands"); return 1; }
    if (rc) { set_err(out, "out of memory (game)"); return 2; }
    return 0;
}

int gg_build_random(const gg_random_params *p, gg_game *out) {
    memset(out, 0, sizeof *out);
    if (p->n_types1 <= 0 || p->n_types2 <= 0 || p->max_actions < 1 || p->max_actions > 8 || p->max_chance < 1 ||
        p->max_chance > 8) {
        set_err(out, "bad random params"); return 1;
    }
    rng64 r = { p->seed * 0x2545F4914F6CDD1Dull + 17 };
    pubtree t = { 0, 0, 0, 0 };
    pub_reserve(&t, 1);
    pub_fill_random(&t, p, &r, 0, 0, 0x51ED270B27u, -1, -1);
    if (t.err) { free(t.v); set_err(out, "out of memory (public tree)"); return 2; }
    gg_hand *H1 = (gg_hand *)calloc((size_t)p->n_types1, sizeof(gg_hand));
    gg_hand *H2 = (gg_hand *)calloc((size_t)p->n_types2, sizeof(gg_hand));
    for (int i = 0; i < p->n_types1; i++) { H1[i].card[0] = H1[i].card[1] = -1; H1[i].gid = i; H1[i].weight = 0.1 + rng_unif(&r); }
    for (int i = 0; i < p->n_types2; i++) { H2[i].card[0] = H2[i].card[1] = -1; H2[i].gid = i; H2[i].weight = 0.1 + rng_unif(&r); }
    payctx pc = { 1, GG_PAY_HASH, p->seed };
    int rc = emit_game(out, &t, p->n_types1, H1, p->n_types2, H2, 0, &pc);
    out->pot_at_root = 1.0;
    export_pub(out, &t);
    free(H1); free(H2); free(t.v);
    if (rc) { set_err(out, "out of memory (game)"); return 2; }
    return 0;
}

void gg_free(gg_game *g) {
    free(g->type); free(g->child_begin); free(g->n_children); free(g->children); free(g->prob);
    free(g->key); free(g->payoff); free(g->pub); free(g->pair); free(g->pair_h1); free(g->pair_h2);
    free(g->pub_type); free(g->pub_c1); free(g->pub_c2); free(g->pub_round); free(g->pub_depth);
    free(g->pub_parent); free(g->pub_sym);
    memset(g, 0, sizeof *g);
}
