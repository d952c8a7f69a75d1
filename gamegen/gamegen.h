/* gamegen.h -- seeded synthetic game builders.
 *
 * This module only produces INPUTS: explicit game trees in the tabular form
 * that a CFR compiler consumes (a node table with type, acting player,
 * information-set key, children and terminal payoff, plus a chance
 * probability for every chance edge).  It holds none of the solver's
 * arithmetic: no reach, value, regret or strategy computation happens here.
 * Both the CFR library and the CPU oracle read its output; neither is
 * imported by it.
 *
 * Every game is "public tree x private deal": a root deal of private hands
 * (jointly, or P1 then P2), followed by a public tree of betting, public card
 * deals and terminals that is identical for every hand pair except that cards
 * held by a player cannot be dealt publicly.  An information set is
 * (player, own hand, public history), which gives perfect recall.
 */
#ifndef GAMEGEN_H
#define GAMEGEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GG_CHANCE = 0, GG_P1 = 1, GG_P2 = 2, GG_TERMINAL = 3 };

/* Betting model of a round. */
enum { GG_BET_LIMIT = 0, /* not facing: check, raise; facing: fold, call, raise */
       GG_BET_POT = 1    /* not facing: check, half-pot, pot; facing: fold, call, half-pot, pot */ };

/* Terminal payoff model. */
enum { GG_PAY_SHOWDOWN = 0, /* chips: fold loses own contribution; showdown by rank with board pairing */
       GG_PAY_HASH = 1      /* 2U-1, U from SplitMix64 keyed by (seed, hands, public history) */ };

/* A private hand: up to two hole cards (-1 = none) and a global id used by
 * the hash payoff; weight enters the root deal probability. */
typedef struct {
    int8_t  card[2];
    int32_t gid;
    double  weight;
} gg_hand;

typedef struct {
    int      n_ranks, n_suits;      /* deck = n_ranks*n_suits cards, card c has rank c/n_suits */
    int      n_hands1, n_hands2;
    const gg_hand *hands1, *hands2;
    int      sequential_deal;       /* 0: one chance node over compatible pairs; 1: P1 hand then P2 hand */
    int      n_rounds;              /* betting rounds played (1..4) */
    int      board_before[4];       /* public cards dealt before round r */
    int      n_fixed_board;         /* cards already on the board at the public root */
    int8_t   fixed_board[4];
    int      betting;               /* GG_BET_* */
    int      raise_cap;             /* raises per round */
    double   raise_size[4];         /* limit betting: chips per raise in round r */
    double   contrib1, contrib2;    /* chips in the pot at the public root (antes plus earlier rounds) */
    int      payoff_mode;           /* GG_PAY_* */
    uint64_t seed;                  /* hash payoff seed */
    uint64_t root_hash;             /* content hash of the public history at the public root */
    int      first_round;           /* index of the first round played (for subgames cut mid-game) */
} gg_card_params;

typedef struct {
    uint64_t seed;
    int      n_types1, n_types2;    /* private types per player */
    int      max_depth;             /* public-tree depth cap */
    double   p_terminal, p_chance;  /* per-node probabilities of terminal / chance */
    int      max_actions;           /* decision actions 1..max_actions */
    int      max_chance;            /* chance outcomes 1..max_chance */
} gg_random_params;

/* The produced game.  Node ids are 0..n_nodes-1 with the root at 0; the
 * children of node n are children[child_begin[n] .. child_begin[n]+n_children[n])
 * in action order, and prob[] is aligned with children[] (probability of the
 * chance outcome; 0 for decision edges). key[] is the information-set key of
 * decision nodes (-1 otherwise), payoff[] the payoff to player 1 at terminals,
 * pub[] the public-state id of every node (-1 for deal nodes). */
typedef struct {
    int64_t  n_nodes, n_edges;
    int8_t  *type;
    int64_t *child_begin;
    int32_t *n_children;
    int64_t *children;
    double  *prob;
    int64_t *key;
    double  *payoff;
    int64_t *pub;
    int64_t  n_pub;                 /* public-tree size */
    double   pot_at_root;           /* contrib1+contrib2 at the public root */
    /* per public node (n_pub): owner/type, contributions, round and action path length;
     * used by feature builders for learned warm starts */
    int8_t  *pub_type;
    double  *pub_c1, *pub_c2;
    int8_t  *pub_round;
    int8_t  *pub_depth;
    int32_t *pub_parent;
    int8_t  *pub_sym;               /* symbol on the edge into the public node (-1 root) */
    /* per node: index of its private pair (-1 for deal nodes) */
    int32_t *pair;
    int32_t *pair_h1, *pair_h2;     /* hand indices of each pair */
    int64_t  n_pairs;
    int      error;
    char     msg[160];
} gg_game;

int  gg_build_card(const gg_card_params *p, gg_game *out);
int  gg_build_random(const gg_random_params *p, gg_game *out);
void gg_free(gg_game *g);
/* content hash of a public history prefix: apply symbols to a hash state
 * (symbols: 0 fold, 1 check/call, 2 raise/half-pot, 3 pot, 16+c card c) */
uint64_t gg_hash_step(uint64_t h, int sym);
uint64_t gg_splitmix64(uint64_t x);

#ifdef __cplusplus
}
#endif
#endif
