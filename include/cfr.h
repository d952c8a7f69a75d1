/* cfr.h -- C ABI of the MI355X compiled-CFR library.
 *
 * One CFR iteration over a two-player zero-sum perfect-recall game compiled
 * to static, depth-sorted arrays (paper: Section 4 "Compiling CFR onto
 * Accelerators", Algorithm 'alg:iteration'; compiler passes: Appendix H,
 * Algorithm 'alg:compile'):
 *   regret matching (eq. rm) -> forward reach pass per depth level (eqs.
 *   reach, lanes) -> backward counterfactual-value pass per depth level
 *   (eq. cfv with chance folded into a values template, eq. template) ->
 *   per-information-set regret accumulation (eqs. regret, instregret) with
 *   the CFR+ clamp -> FP64 average-strategy update (eq. rm, Proposition 4).
 * All of it runs in hand-written gfx950 HIP kernels; one iteration (or k) is
 * captured into a hipGraph and replayed.
 *
 * Conventions for every entry point:
 *  - Every function returns cfr_status; nothing throws across the ABI.  On
 *    failure a message is kept per thread and returned by cfr_last_error().
 *  - Pointers are plain host or device pointers, as each argument states.
 *    The caller owns every input; cfr_compile copies what it needs and keeps
 *    no caller pointer.  The handle owns all device memory until
 *    cfr_destroy.
 *  - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  Work is enqueued asynchronously unless stated.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Slot order: every per-slot array crossing the ABI (strategies, regrets,
 *    strategy sums) is in CANONICAL order: information sets numbered by first
 *    occurrence in breadth-first node order (children in action order), the
 *    actions of a set contiguous.  cfr_layout_host() returns that numbering.
 */
#ifndef CFR_H
#define CFR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CFR_OK = 0,
    CFR_EINVAL = 1,         /* invalid argument or invalid game */
    CFR_ENOMEM = 2,         /* host or device allocation failed */
    CFR_EDEVICE = 3,        /* a HIP call failed */
    CFR_EGRAPH = 4,         /* graph capture or launch failed */
    CFR_ESTATE = 5,         /* handle state forbids the call (e.g. a persistent buffer was rebound) */
    CFR_EUNSUPPORTED = 6    /* valid request this build does not support */
} cfr_status;

enum { CFR_NODE_CHANCE = 0, CFR_NODE_P1 = 1, CFR_NODE_P2 = 2, CFR_NODE_TERMINAL = 3 };

/* Explicit game specification (paper Appendix H, "Input representation"):
 * a node table with type, acting player, information-set key, children in
 * action order and terminal payoff, plus the chance probability of every
 * chance outcome.  All arrays are HOST memory and are only read.
 *   num_nodes      number of nodes; ids 0..num_nodes-1 in any order
 *   root           id of the root
 *   node_type      [num_nodes] CFR_NODE_*
 *   child_begin    [num_nodes] index into children[] of the node's first child
 *   num_children   [num_nodes] 0 for terminals, >= 1 otherwise (<= 64 at decision nodes)
 *   children       child ids, children[child_begin[n] + a] is the child after action a
 *   chance_prob    aligned with children[]; read only below chance nodes; each chance
 *                  node's probabilities must be >= 0 and sum to 1 within 1e-9
 *   infoset_key    [num_nodes] information-set key of decision nodes (ignored elsewhere);
 *                  members of one set must share player and action count
 *   payoff         [num_nodes] payoff to player 1 at terminals (player 2 receives -payoff)
 *   public_key     [num_nodes] optional (NULL): public-state id of every node; enables
 *                  CFR_LAYOUT_PUBLIC
 *   pot            exploitability unit (> 0) reported back by cfr_counts
 *   root_hand1, root_hand2
 *                  optional (NULL): for a game whose root is a chance node dealing one private hand
 *                  to each player (a subgame's joint deal), the hands dealt by root child a, as indices
 *                  into the range vectors of cfr_set_root_ranges: [num_children[root]] each, in
 *                  [0, num_hands1) and [0, num_hands2)
 *   num_hands1, num_hands2
 *                  lengths of the two range vectors (read only when root_hand1 is given)
 * Validation (Algorithm 'alg:compile', first pass, plus perfect recall): a tree reachable
 * from root with one parent per non-root node, valid types, chance sums, information sets
 * owned by one player with equal action counts, and identical own-action sequences for all
 * members of a set.  Violations return CFR_EINVAL. */
typedef struct {
    int64_t        num_nodes;
    int64_t        root;
    const int8_t  *node_type;
    const int64_t *child_begin;
    const int32_t *num_children;
    const int64_t *children;
    const double  *chance_prob;
    const int64_t *infoset_key;
    const double  *payoff;
    const int64_t *public_key;
    double         pot;
    const int32_t *root_hand1, *root_hand2;
    int32_t        num_hands1, num_hands2;
} cfr_game_desc;

/* Update rules (paper Sec. 6, "Update rule and update order"); the constants the paper leaves out
 * are those of the published methods:
 *   CFR+   R = max(R + r, 0); average weight w_t (CFR_AVG_*)
 *   CFR    R = R + r;         average weight w_t
 *   DCFR   R = R + r, then multiplied by t^1.5/(t^1.5+1) where positive and by 1/2 where not;
 *          strategy sums S = (S + pi_i sigma) (t/(t+1))^2 (averaging option ignored)
 *   PCFR+  R = max(R + r, 0); the next strategy is regret matching of R + r (the latest
 *          instantaneous regret as the prediction); average weight t^2 (averaging option ignored)
 * Alternating order: each iteration runs player 1's half (its regrets, sums and strategy) and then
 * player 2's half against player 1's updated strategy, both with the weights of iteration t. */
enum { CFR_RULE_CFR_PLUS = 0, CFR_RULE_CFR = 1, CFR_RULE_DCFR = 2, CFR_RULE_PCFR_PLUS = 3 };
enum { CFR_AVG_LINEAR = 0, CFR_AVG_UNIFORM = 1 };       /* w_t = t or 1 (CFR and CFR+) */
enum { CFR_ORDER_SIMULTANEOUS = 0, CFR_ORDER_ALTERNATING = 1 };
/* Device node order within a depth level.  BFS: the canonical order.  PUBLIC: internal nodes
 * first, then terminals, each grouped by public state (first occurrence), canonical order
 * inside a group; this keeps an information set's members and each level's writes together. */
enum { CFR_LAYOUT_BFS = 0, CFR_LAYOUT_PUBLIC = 1 };
enum { CFR_STRATEGY_CURRENT = 0, CFR_STRATEGY_AVERAGE = 1 };
enum { CFR_PRECISION_FP32 = 0, CFR_PRECISION_FP64 = 1 };
/* Schedules (cfr_options.persistent, cfr_set_schedule):
 *   LEVEL       one launch per depth level, the iteration captured once and replayed (default)
 *   PERSISTENT  one launch per cfr_iterate call running all n iterations of every game of a batch,
 *               per-game barriers between levels; workgroups claim (game, rank) tickets in order from
 *               per-XCD queues (cfr_persistent_plan_host), so a barrier only waits for running ones
 *   LDS         one workgroup per cfr_iterate call running all n iterations of one tiny standalone
 *               game with its whole state in LDS (paper Sec. Results, cross-framework timing: the fixed
 *               launch-and-replay floor per iteration that small games cannot fill):
 *               values, both reach lanes, strategy, regrets, strategy sums (and the PCFR+
 *               prediction) must fit the device's LDS per workgroup, and sets have at most 16
 *               actions; same arithmetic as LEVEL, bitwise equal iterates */
enum { CFR_SCHEDULE_LEVEL = 0, CFR_SCHEDULE_PERSISTENT = 1, CFR_SCHEDULE_LDS = 2 };

typedef struct {
    int rule;              /* CFR_RULE_* (default CFR+) */
    int averaging;         /* CFR_AVG_* (default linear) */
    int order;             /* CFR_ORDER_* (default simultaneous) */
    int iters_per_graph;   /* k iterations captured per graph (default 1) */
    int layout;            /* CFR_LAYOUT_* (default PUBLIC; without public keys it orders internal
                              nodes before terminals inside each depth) */
    int use_graph;         /* 1: hipGraph replay (default); 0: direct kernel launches */
    int device;            /* HIP device ordinal (default 0) */
    int test_fail_capture; /* test hook: treat graph capture as failed (warns once, launches directly) */
    int precision;         /* CFR_PRECISION_*: type of reach, values, regrets and strategy (default FP32);
                              strategy sums are FP64 in both */
    int persistent;        /* schedule, CFR_SCHEDULE_* (default LEVEL); LDS fails with CFR_EINVAL when the
                              game does not fit or is a batch */
    int wg_nodes;          /* persistent form: target nodes per workgroup (0 = 16384); cfr_autotune picks it */
    int lifecycle;         /* 1: keep per terminal its node, payoff and chance product (and each game's root
                              chance) on the device, for cfr_set_payoffs / cfr_set_root_chance (default 0) */
    int affine;            /* 1 (default): when the PUBLIC layout places child a of every member h of a set
                              at h + offset(set, a), the update pass reads one offset per slot instead of
                              the explicit child list (same arithmetic, bitwise equal results); 0: always
                              read the child list */
    int keep_layout;       /* 1: keep every game's canonical arrays on the host for cfr_get_layout (about
                              30 bytes per node of host memory; default 0) */
    int group_sets;        /* sets per update group of the backward/update pass: 0 (default) chooses 128
                              or 256 from the game's (or batch's) set sizes, 128 or 256 forces it; any
                              other value fails with CFR_EINVAL.  Results do not depend on it (each
                              set's reduction order is fixed), only the speed does. */
} cfr_options;

/* Sizes of a compiled game.  blocks = number of depth levels that hold edges (D of eq. blocks). */
typedef struct {
    int64_t nodes, edges, terminals, decision_nodes, infosets, slots;
    int32_t max_depth, blocks, max_actions, br_supported;
    int64_t device_bytes;          /* device memory held by the handle */
    int64_t kernels_per_iteration; /* launches in one iteration (the operation-count gate) */
    double  pot;
    int32_t child_addressing;      /* update pass: 0 implicit (BFS), 1 explicit child list, 2 affine offsets */
    int32_t node_order_groups;     /* affine update groups whose members are listed in node order (their sets
                                      interleave); 0 in the counts of cfr_layout_host and cfr_get_layout */
    int64_t node_order_members;    /* members of those groups */
    int32_t group_sets;            /* sets per update group (128 or 256); 0 in the counts of cfr_layout_host
                                      and cfr_get_layout */
    int32_t update_groups;         /* update groups (one workgroup each per iteration); 0 there too */
} cfr_counts_t;

/* Canonical compiled arrays (host copies), all in canonical numbering:
 *   depth_off [max_depth+2]  nodes of depth d are [depth_off[d], depth_off[d+1])
 *   parent    [nodes]        -1 at the root
 *   child_off [nodes+1]      children of n are [child_off[n], child_off[n+1])
 *   in_slot   [nodes]        slot of the edge into n, -1 below chance and at the root
 *   node_infoset [nodes]     -1 at non-decision nodes
 *   node_type [nodes]
 *   tmpl      [nodes]        pi_c(z) u(z) at terminals, rounded once to float (eq. template), 0 elsewhere
 *   slot_off  [infosets+1], mem_off [infosets+1], mem_node [decision_nodes] (ascending)
 *   iset_player [infosets], iset_key [infosets] */
typedef struct {
    cfr_counts_t counts;
    int32_t *depth_off, *parent, *child_off, *in_slot, *node_infoset;
    int8_t  *node_type;
    float   *tmpl;
    int32_t *slot_off, *mem_off, *mem_node;
    int8_t  *iset_player;
    int64_t *iset_key;
} cfr_layout;

typedef struct cfr_handle cfr_handle;

/* Fill *opt with the defaults (CFR+, linear, simultaneous, k=1, PUBLIC layout, graph on, device 0,
 * FP32). */
void cfr_default_options(cfr_options *opt);

/* Host-only compile (no GPU touched): validate the game and return its canonical arrays
 * in *out (library-allocated; release with cfr_layout_free).  The arrays are those cfr_compile
 * builds for the same description (Appendix H, Algorithm 'alg:compile', passes 1-7). */
cfr_status cfr_layout_host(const cfr_game_desc *game, cfr_layout *out);
void cfr_layout_free(cfr_layout *layout);

/* The canonical arrays of game `game` (in [0, n_games)) of a compiled handle, as cfr_layout_host
 * returns them (library-allocated host copies; release with cfr_layout_free).  The handle must have
 * been compiled with options.keep_layout = 1 (CFR_ESTATE otherwise); counts.device_bytes and
 * counts.kernels_per_iteration are those of the whole handle. */
cfr_status cfr_get_layout(cfr_handle *h, int32_t game, cfr_layout *out);

/* Compile a game onto the device (Algorithm 'alg:compile'): validate, number nodes
 * breadth-first, build depth offsets, information sets and slots, the CSR arrays and
 * member lists, fold chance into the values template, copy everything to the device once,
 * and set R = 0, sbar = 0, t = 0, sigma = uniform.  opt may be NULL (defaults).
 * On success *out receives a new handle. */
cfr_status cfr_compile(const cfr_game_desc *game, const cfr_options *opt, cfr_handle **out);

/* Batched form: compile n independent games (e.g. subgames of one game with their own root
 * ranges) into one handle.  They are laid out as a depth-major forest -- the depth-d nodes,
 * information sets and slots of game 0, then of game 1, ... -- so one launch per level (or one
 * persistent launch, see cfr_options.persistent) advances every game.  Per-slot arrays at the ABI
 * hold game 0's canonical slots, then game 1's (offsets from cfr_batch_size).  Games are
 * validated one by one; the message of a failure names the game.  n == 1 equals cfr_compile. */
cfr_status cfr_compile_batch(const cfr_game_desc *games, int32_t n, const cfr_options *opt, cfr_handle **out);

/* Schedule chosen by cfr_autotune. */
typedef struct {
    int32_t persistent;        /* chosen schedule, CFR_SCHEDULE_* */
    int32_t wg_nodes;          /* persistent form: target nodes per workgroup */
    int32_t blocks;            /* workgroups of the launch (persistent form; 1 for LDS; 0 for LEVEL) */
    int32_t candidates;        /* schedules measured (0 when read from the cache) */
    double  ms_per_iteration;  /* measured time of the chosen schedule */
    int32_t failed;            /* persistent candidates dropped because a per-game barrier timed out */
} cfr_tune_result;

/* Autotuner: time `iters` iterations under each candidate schedule -- one launch per level, the
 * persistent launch at several workgroup sizes, and for one game that fits, the LDS schedule --
 * keep the fastest, and reset the solver
 * state (the measurement iterations are discarded).  With cache_path != NULL the choice is read
 * from / appended to that text file, keyed by device name, precision and the handle's sizes.
 * Synchronous. */
cfr_status cfr_autotune(cfr_handle *h, int64_t iters, void *stream, const char *cache_path, cfr_tune_result *out);

/* Select a schedule explicitly (as cfr_autotune would): persistent = CFR_SCHEDULE_* and, for the
 * persistent form, the target nodes per workgroup (0 = 16384).  The solver state is kept.  Errors:
 * CFR_EINVAL for an unknown schedule, or LDS for a batch, a game over the LDS budget or sets with
 * more than 16 actions (the schedule then stays as it was). */
cfr_status cfr_set_schedule(cfr_handle *h, int32_t persistent, int32_t wg_nodes);

/* Host-only (no GPU touched): the work plan the persistent schedule builds for n games of nodes[g]
 * nodes (the batched form is not in the paper; its concluding remarks motivate one launch per batch of
 * solves).  Game g gets W[g] = max(1, ceil(nodes[g] / wg_nodes_used)) workgroups ("ranks"), which are
 * consecutive tickets of queue[g], one of 8 per-XCD queues (games placed largest first on the least
 * loaded queue); q_off[9] gives each queue's ticket range; *wg_nodes_used is wg_nodes (0: 16384)
 * doubled until every W[g] <= max_w.  Workgroups claim tickets in order, so a game's barrier waits only
 * for ranks already claimed by running workgroups, and at most one game per queue is partly claimed:
 * the launch progresses whenever 8 (max_w - 1) + 1 workgroups can be resident.  cfr_set_schedule uses
 * max_w = a quarter of one XCD's resident workgroups.  Caller-owned outputs W[n], queue[n], q_off[9].
 * CFR_EINVAL for bad arguments, CFR_EUNSUPPORTED if no wg_nodes below 2^30 fits. */
cfr_status cfr_persistent_plan_host(const int64_t *nodes, int32_t n, int32_t wg_nodes, int32_t max_w, int32_t *W,
                                    int32_t *queue, int32_t *q_off, int32_t *wg_nodes_used);

/* Number of games in the handle and (if slot_base != NULL) the n + 1 offsets of each game's
 * canonical slots in the per-slot arrays. */
cfr_status cfr_batch_size(cfr_handle *h, int32_t *n_games, int64_t *slot_base);

/* Per-game exploitability of the average profile: arrays of n entries (any may be NULL), as
 * cfr_exploitability computes for one game.  Synchronises `stream`. */
cfr_status cfr_batch_exploitability(cfr_handle *h, void *stream, double *expl, double *br1, double *br2,
                                    double *value_avg, int32_t n);

/* Run n CFR iterations on `stream` (asynchronous): per iteration, regret matching (eq. rm), the
 * forward reach pass and the backward value pass level by level with the regret, clamp and average
 * updates fused into the backward levels (Algorithm 'alg:iteration'; Table 'tab:opsteps').  The first
 * call captures the iteration body into a hipGraph (after one direct iteration that counts toward n)
 * and later calls replay it (Sec. 4, "CUDA-graph execution").  n == 0 is a no-op.  Returns CFR_ESTATE
 * if a persistent buffer recorded at capture time has changed, or after a persistent launch stopped
 * part-way (until cfr_reset or cfr_set_state).  Under the persistent schedule the call is one launch
 * that runs all n iterations and synchronises `stream`, so that a per-game barrier time-out
 * (CFR_EDEVICE) is reported by the call that hit it. */
cfr_status cfr_iterate(cfr_handle *h, int64_t n, void *stream);

/* Iterations completed so far (host count). */
cfr_status cfr_iterations(cfr_handle *h, int64_t *t);

/* Write the current strategy (regret matching of the latest regrets, eq. rm: the strategy
 * the next iteration plays) or the normalised average strategy (the strategy sums of eq. rm over
 * their total; uniform where the sum is 0) as float32 into dst[len] in canonical slot order; len
 * must equal the slot count.
 * dst_on_device selects a device (1) or host (0) pointer; a host destination synchronises
 * the stream. */
cfr_status cfr_strategy(cfr_handle *h, int which, float *dst, int64_t len, int dst_on_device, void *stream);

/* Exploitability of the average profile (eq. exploitability): expl = (BR_1 + BR_2)/2 in payoff
 * units, with br1/br2 the best-response values and value_avg player 1's value of the average
 * profile, all computed in FP64 on the device by a level-synchronous best response over the
 * compiled arrays.  Synchronises `stream`.  Any output pointer may be NULL.  CFR_EINVAL on a
 * handle holding several games (use cfr_batch_exploitability). */
cfr_status cfr_exploitability(cfr_handle *h, void *stream, double *expl, double *br1, double *br2,
                              double *value_avg);

/* Zero regrets, strategy sums and the iteration counter, reset sigma to uniform; nothing is
 * reallocated, so a captured graph stays valid (paper Appendix H, reset()).  Synchronous: waits
 * for all queued device work first. */
cfr_status cfr_reset(cfr_handle *h);

/* Copy regrets and strategy sums to host float64 arrays of `len` slots (either pointer may be
 * NULL), canonical order; FP32 regrets are widened exactly.  Synchronises `stream`. */
cfr_status cfr_get_state(cfr_handle *h, double *regrets, double *strategy_sum, int64_t len, void *stream);

/* Replace the cumulative regrets R (eq. regret) with r0[len] (canonical order; host or device pointer
 * per src_on_device) and recompute the current strategy from them by regret matching (eq. rm): a warm
 * start.  Strategy sums and the counter are left as they are (call cfr_reset first for a fresh solve);
 * under PCFR+ the prediction is cleared.  Host sources synchronise `stream`. */
cfr_status cfr_set_regrets(cfr_handle *h, const float *r0, int64_t len, int src_on_device, void *stream);

/* Checkpoint/resume: replace the solver state with host FP64 arrays of `len` slots in canonical order
 * -- cumulative regrets (eq. regret), strategy sums (eq. rm) and, under PCFR+, the prediction (the
 * previous iteration's instantaneous regret) -- and set the iteration counter to t (the next
 * iteration is t + 1, with that iteration's averaging weight and discounts).  Any array may be NULL:
 * regrets and sums are then left as they are, the prediction is cleared.  Values are rounded to the
 * state type; the current strategy is recomputed (eq. rm).  A state taken with cfr_get_state (and
 * cfr_get_prediction) after t iterations resumes the solve exactly.  CFR_EINVAL for a prediction
 * under another rule.  Synchronous. */
cfr_status cfr_set_state(cfr_handle *h, const double *regrets, const double *strategy_sum, const double *prediction,
                         int64_t len, int64_t t, void *stream);

/* PCFR+ prediction (the latest instantaneous regret) as host FP64 [len], canonical order; CFR_EINVAL
 * under another rule.  Synchronises `stream`. */
cfr_status cfr_get_prediction(cfr_handle *h, double *prediction, int64_t len, void *stream);

/* The state of one game of a batch: its cumulative regrets (eq. regret), strategy sums (eq. rm) and,
 * under PCFR+, prediction, as host FP64 arrays of len = the game's slot count, in that game's canonical
 * slot order (slots [slot_base[game], slot_base[game + 1]) of cfr_batch_size).  Only that game's slots
 * are copied.  Any pointer may be NULL; CFR_EINVAL for a game out of range, another len, or a
 * prediction under another rule.  Synchronises `stream`.  With cfr_set_state (and the batch's
 * iteration count) on a handle compiled from that game alone the game continues bitwise as it would in
 * the batch: a batch's last small games can move to the LDS-resident schedule. */
cfr_status cfr_get_game_state(cfr_handle *h, int32_t game, double *regrets, double *strategy_sum,
                              double *prediction, int64_t len, void *stream);

/* In-place re-solve (paper Appendix H, set_payoffs and set_root_chance; Table 'tab:lifecycle'):
 * rewrite the chance-folded template v_tmpl(z) = pi_c(z) u(z) of one game of the handle (game in
 * [0, n_games)) without reallocating anything, so a captured graph stays valid.  The solver state
 * (regrets, strategy sums, counter) is left alone: call cfr_reset for a fresh solve, or continue
 * from the previous solution.  Both need the handle compiled with options.lifecycle = 1
 * (CFR_ESTATE otherwise), wait for queued work on `stream` to read the host array and return
 * with the rewrite queued on `stream`.
 * cfr_set_payoffs: payoff[num_nodes] in the game description's node numbering (only terminal
 *   entries are read; finite), num_nodes as compiled.
 * cfr_set_root_chance: the root must be a chance node; prob[n] gives its children's probabilities
 *   in the description's child order (finite, >= 0, summing to 1 within 1e-9).  Terminals below
 *   child a get pi_c(z) = prob[a] * (the chance product below the root). */
cfr_status cfr_set_payoffs(cfr_handle *h, int32_t game, const double *payoff, int64_t num_nodes, void *stream);
cfr_status cfr_set_root_chance(cfr_handle *h, int32_t game, const double *prob, int64_t n, void *stream);

/* In-place re-solve with new root ranges (paper Appendix H, set_root_ranges; Table 'tab:lifecycle'):
 * for a game compiled with options.lifecycle = 1 whose description gave root_hand1/root_hand2, the
 * root chance becomes p(a) = r1[root_hand1[a]] r2[root_hand2[a]] / W with W the sum of those products
 * over the root's children in child order (the joint deal of the two private hands, restricted to the
 * dealt pairs), and the template is rewritten as by cfr_set_root_chance.  r1 [n1], r2 [n2]: host,
 * finite, >= 0, n1 = num_hands1 and n2 = num_hands2 of the description.  CFR_ESTATE without lifecycle
 * records or without the hand map; CFR_EINVAL if W is 0.  Returns with the rewrite queued on
 * `stream` (the host arrays are read before it returns). */
cfr_status cfr_set_root_ranges(cfr_handle *h, int32_t game, const double *r1, int64_t n1, const double *r2, int64_t n2,
                               void *stream);

/* Retire games of a batch, or bring them back (the batched form is not in the paper; its concluding
 * remarks motivate repeated subgame solves, and a solve stops once its subgame is good enough):
 * active[n] (host, n = the number of games) 0 retires a game.  cfr_iterate then launches only the
 * active games' update groups and chance nodes and the forward tiles that hold an active game (lists
 * built here; the iteration graphs are captured again on the next cfr_iterate), so a retired game's
 * state (regrets, strategy sums, strategy, values) stays as it was while the other games iterate,
 * bitwise as if it were not in the batch; the shared counter still advances, so a game brought back
 * continues with the current iteration's averaging weight.  cfr_profile's byte figures keep counting
 * every game.  Exploitability and strategies are still reported for every game.
 * Level-synchronous schedule only: CFR_EUNSUPPORTED under the persistent or LDS schedule, and
 * while a game is retired cfr_set_schedule to those, cfr_autotune and persistent iterations are
 * refused (CFR_ESTATE).  cfr_reset brings every game back.  A single game cannot be retired
 * (CFR_EUNSUPPORTED for active[0] = 0).  Synchronises the device (queued iterations read the lists
 * and graphs it replaces) and returns with the new lists in place; `stream` is waited for first. */
cfr_status cfr_set_active(cfr_handle *h, const uint8_t *active, int32_t n, void *stream);

/* Sizes and per-iteration launch count of a compiled game. */
cfr_status cfr_counts(cfr_handle *h, cfr_counts_t *out);

/* Per-kernel measurement.  Runs n iterations with direct launches on `stream`, recording a HIP
 * event before and after every launch, and reports for each kernel of the iteration body:
 *   name                  the kernel's symbol name (as profilers list it, without namespace)
 *   launches_per_iteration
 *   bytes_per_iteration   bytes of all its launches in one iteration under this design: each
 *                         index, state and value element the kernel reads or writes, counted once
 *   method_bytes_per_iteration
 *                         the method's per-unit byte figures (per edge, node, terminal, decision
 *                         node and edge, information set and slot, with 4-byte indices and the
 *                         state width) applied to the units its launches process
 *   ms_per_iteration      mean over the n iterations of the summed durations of its launches
 * The iterations advance the solver like cfr_iterate.  Writes up to max_out entries to out and
 * their number to *n_out.  Synchronises `stream`. */
typedef struct {
    char    name[32];
    int64_t launches_per_iteration;
    double  bytes_per_iteration;
    double  method_bytes_per_iteration;
    double  ms_per_iteration;
} cfr_kernel_stat;
cfr_status cfr_profile(cfr_handle *h, int64_t n, void *stream, cfr_kernel_stat *out, int32_t max_out,
                       int32_t *n_out);

/* Test hook: shift one persistent device pointer by `delta` elements (0 restores), so that
 * the rebinding guard can be exercised.  which: 0 regrets, 1 strategy sums, 2 strategy. */
cfr_status cfr_debug_rebind(cfr_handle *h, int which, int64_t delta);

/* Release the handle and all its device memory after the device has finished all queued work.
 * NULL is ignored. */
void cfr_destroy(cfr_handle *h);

/* Message of the last failed call on this thread ("" if none). */
const char *cfr_last_error(void);

/* ---- Learned warm start --------------------------------------------------------------------
 * Not part of the paper: a small network proposes initial regrets per information set, CFR+ runs
 * from them, and exact exploitability judges the result.  Zero initial regrets (the uniform
 * strategy, cfr_reset) remain the fallback, and sets with more than CFR_MLP_OUT actions always
 * start uniform.
 *
 * Network: x (in_dim bf16) -> n_hidden ReLU layers of `hidden` units -> CFR_MLP_OUT logits z.
 * Parameters form one flat float32 vector, layer by layer: W_l row-major [fan_in][fan_out], then
 * b_l [fan_out].  Hidden products run on the BF16 matrix cores with FP32 accumulation; bf16 are
 * stored: the rows, the weight copies, hidden activations and hidden pre-activation gradients.
 * Loss of a row with n legal actions (the first n outputs), target distribution t and weight w:
 *   p_a = softplus(z_a), q = p / sum_a p_a, CE = -sum_a t_a log q_a,  L = sum w CE / sum w.
 * Optimiser: Adam with bias correction on the FP32 master parameters.
 * Every reduction runs in a fixed order, so calls are bitwise reproducible. */
#define CFR_FEATURES 128
#define CFR_MLP_OUT 4
enum { CFR_MLP_PARAMS = 0, CFR_MLP_GRADS = 1, CFR_MLP_ADAM_M = 2, CFR_MLP_ADAM_V = 3 };

typedef struct cfr_mlp cfr_mlp;
typedef struct {
    int32_t in_dim;    /* 64, 128 or 256 (CFR_FEATURES for rows made by cfr_features) */
    int32_t hidden;    /* 64, 128 or 256 */
    int32_t n_hidden;  /* 1..4 */
    int32_t max_rows;  /* rows per training call and per inference chunk, 1..2^20 */
    int32_t device;
    float   beta1, beta2, eps;  /* Adam */
} cfr_mlp_desc;

/* 128 -> 3 x 256 -> 4, max_rows 4096, device 0, Adam 0.9 / 0.999 / 1e-8. */
void cfr_mlp_default_desc(cfr_mlp_desc *d);
/* Allocate a network (all device memory is owned by it); parameters start at zero. */
cfr_status cfr_mlp_create(const cfr_mlp_desc *d, cfr_mlp **out);
cfr_status cfr_mlp_num_params(cfr_mlp *n, int64_t *count);
/* Load the flat parameter vector from host memory; clears the Adam moments and step count.
 * Synchronous. */
cfr_status cfr_mlp_set_params(cfr_mlp *n, const float *params, int64_t len);
/* Copy a flat host vector out: CFR_MLP_PARAMS, CFR_MLP_GRADS (of the last backward call),
 * CFR_MLP_ADAM_M or CFR_MLP_ADAM_V.  Synchronous. */
cfr_status cfr_mlp_get(cfr_mlp *n, int which, float *dst, int64_t len);
/* Logits z[rows][4] (device, float32) of device rows x[rows][in_dim] (bf16), on `stream`.  Any
 * number of rows: one fused launch per 2^27 rows keeps each block's activations in LDS (no row limit,
 * no activation buffers), after a small launch that refreshes the network's transposed bf16 weight
 * copy; calls on one network that overlap on different streams (with each other or with training)
 * race on that copy and must be ordered by the caller. */
cfr_status cfr_mlp_forward(cfr_mlp *n, const void *x, int64_t rows, float *z, void *stream);
/* Loss and parameter gradients of one minibatch of rows <= max_rows, on `stream`.  Device
 * arrays: x [.][in_dim] bf16, target [.][4] float32 (entries past a row's legal actions are
 * ignored), weight [.] float32 or NULL (all 1), nact [.] legal actions per row (1..4; other values
 * are clamped).  With idx (device int32 [rows]) the minibatch is rows idx[r] of arrays holding
 * n_data rows (indices are clamped into range); without it, the first `rows` rows.  If loss is
 * not NULL the call synchronises `stream` and writes L there. */
cfr_status cfr_mlp_backward(cfr_mlp *n, const void *x, const float *target, const float *weight,
                            const uint8_t *nact, const int32_t *idx, int64_t n_data, int64_t rows, double *loss,
                            void *stream);
/* Logits bitwise equal to cfr_mlp_forward's (computed layer by layer, each hidden layer's activations
 * staged in device memory), for callers that
 * cannot allocate device memory: code under hipGraph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The call allocates nothing (no hipMalloc, hipFree or allocating library call):
 * the hidden activations go to one static device array of 2 x 8192 x 256 bf16 (8 MiB) that each GPU
 * the library runs on holds until the process ends; its device address is looked up on the first
 * call on a device.  rows <= 8192 (CFR_EINVAL beyond; cfr_mlp_forward has no such limit), the network's
 * hidden width <= 256.  Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other threads, other networks) race and must be serialised by the caller; each call
 * writes the activations it reads, so nothing has to be cleared between calls.  x, z as for
 * cfr_mlp_forward; enqueued on `stream`. */
cfr_status cfr_mlp_forward_noalloc(cfr_mlp *n, const void *x, int64_t rows, float *z, void *stream);
/* One Adam step with learning rate lr on the gradients of the last backward call. */
cfr_status cfr_mlp_adam(cfr_mlp *n, float lr, void *stream);
/* cfr_mlp_backward followed by cfr_mlp_adam. */
cfr_status cfr_mlp_train_step(cfr_mlp *n, const void *x, const float *target, const float *weight,
                              const uint8_t *nact, const int32_t *idx, int64_t n_data, int64_t rows, float lr,
                              double *loss, void *stream);
/* Release the network after the device has finished queued work; NULL is ignored. */
void cfr_mlp_destroy(cfr_mlp *n);

/* Number of information sets of the handle (rows of cfr_features: every game's sets in canonical
 * order, games in order). */
cfr_status cfr_num_infosets(cfr_handle *h, int64_t *count);
/* Feature rows of every information set into x[rows][CFR_FEATURES] (device, bf16), on `stream`:
 *   0-63    one-hot bucket[i] (device int16; values outside 0..63: none)
 *   64-95   one-hot history[i] (device int16; values outside 0..31: none)
 *   96-103  scalars[i][0..7] (device float32)
 *   104-107 legal-action mask (first min(n, 4) actions)
 *   108-111 the instantaneous regrets of the uniform strategy (eq. instregret at sigma uniform)
 *           of the first four actions over the sum of their magnitudes (0 for sets of > 4 actions)
 *   112-115 regret matching (plus) of those regrets
 *   116     acting player (0 for player 1, 1 for player 2); 117-119 zero
 *   120-123 the current strategy after the probe (first four actions; uniform without a probe)
 *   124-127 the normalised average strategy after the probe (uniform without a probe or sum 0)
 *   (120-127 are zero for sets of more than four actions.)
 * The regrets of 108-115 come from one plain (unclamped, uniformly weighted) iteration from zero
 * regrets, after which the handle is reset (regrets, strategy sums and counter zero, as after
 * cfr_reset).  It also records m(I), the sum of the magnitudes of those (up to four) regrets, for
 * cfr_warm_start.  Then, if probe_iters > 0, it runs the first probe_iters iterations of the solve
 * (as cfr_iterate) and leaves the handle there: a warm start then continues from iteration
 * probe_iters with the strategy sums of the probe.  rows must equal cfr_num_infosets. */
cfr_status cfr_features(cfr_handle *h, const int16_t *bucket, const int16_t *history, const float *scalars,
                        int32_t probe_iters, void *x, int64_t rows, void *stream);
/* m(I) of every information set (rows floats, device), as recorded by the last cfr_features call
 * (CFR_ESTATE if there was none), on `stream`. */
cfr_status cfr_regret_unit(cfr_handle *h, float *unit, int64_t rows, void *stream);
/* Warm start: run the network on rows x (as made by cfr_features) and set the cumulative regrets
 * to scale * m(I) * softplus(z) for the legal actions of every set with at most 4 actions, 0 for
 * larger sets (add = 0; this also clears the PCFR+ prediction), or add that to the current
 * regrets (add = 1, keeping whatever a probe accumulated), then recompute the current strategy.  m(I) is the sum of
 * the magnitudes of the set's instantaneous regrets under the uniform strategy, recorded by the
 * last cfr_features call (CFR_ESTATE if there was none), so scale counts iterations' worth of
 * regret.  Strategy sums and the counter are left as they are.  scale = 0 gives the uniform start. */
cfr_status cfr_warm_start(cfr_handle *h, cfr_mlp *n, const void *x, int64_t rows, float scale, int32_t add,
                          void *stream);


#ifdef __cplusplus
}
#endif
#endif
