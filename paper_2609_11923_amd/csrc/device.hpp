// device.hpp -- device-side data of a compiled game and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/cfr.h"

namespace cfrx {

// Edge code stored with every node for the edge into it:
//   bits 0-1  owner of the parent (0 chance / root, 1 player 1, 2 player 2)
//   bit  2    the node is internal (has children); terminals carry no reach
//   bits 3-30 slot of the edge (decision parents only)
constexpr int CODE_OWNER_MASK = 3;
constexpr int CODE_INTERNAL = 4;
constexpr int CODE_SLOT_SHIFT = 3;
// Member-list entries: node id in bits 0-30, bit 31 set when the set belongs to player 2;
// paired with the node's first edge so that no edge-offset lookup sits on the load chain.
constexpr int32_t MEMBER_NODE_MASK = 0x7fffffff;
constexpr int32_t MEMBER_P2 = (int32_t)0x80000000u;
// fields per (game, depth) in game_range: node lo/hi, group lo/hi, chance lo/hi, big chance lo/hi
constexpr int GR_FIELDS_DEV = 8;
// bound on one barrier wait, in seconds of the device's constant-rate clock: a stuck wait raises
// the error flag (the launch then reports CFR_EDEVICE) instead of hanging.  A count of polls is no
// time bound: under contention one acquire poll can take microseconds.
constexpr double BARRIER_TIMEOUT_S = 2.0;
// DCFR's published constants (the paper names the rule but not its constants)
constexpr double DCFR_ALPHA = 1.5, DCFR_BETA = 0.0, DCFR_GAMMA = 2.0;

struct DevGame {
    int32_t N = 0, I = 0, A = 0, Ndec = 0, max_depth = 0, max_actions = 0;
    int fp64 = 0;                 // state type: 0 float (paper's configured dtype), 1 double
    int rule = 0;                 // CFR_RULE_* (selects the update's instantiation)
    // structure (read-only after compile)
    int explicit_kids = 0;        // 1: child a of n is kid[kid_off[n] + a]; 0: it is kid_off[n] + a
    int2 *up = nullptr;           // [N]   (parent, edge code)
    int32_t *kid_off = nullptr;   // [N+1] edges of n are [kid_off[n], kid_off[n+1])
    int32_t *kid = nullptr;       // [E]   child of each edge (explicit layouts only)
    // affine layouts (explicit, and child a of every member h of a set is h + koff[slot a]): the
    // update pass reads the per-slot offsets and a compact member list instead of kid[] and mem[]
    int affine = 0;
    int32_t group_sets = 256;     // sets per update group (128 or 256): sizes the affine update's LDS rows
    int32_t *koff = nullptr;      // [A]   child offset of each slot (affine only)
    // member node | MEMBER_P2 bit, per update group in set-major order, or in node order where that
    // touches far fewer cache lines (grp_perm[g] = 1; mpos then gives each member's set-major position
    // in its group) (affine only)
    int32_t *mnode = nullptr;     // [Ndec]
    uint16_t *mpos = nullptr;     // [Ndec]
    int8_t *grp_perm = nullptr;   // [G]
    int32_t *slot_map = nullptr;  // [A]   canonical slot -> device slot (nullptr: identity)
    int32_t *node_slot = nullptr; // [N]   first slot of a decision node, -1 otherwise
    int32_t *node_iset = nullptr; // [N]   information set of a decision node, -1 otherwise
    int32_t *slot_off = nullptr;  // [I+1]
    int32_t *mem_off = nullptr;   // [I+1]
    int2 *mem = nullptr;          // [Ndec]  members: (node | MEMBER_P2 bit, first edge of the node)
    int8_t *iset_player = nullptr;// [I]
    int32_t G = 0;                // update groups
    int32_t *grp_iset_off = nullptr; // [G+1]
    // host copies of per-depth ranges (launch parameters)
    const int32_t *grp_depth_off = nullptr;  // [max_depth+2] groups of depth d
    const int32_t *chance_off = nullptr;     // [max_depth+2] chance nodes of depth d
    int32_t *chance_node = nullptr;          // device: internal chance nodes by depth (small fan-out)
    const int32_t *bigc_off = nullptr;       // [max_depth+2] big-fan-out chance nodes of depth d
    int32_t *bigc_node = nullptr;            // device: chance nodes with fan-out above BIG_FANOUT
    // batches with retired games (cfr_set_active): the work that still runs, per depth -- forward
    // tiles (index within the depth's tiles), update groups, chance nodes and big chance nodes --
    // listed on the device at [off[d], off[d] + cnt[d]) of each list (host offsets and counts);
    // use_lists = 0 while every game iterates (the identity)
    int use_lists = 0;
    int32_t *fwd_list = nullptr, *grp_list = nullptr, *chance_list = nullptr, *bigc_list = nullptr;
    const int64_t *fwd_off = nullptr, *grp_off = nullptr, *chance_off_l = nullptr, *bigc_off_l = nullptr;
    // iteration state, element type float or double (fp64)
    void *v = nullptr;            // [N]   player-1 chance-weighted values; terminals hold the template
    void *reach = nullptr;        // [2N]  lane 0: player 1 reach, lane 1: player 2 reach
    void *sigma = nullptr;        // [A]   current strategy
    void *R = nullptr;            // [A]   cumulative regrets
    void *pred = nullptr;         // [A]   PCFR+ prediction (the latest instantaneous regret), else nullptr
    double *sbar = nullptr;       // [A]   strategy sums (FP64)
    int32_t *t = nullptr;         // [1]   iterations started (device counter)
    // evaluation scratch (best response, FP64)
    double *vbr = nullptr;        // [N]   terminals hold pi_c(z) u(z) in double
    double *qbr = nullptr;        // [N]   opponent reach of the best responder
    double *sigbar = nullptr;     // [A]   normalised average strategy
    int32_t *astar = nullptr;     // [I]   best-response action
    float *out = nullptr;         // [A]   staging for strategy output (canonical order)
    float *out2 = nullptr;        // [A]   staging in device order
};

struct IterFlags {
    int rule;     // CFR_RULE_*
    int linear;   // w_t = t (CFR and CFR+)
    int upd;      // players whose sets a level updates: bit 0 player 1, bit 1 player 2
};

// one level of the forward reach pass: nodes [lo, hi) of one depth; tick != nullptr bumps the counter
hipError_t launch_forward(const DevGame &g, int d, int32_t lo, int32_t hi, int32_t *tick, hipStream_t s);
// one level of the backward value pass fused with the update of the information sets on it
// (regrets, clamp, average, regret matching of the next strategy)
hipError_t launch_level(const DevGame &g, int d, IterFlags f, hipStream_t s);
// sigma <- regret matching of R (all information sets)
hipError_t launch_regret_matching(const DevGame &g, hipStream_t s);
// The persistent batched launch: tickets (one int4 per rank: game, rank, workgroups of the game),
// queue by queue (one queue per XCD, q_off [PERSISTENT_QUEUES + 1]), per-game level ranges and depths,
// barrier counters [n_games] followed by the queues' claim counters [PERSISTENT_QUEUES], and the
// time-out flag (all device memory).
constexpr int PERSISTENT_QUEUES = 8;
struct PersistentPlan {
    int32_t blocks = 0, n_games = 0, max_depth = 0, n_tickets = 0, wg_nodes = 0, max_W = 0;
    int4 *tickets = nullptr;
    int32_t *q_off = nullptr, *claim = nullptr;
    int32_t *game_range = nullptr, *game_depth = nullptr, *barrier = nullptr, *err = nullptr;
    int64_t timeout_ticks = 0;   // BARRIER_TIMEOUT_S in ticks of wall_clock64()
};
// zero the barrier and claim counters, run T iterations of every game in one launch (both halves of
// each iteration when alternating), advance the counter by T
hipError_t launch_persistent(const DevGame &g, const PersistentPlan &p, int32_t T, IterFlags f, int alternating,
                             hipStream_t s);
// resident blocks per compute unit of the persistent kernel for this game's configuration
hipError_t persistent_occupancy(const DevGame &g, int *blocks_per_cu);
// The LDS-resident schedule of a single tiny game: one workgroup runs T iterations (both halves
// when alternating) with the whole state in LDS, then the counter advances by T.  game_range is the
// game's per-depth range table on the device.  lds_schedule_bytes is the dynamic LDS it needs;
// prepare_lds raises the kernel's limit to it (once, before launches or capture) and fails for
// more than 16 actions per set.
size_t lds_schedule_bytes(int32_t N, int32_t A, int fp64, int pred);
hipError_t prepare_lds(const DevGame &g, int rule, size_t *bytes);
hipError_t launch_lds(const DevGame &g, const int32_t *game_range, int32_t T, IterFlags f, int alternating,
                      hipStream_t s);
// counter bump for games without edges
hipError_t launch_tick(const DevGame &g, hipStream_t s);
// out2[q] <- normalised average strategy (float, device order), sigbar[q] <- same in double
hipError_t launch_average(const DevGame &g, hipStream_t s);
// out-of-band conversions between device slot order and canonical order:
// dst[q] <- sigma[map q] as float; dst[q] <- src[map q]; R[map q] <- src[q]
hipError_t launch_sigma_to_float(const DevGame &g, float *dst, hipStream_t s);
hipError_t launch_gather_float(const DevGame &g, const float *src, float *dst, hipStream_t s);
hipError_t launch_regrets_from_float(const DevGame &g, const float *src, hipStream_t s);
// R[map q] += src[q] (canonical float source)
hipError_t launch_regrets_add_float(const DevGame &g, const float *src, hipStream_t s);
// dst[map q] <- src[q] for a canonical FP64 source, into the state type (state_type) or into FP64
hipError_t launch_scatter_double(const DevGame &g, const double *src, void *dst, bool state_type, hipStream_t s);
// zero A slots of the state type
hipError_t launch_fill_state(const DevGame &g, void *dst, hipStream_t s);
// in-place re-solve: u[j] <- payoff_in[in[j]] for records [lo, hi); then the template of those
// terminals: v = vbr = (root ? root[branch] * pic : pic) * u
hipError_t launch_gather_payoffs(int64_t lo, int64_t hi, const int32_t *in, const double *payoff_in, double *u,
                                 hipStream_t s);
hipError_t launch_template(const DevGame &g, int64_t lo, int64_t hi, const int32_t *node, const int32_t *branch,
                           const double *u, const double *pic, const double *root, hipStream_t s);
// best response pieces (FP64); br = 1 or 2 selects the best responder, 0 evaluates the average profile
hipError_t launch_br_forward(const DevGame &g, int32_t lo, int32_t hi, int br, hipStream_t s);
hipError_t launch_br_argmax(const DevGame &g, int32_t ilo, int32_t ihi, int br, hipStream_t s);
hipError_t launch_br_backward(const DevGame &g, int32_t lo, int32_t hi, int br, hipStream_t s);

}  // namespace cfrx
