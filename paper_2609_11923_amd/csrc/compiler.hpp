// compiler.hpp -- host-side game compiler (paper Appendix H, Algorithm 'alg:compile').
//
// Turns an explicit game specification into the canonical compiled arrays:
// breadth-first node numbering (parent before child, children in action
// order, hence sorted by depth), depth offsets, parent and child CSR,
// information sets numbered by first occurrence, slot offsets, member lists,
// and the chance-folded values template v_tmpl(z) = pi_c(z) u(z) (eq.
// template).  No device code lives here.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cfr.h"

namespace cfrx {

struct Layout {
    int64_t N = 0, E = 0, Z = 0, Ndec = 0, I = 0, A = 0;
    int max_depth = 0, D = 0, max_actions = 0;
    bool br_ok = true;                   // every information set lies on one depth
    std::vector<int32_t> depth_off;      // [max_depth + 2]
    std::vector<int32_t> parent;         // [N]
    std::vector<int32_t> child_off;      // [N + 1]
    std::vector<int32_t> in_slot;        // [N]
    std::vector<int32_t> node_infoset;   // [N]
    std::vector<int8_t> node_type;       // [N]
    std::vector<float> tmpl;             // [N]
    std::vector<double> tmpl64;          // [N] pi_c(z) u(z) in double
    std::vector<int32_t> slot_off;       // [I + 1]
    std::vector<int32_t> mem_off;        // [I + 1]
    std::vector<int32_t> mem_node;       // [Ndec]
    std::vector<int8_t> iset_player;     // [I]
    std::vector<int64_t> iset_key;       // [I]
    std::vector<int32_t> iset_depth_off; // [max_depth + 2] infosets whose members sit at depth d
    std::vector<int64_t> public_key;     // [N] canonical order, empty if not given
    // set before build_layout to keep the canonical -> input node map (in-place re-solve support)
    bool keep_maps = false;
    std::vector<int32_t> input_id;       // [N] input node id of canonical node k (keep_maps only)
};

// Validate and compile.  Returns CFR_OK or CFR_EINVAL / CFR_ENOMEM with a message in err.
cfr_status build_layout(const cfr_game_desc *g, Layout &out, std::string &err);

// Sets per update group: at most the 256-thread block (one thread per set).  A game (or batch) uses
// a bound of 128 or 256 (DeviceLayout::group_sets); the affine update sizes its per-set LDS rows by
// it, so the smaller bound leaves room for more resident blocks.
constexpr int GROUP_SETS_MAX = 256;

// The node order the kernels run on.  Depth ranges are those of the canonical layout; inside
// each depth the nodes are permuted:
//   BFS     canonical order (children of a node are consecutive ids, so child lists stay
//           implicit: child a of h is kid_off[h] + a)
//   PUBLIC  decision nodes first, then chance nodes, then terminals; each part grouped by public
//           state (states ranked by first occurrence in canonical order), canonical order inside
//           a group.
//           Members of an information set then sit in one public-state block, children of a
//           block's nodes sit in the child states' blocks at the same rank, and every write of
//           a level pass lands in one dense range.  Child lists are explicit (kid[]).
// Information sets are renumbered by first member in device order (hence depth-sorted) and
// slots follow them; slot_canon_to_dev maps the canonical slot numbering of the ABI.
struct DeviceLayout {
    bool explicit_kids = false;
    std::vector<int32_t> depth_off;      // [max_depth + 2]
    std::vector<int32_t> int_end;        // [max_depth + 1] internal nodes of depth d: [depth_off[d], int_end[d])
    std::vector<int32_t> up_parent;      // [N] parent (device id), -1 at the root
    std::vector<int32_t> up_code;        // [N] edge code (see device.hpp), slot in device numbering
    std::vector<int32_t> kid_off;        // [N + 1]
    std::vector<int32_t> kid;            // [E] when explicit_kids
    std::vector<int32_t> node_slot;      // [N] first device slot of a decision node, -1 otherwise
    std::vector<int32_t> node_iset;      // [N] device information set, -1 otherwise
    std::vector<int32_t> slot_off, mem_off, mem_node;
    std::vector<int8_t> iset_player;
    std::vector<int32_t> iset_depth_off; // [max_depth + 2]
    std::vector<float> tmpl;             // [N]
    std::vector<double> tmpl64;          // [N]
    std::vector<int32_t> slot_canon_to_dev; // [A], empty when identical
    std::vector<int32_t> node_dev;       // [N] device id of canonical node k (Layout::keep_maps only)
    // update groups: runs of consecutive information sets of one depth with at most group_cap
    // members and at most group_sets sets in total (a set with more members forms a group of its
    // own); group g holds sets [grp_iset_off[g], grp_iset_off[g + 1]); the groups of depth d are
    // [grp_depth_off[d], grp_depth_off[d + 1])
    std::vector<int32_t> grp_iset_off;
    std::vector<int32_t> grp_depth_off;  // [max_depth + 2]
    int32_t group_cap = 0;               // members per group (group_members)
    int32_t group_sets = GROUP_SETS_MAX; // sets per group, 128 or 256
    int64_t groups_by_bound[2] = {0, 0}; // groups this layout forms with at most 128 / 256 sets
    // internal chance nodes by depth: chance_node[chance_off[d] .. chance_off[d + 1]) for fan-out
    // <= BIG_FANOUT (one thread each), bigc_node[bigc_off[d] .. bigc_off[d + 1]) above it (one
    // workgroup each)
    std::vector<int32_t> chance_node;
    std::vector<int32_t> chance_off;     // [max_depth + 2]
    std::vector<int32_t> bigc_node;
    std::vector<int32_t> bigc_off;       // [max_depth + 2]
    // forests (batches of independent games, depth-major: the depth-d nodes of game 0, then of
    // game 1, ...; likewise information sets, slots, groups and chance nodes)
    int32_t n_games = 1;
    std::vector<int32_t> game_root;      // [n] forest id of each game's root (= its index)
    std::vector<int64_t> game_slot_base; // [n + 1] offsets of each game's canonical slots at the ABI
    std::vector<int32_t> game_depth;     // [n] max depth of each game
    // per game and depth d (stride GR_FIELDS): node, group, chance-node and big-chance-node ranges
    std::vector<int32_t> game_range;     // [n * (max_depth + 1) * GR_FIELDS]
};

constexpr int GR_FIELDS = 8;  // node lo/hi, group lo/hi, chance lo/hi, big chance lo/hi
constexpr int BIG_FANOUT = 64;

// members per update group (members per thread times the 256-thread block): with at most 4 actions
// per set four per thread for FP32 state and two for FP64 (whose LDS staging is twice as large),
// else one.  The update kernels' members per thread must match.
inline int group_members(int max_actions, bool fp64) { return max_actions <= 4 ? (fp64 ? 512 : 1024) : 256; }

// group_actions: the action bound the update groups are sized for (>= L.max_actions); fp64: the state
// type of the kernels, which sets the group capacity (group_members); group_sets: the set bound of the
// update groups, 128 or 256, or 0 to choose it from this game alone (choose_group_sets)
cfr_status build_device_layout(const Layout &L, int layout_kind, int group_actions, bool fp64, int group_sets,
                               DeviceLayout &out, std::string &err);

// (Re)form D's update groups with at most D.group_cap members and `sets` sets each, runs of consecutive
// information sets of one depth (a set with more members forms a group of its own); also refreshes
// the group fields of a single game's range table.  Counts for both bounds are in D.groups_by_bound.
cfr_status set_update_groups(DeviceLayout &D, int32_t sets, std::string &err);

// The set bound for update groups that number g128 with at most 128 sets and g256 with at most 256:
// 128 unless it splits groups that the member capacity alone would keep whole (more than 30 % more
// groups).  Measured on the large card game (FP32 state): with about 8 members per set 128 is 4 %
// faster per iteration (6 resident blocks per compute unit instead of 5), with 6.2 members per set
// (29 % more groups) 1 % faster, with 4.4 (81 % more groups) 4 % slower and with 3.3 7 % slower.
inline int32_t choose_group_sets(int64_t g128, int64_t g256) { return g128 * 10 <= g256 * 13 ? 128 : GROUP_SETS_MAX; }

// Affine children: in an explicit layout, when every member h of every information set reaches its
// child under action a at h + koff[slot a] (one offset per slot, shared by the set's members), fill
// koff [A] and return true; otherwise return false (koff cleared).  Public-state layouts of card
// games have this property: the members of a set lie in one public-state block and the child
// block of an action keeps the block's node order.
bool slot_child_offsets(const DeviceLayout &D, std::vector<int32_t> &koff);

// Work plan of the persistent schedule.  Game g gets W_g = max(1, ceil(nodes_g / wg_nodes)) workgroups
// ("ranks"); games are placed largest first on the least loaded of n_queues queues (one per XCD) and a
// game's ranks are consecutive tickets of its queue.  Workgroups claim tickets in order at run time, so
// the ranks of a game are claimed by running workgroups one after another and a game's per-level
// barrier waits only for workgroups that have started: what must fit on the device at once is one
// game's W_g workgroups (not the whole grid).  wg_nodes is doubled until every W_g <= max_w.
struct PersistentWork {
    int32_t wg_nodes = 0;                 // target nodes per workgroup used
    int32_t max_W = 0;                    // largest W_g
    std::vector<int32_t> W;               // [n] workgroups of each game
    std::vector<int32_t> queue;           // [n] queue of each game
    std::vector<int32_t> q_off;           // [n_queues + 1] tickets of queue q are [q_off[q], q_off[q + 1])
    std::vector<int32_t> ticket;          // [tickets * 3]: game, rank, W_g of each ticket, queue by queue
    std::vector<int64_t> load;            // [n_queues] nodes per queue
};
bool plan_persistent(const std::vector<int64_t> &nodes, int32_t wg_nodes, int32_t max_w, int n_queues,
                     PersistentWork &out, std::string &err);

// Merge the device layouts of independent games into one depth-major forest (see DeviceLayout).
// Ls and Ds are consumed (moved or cleared).  A single game is moved through unchanged.
cfr_status build_forest(std::vector<Layout> &Ls, std::vector<DeviceLayout> &Ds, DeviceLayout &F, std::string &err);

}  // namespace cfrx
