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
};

// Validate and compile.  Returns CFR_OK or CFR_EINVAL / CFR_ENOMEM with a message in err.
cfr_status build_layout(const cfr_game_desc *g, Layout &out, std::string &err);

}  // namespace cfrx
