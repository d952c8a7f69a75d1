// compiler.cpp -- host-side game compiler (paper Appendix H, Algorithm 'alg:compile',
// passes 1-7: validate, slots, node arrays, edge arrays, depth schedule, chance
// folding, index emission).  See compiler.hpp for the produced arrays.
#include "compiler.hpp"

#include <cmath>
#include <cstring>
#include <algorithm>
#include <new>

namespace cfrx {
namespace {

inline uint64_t mix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// open-addressing map int64 key -> int32 index
struct KeyMap {
    std::vector<int64_t> keys;
    std::vector<int32_t> vals;
    uint64_t mask = 0;
    explicit KeyMap(int64_t expect) {
        uint64_t cap = 16;
        while (cap < (uint64_t)expect * 2 + 16) cap <<= 1;
        keys.assign(cap, 0);
        vals.assign(cap, -1);
        mask = cap - 1;
    }
    // returns existing index, or inserts `fresh` and returns it
    int32_t find_or_insert(int64_t key, int32_t fresh) {
        uint64_t h = mix((uint64_t)key) & mask;
        for (;;) {
            if (vals[h] < 0) { keys[h] = key; vals[h] = fresh; return fresh; }
            if (keys[h] == key) return vals[h];
            h = (h + 1) & mask;
        }
    }
};

}  // namespace

cfr_status build_layout(const cfr_game_desc *g, Layout &L, std::string &err) {
    try {
        if (!g) { err = "game description is NULL"; return CFR_EINVAL; }
        const int64_t N = g->num_nodes;
        if (N <= 0 || N > 0x7fffffffLL) { err = "num_nodes must be in [1, 2^31)"; return CFR_EINVAL; }
        if (g->root < 0 || g->root >= N) { err = "root out of range"; return CFR_EINVAL; }
        if (!g->node_type || !g->child_begin || !g->num_children || !g->payoff || !g->infoset_key) {
            err = "missing node array"; return CFR_EINVAL;
        }
        if (!(g->pot > 0.0)) { err = "pot must be > 0"; return CFR_EINVAL; }
        int64_t E = 0;
        for (int64_t n = 0; n < N; n++) {
            int t = g->node_type[n];
            int32_t k = g->num_children[n];
            if (t < 0 || t > 3) { err = "invalid node type at node " + std::to_string(n); return CFR_EINVAL; }
            if (k < 0) { err = "negative child count"; return CFR_EINVAL; }
            if (t == CFR_NODE_TERMINAL && k != 0) { err = "terminal node with children"; return CFR_EINVAL; }
            if (t != CFR_NODE_TERMINAL && k == 0) { err = "non-terminal node without children"; return CFR_EINVAL; }
            if ((t == CFR_NODE_P1 || t == CFR_NODE_P2) && k > 64) {
                err = "decision node with more than 64 actions"; return CFR_EINVAL;
            }
            E += k;
        }
        if (E > 0 && !g->children) { err = "children array is NULL"; return CFR_EINVAL; }
        for (int64_t n = 0; n < N; n++) {
            int32_t k = g->num_children[n];
            if (k == 0) continue;
            if (g->child_begin[n] < 0) { err = "negative child_begin"; return CFR_EINVAL; }
            for (int32_t a = 0; a < k; a++) {
                int64_t c = g->children[g->child_begin[n] + a];
                if (c < 0 || c >= N) { err = "child id out of range"; return CFR_EINVAL; }
            }
            if (g->node_type[n] == CFR_NODE_CHANCE) {
                if (!g->chance_prob) { err = "chance_prob array is NULL"; return CFR_EINVAL; }
                double s = 0.0;
                for (int32_t a = 0; a < k; a++) {
                    double p = g->chance_prob[g->child_begin[n] + a];
                    if (!(p >= 0.0) || !std::isfinite(p)) { err = "invalid chance probability"; return CFR_EINVAL; }
                    s += p;
                }
                if (std::fabs(s - 1.0) > 1e-9) { err = "chance probabilities do not sum to 1"; return CFR_EINVAL; }
            }
        }
        // ---- pass 3/5: breadth-first numbering (parent before child) and depths
        std::vector<int32_t> canon((size_t)N, -1);
        std::vector<int32_t> order((size_t)N);
        std::vector<int32_t> depth((size_t)N);
        int64_t tail = 0;
        order[tail++] = (int32_t)g->root;
        canon[g->root] = 0;
        depth[0] = 0;
        int max_depth = 0;
        for (int64_t k = 0; k < tail; k++) {
            int64_t h = order[k];
            int32_t nk = g->num_children[h];
            for (int32_t a = 0; a < nk; a++) {
                int64_t c = g->children[g->child_begin[h] + a];
                if (canon[c] >= 0) { err = "not a tree: node " + std::to_string(c) + " reached twice"; return CFR_EINVAL; }
                canon[c] = (int32_t)tail;
                depth[tail] = depth[k] + 1;
                if (depth[tail] > max_depth) max_depth = depth[tail];
                order[tail++] = (int32_t)c;
            }
        }
        if (tail != N) { err = "not a tree: " + std::to_string(N - tail) + " node(s) unreachable from the root"; return CFR_EINVAL; }
        L.N = N; L.E = E; L.max_depth = max_depth; L.D = N > 1 ? max_depth : 0;
        L.depth_off.assign((size_t)max_depth + 2, 0);
        for (int64_t k = 0; k < N; k++) L.depth_off[depth[k] + 1]++;
        for (int d = 0; d <= max_depth; d++) L.depth_off[d + 1] += L.depth_off[d];
        // ---- pass 2: information sets by first occurrence, slots
        L.node_type.resize((size_t)N);
        L.node_infoset.assign((size_t)N, -1);
        std::vector<int32_t> iset_nA, iset_depth;
        KeyMap km(1024);
        {
            int64_t ndec = 0;
            for (int64_t n = 0; n < N; n++) ndec += (g->node_type[n] == CFR_NODE_P1 || g->node_type[n] == CFR_NODE_P2);
            km = KeyMap(ndec);
        }
        int64_t Z = 0, Ndec = 0;
        int max_actions = 0;
        for (int64_t k = 0; k < N; k++) {
            int64_t h = order[k];
            int t = g->node_type[h];
            L.node_type[k] = (int8_t)t;
            if (t == CFR_NODE_TERMINAL) { Z++; continue; }
            if (t == CFR_NODE_CHANCE) continue;
            Ndec++;
            int32_t nk = g->num_children[h];
            if (nk > max_actions) max_actions = nk;
            int32_t fresh = (int32_t)L.iset_player.size();
            int32_t idx = km.find_or_insert(g->infoset_key[h], fresh);
            if (idx == fresh) {
                L.iset_player.push_back((int8_t)t);
                L.iset_key.push_back(g->infoset_key[h]);
                iset_nA.push_back(nk);
                iset_depth.push_back(depth[k]);
            } else {
                if (L.iset_player[idx] != t) { err = "information set spans players (key " + std::to_string(g->infoset_key[h]) + ")"; return CFR_EINVAL; }
                if (iset_nA[idx] != nk) { err = "information set members differ in action count (key " + std::to_string(g->infoset_key[h]) + ")"; return CFR_EINVAL; }
                if (iset_depth[idx] != depth[k]) L.br_ok = false;
            }
            L.node_infoset[k] = idx;
        }
        const int64_t I = (int64_t)L.iset_player.size();
        L.I = I; L.Z = Z; L.Ndec = Ndec; L.max_actions = max_actions;
        L.slot_off.assign((size_t)I + 1, 0);
        for (int64_t i = 0; i < I; i++) L.slot_off[i + 1] = L.slot_off[i] + iset_nA[i];
        L.A = L.slot_off[I];
        if (L.A > (1LL << 28)) { err = "more than 2^28 information-set actions"; return CFR_EINVAL; }
        if (L.keep_maps) L.input_id = order;
        // ---- pass 4/6: edge arrays in canonical numbering, chance folding, perfect recall
        L.parent.assign((size_t)N, -1);
        L.child_off.assign((size_t)N + 1, 0);
        L.in_slot.assign((size_t)N, -1);
        L.tmpl.assign((size_t)N, 0.0f);
        L.tmpl64.assign((size_t)N, 0.0);
        std::vector<double> pic((size_t)N);
        std::vector<uint64_t> seq1((size_t)N), seq2((size_t)N);
        std::vector<uint64_t> iset_seq((size_t)I, 0);
        std::vector<uint8_t> iset_seen((size_t)I, 0);
        pic[0] = 1.0; seq1[0] = 0; seq2[0] = 0;
        int32_t next = 1;
        for (int64_t k = 0; k < N; k++) {
            int64_t h = order[k];
            int t = L.node_type[k];
            L.child_off[k] = next;
            int32_t nk = g->num_children[h];
            int32_t I_h = L.node_infoset[k];
            if (I_h >= 0) {
                uint64_t own = t == CFR_NODE_P1 ? seq1[k] : seq2[k];
                if (!iset_seen[I_h]) { iset_seen[I_h] = 1; iset_seq[I_h] = own; }
                else if (iset_seq[I_h] != own) {
                    err = "not perfect recall: members of information set (key " + std::to_string(L.iset_key[I_h]) +
                          ") have different own-action histories";
                    return CFR_EINVAL;
                }
            }
            for (int32_t a = 0; a < nk; a++) {
                int32_t ck = next++;
                L.parent[ck] = (int32_t)k;
                seq1[ck] = seq1[k]; seq2[ck] = seq2[k];
                if (t == CFR_NODE_CHANCE) {
                    pic[ck] = pic[k] * g->chance_prob[g->child_begin[h] + a];
                } else {
                    pic[ck] = pic[k];
                    int32_t q = L.slot_off[I_h] + a;
                    L.in_slot[ck] = q;
                    uint64_t &s = t == CFR_NODE_P1 ? seq1[ck] : seq2[ck];
                    s = mix(s ^ ((uint64_t)q + 1) * 0x100000001B3ull);
                }
            }
            if (t == CFR_NODE_TERMINAL) {
                double v = pic[k] * g->payoff[h];
                L.tmpl64[k] = v;
                L.tmpl[k] = (float)v;
            }
        }
        L.child_off[N] = next;
        // ---- pass 7: member lists (ascending canonical id) and per-depth infoset ranges
        L.mem_off.assign((size_t)I + 1, 0);
        for (int64_t k = 0; k < N; k++) if (L.node_infoset[k] >= 0) L.mem_off[L.node_infoset[k] + 1]++;
        for (int64_t i = 0; i < I; i++) L.mem_off[i + 1] += L.mem_off[i];
        L.mem_node.assign((size_t)Ndec, 0);
        {
            std::vector<int32_t> fill(L.mem_off.begin(), L.mem_off.end() - 1);
            for (int64_t k = 0; k < N; k++) {
                int32_t i = L.node_infoset[k];
                if (i >= 0) L.mem_node[fill[i]++] = (int32_t)k;
            }
        }
        L.iset_depth_off.assign((size_t)max_depth + 2, (int32_t)I);
        {
            int32_t i = 0;
            for (int d = 0; d <= max_depth + 1; d++) {
                while (i < I && iset_depth[i] < d) i++;
                L.iset_depth_off[d] = i;
            }
        }
        if (g->public_key) {
            L.public_key.resize((size_t)N);
            for (int64_t k = 0; k < N; k++) L.public_key[k] = g->public_key[order[k]];
        }
        return CFR_OK;
    } catch (const std::bad_alloc &) {
        err = "host allocation failed while compiling the game";
        return CFR_ENOMEM;
    }
}

namespace {
// edge code: owner of the parent in bits 0-1, internal flag in bit 2, slot from bit 3
inline int32_t edge_code(int owner, bool internal, int32_t slot) {
    return (int32_t)(((uint32_t)slot << 3) | (internal ? 4u : 0u) | (uint32_t)owner);
}
}  // namespace

namespace {
// Groups of D with at most cap members and `sets` sets; the offsets are stored when iset_off is given.
int64_t form_groups(const DeviceLayout &D, int32_t cap, int32_t sets, std::vector<int32_t> *iset_off,
                    std::vector<int32_t> *depth_off) {
    const int md = (int)D.iset_depth_off.size() - 2;
    if (iset_off) {
        iset_off->assign(1, 0);
        depth_off->assign((size_t)md + 2, 0);
    }
    int64_t G = 0;
    for (int d = 0; d <= md; d++) {
        int32_t members = 0, n = 0;
        for (int32_t i = D.iset_depth_off[d]; i < D.iset_depth_off[d + 1]; i++) {
            const int32_t m = D.mem_off[i + 1] - D.mem_off[i];
            if (n > 0 && (members + m > cap || n + 1 > sets)) {
                if (iset_off) iset_off->push_back(i);
                G++;
                members = 0; n = 0;
            }
            members += m; n++;
        }
        if (n > 0) {
            if (iset_off) iset_off->push_back(D.iset_depth_off[d + 1]);
            G++;
        }
        if (iset_off) (*depth_off)[d + 1] = (int32_t)iset_off->size() - 1;
    }
    return G;
}
}  // namespace

cfr_status set_update_groups(DeviceLayout &D, int32_t sets, std::string &err) {
    const int32_t cap = D.group_cap;
    D.groups_by_bound[0] = form_groups(D, cap, 128, nullptr, nullptr);
    D.groups_by_bound[1] = form_groups(D, cap, GROUP_SETS_MAX, nullptr, nullptr);
    if (sets == 0) sets = choose_group_sets(D.groups_by_bound[0], D.groups_by_bound[1]);
    if (sets != 128 && sets != GROUP_SETS_MAX) {
        err = "update groups hold at most 128 or 256 sets";
        return CFR_EINVAL;
    }
    D.group_sets = sets;
    form_groups(D, cap, sets, &D.grp_iset_off, &D.grp_depth_off);
    // the update kernels stream a group through LDS in chunks of `cap` members and map members to
    // sets for the first chunk only: a group that needs several chunks must hold a single set
    for (size_t gi = 0; gi + 1 < D.grp_iset_off.size(); gi++) {
        const int32_t i0 = D.grp_iset_off[gi], i1 = D.grp_iset_off[gi + 1];
        if (i1 - i0 > 1 && D.mem_off[i1] - D.mem_off[i0] > cap) {
            err = "internal: an update group of several sets exceeds one staging chunk";
            return CFR_EINVAL;
        }
    }
    const int md = (int)D.grp_depth_off.size() - 2;
    if (D.n_games == 1 && D.game_range.size() == (size_t)(md + 1) * GR_FIELDS)
        for (int d = 0; d <= md; d++) {
            D.game_range[(size_t)d * GR_FIELDS + 2] = D.grp_depth_off[d];
            D.game_range[(size_t)d * GR_FIELDS + 3] = D.grp_depth_off[d + 1];
        }
    return CFR_OK;
}

cfr_status build_device_layout(const Layout &L, int kind, int group_actions, bool fp64, int group_sets,
                               DeviceLayout &D, std::string &err) {
    try {
        const int64_t N = L.N, I = L.I, A = L.A;
        const int md = L.max_depth;
        const bool pub = kind == CFR_LAYOUT_PUBLIC;
        std::vector<int32_t> perm((size_t)N), inv((size_t)N);
        D.depth_off = L.depth_off;
        D.int_end.assign((size_t)md + 1, 0);
        auto internal = [&](int64_t k) { return L.child_off[k + 1] > L.child_off[k]; };
        if (!pub) {
            for (int64_t k = 0; k < N; k++) perm[k] = inv[k] = (int32_t)k;
            for (int d = 0; d <= md; d++) D.int_end[d] = L.depth_off[d + 1];
        } else {
            const bool have_keys = !L.public_key.empty();
            std::vector<int32_t> rank;
            std::vector<int64_t> count;
            for (int d = 0; d <= md; d++) {
                const int32_t lo = L.depth_off[d], hi = L.depth_off[d + 1];
                const int64_t n = hi - lo;
                // rank public states by first occurrence inside this depth
                rank.assign((size_t)n, 0);
                int32_t R = 1;
                if (have_keys) {
                    KeyMap km(n);
                    R = 0;
                    for (int64_t j = 0; j < n; j++) {
                        int32_t r = km.find_or_insert(L.public_key[lo + j], R);
                        if (r == R) R++;
                        rank[j] = r;
                    }
                    // then order the states by the action count of their decision nodes (ties by
                    // first occurrence), so that consecutive information sets, and hence the update
                    // groups cut from them, mostly share one action count
                    std::vector<int32_t> na((size_t)R, 0), order((size_t)R), to((size_t)R);
                    for (int64_t j = 0; j < n; j++)
                        if (L.node_type[lo + j] == CFR_NODE_P1 || L.node_type[lo + j] == CFR_NODE_P2)
                            na[rank[j]] = std::max<int32_t>(na[rank[j]], L.child_off[lo + j + 1] - L.child_off[lo + j]);
                    for (int32_t r = 0; r < R; r++) order[r] = r;
                    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return na[x] < na[y]; });
                    for (int32_t r = 0; r < R; r++) to[order[r]] = r;
                    for (int64_t j = 0; j < n; j++) rank[j] = to[rank[j]];
                }
                // stable counting sort by (class, rank): decision, chance, terminal
                auto cls = [&](int64_t k) -> int64_t {
                    int t = L.node_type[k];
                    return t == CFR_NODE_TERMINAL ? 2 : (t == CFR_NODE_CHANCE ? 1 : 0);
                };
                count.assign((size_t)3 * R + 1, 0);
                for (int64_t j = 0; j < n; j++) count[cls(lo + j) * R + rank[j] + 1]++;
                for (int64_t b = 0; b < 3 * R; b++) count[b + 1] += count[b];
                int64_t n_int = 0;
                for (int64_t j = 0; j < n; j++) {
                    n_int += internal(lo + j);
                    int64_t pos = count[cls(lo + j) * R + rank[j]]++;
                    perm[lo + j] = (int32_t)(lo + pos);
                    inv[lo + pos] = (int32_t)(lo + j);
                }
                D.int_end[d] = (int32_t)(lo + n_int);
            }
        }
        D.explicit_kids = pub;
        if (L.keep_maps) D.node_dev = perm;
        // information sets renumbered by first member in device order
        std::vector<int32_t> iset_dev((size_t)I, -1), iset_canon;
        iset_canon.reserve((size_t)I);
        for (int64_t x = 0; x < N; x++) {
            int32_t ci = L.node_infoset[inv[x]];
            if (ci >= 0 && iset_dev[ci] < 0) { iset_dev[ci] = (int32_t)iset_canon.size(); iset_canon.push_back(ci); }
        }
        D.slot_off.assign((size_t)I + 1, 0);
        D.iset_player.resize((size_t)I);
        for (int64_t i = 0; i < I; i++) {
            int32_t ci = iset_canon[i];
            D.slot_off[i + 1] = D.slot_off[i] + (L.slot_off[ci + 1] - L.slot_off[ci]);
            D.iset_player[i] = L.iset_player[ci];
        }
        std::vector<int32_t> slot_map((size_t)A);
        for (int64_t ci = 0; ci < I; ci++)
            for (int32_t a = 0; a < L.slot_off[ci + 1] - L.slot_off[ci]; a++)
                slot_map[L.slot_off[ci] + a] = D.slot_off[iset_dev[ci]] + a;
        if (pub) D.slot_canon_to_dev = slot_map; else D.slot_canon_to_dev.clear();
        // members ascending in device order
        D.mem_off.assign((size_t)I + 1, 0);
        for (int64_t x = 0; x < N; x++) {
            int32_t ci = L.node_infoset[inv[x]];
            if (ci >= 0) D.mem_off[iset_dev[ci] + 1]++;
        }
        for (int64_t i = 0; i < I; i++) D.mem_off[i + 1] += D.mem_off[i];
        D.mem_node.assign((size_t)L.Ndec, 0);
        {
            std::vector<int32_t> fill(D.mem_off.begin(), D.mem_off.end() - 1);
            for (int64_t x = 0; x < N; x++) {
                int32_t ci = L.node_infoset[inv[x]];
                if (ci >= 0) {
                    // bit 31 marks members of player-2 sets (kernels mask it off)
                    uint32_t tag = L.iset_player[ci] == CFR_NODE_P2 ? 0x80000000u : 0u;
                    D.mem_node[fill[iset_dev[ci]]++] = (int32_t)((uint32_t)x | tag);
                }
            }
        }
        D.iset_depth_off.assign((size_t)md + 2, (int32_t)I);
        {
            int32_t i = 0;
            for (int d = 0; d <= md + 1; d++) {
                while (i < I) {
                    int32_t x = D.mem_node[D.mem_off[i]] & 0x7fffffff;
                    int dep = 0;
                    while (dep <= md && x >= L.depth_off[dep + 1]) dep++;
                    if (dep >= d) break;
                    i++;
                }
                D.iset_depth_off[d] = i;
            }
        }
        // node arrays in device order
        D.up_parent.assign((size_t)N, -1);
        D.up_code.assign((size_t)N, 0);
        D.node_slot.assign((size_t)N, -1);
        D.node_iset.assign((size_t)N, -1);
        D.tmpl.assign((size_t)N, 0.0f);
        D.tmpl64.assign((size_t)N, 0.0);
        D.kid_off.assign((size_t)N + 1, 0);
        if (pub) D.kid.assign((size_t)L.E, 0);
        int32_t e = 0;
        for (int64_t x = 0; x < N; x++) {
            int64_t k = inv[x];
            int32_t p = L.parent[k];
            int owner = 0;
            if (p >= 0 && (L.node_type[p] == CFR_NODE_P1 || L.node_type[p] == CFR_NODE_P2)) owner = L.node_type[p];
            int32_t slot = owner ? slot_map[L.in_slot[k]] : 0;
            D.up_parent[x] = p >= 0 ? perm[p] : -1;
            D.up_code[x] = edge_code(owner, internal(k), slot);
            int32_t ci = L.node_infoset[k];
            if (ci >= 0) {
                D.node_iset[x] = iset_dev[ci];
                D.node_slot[x] = D.slot_off[iset_dev[ci]];
            }
            D.tmpl[x] = L.tmpl[k];
            D.tmpl64[x] = L.tmpl64[k];
            if (pub) {
                D.kid_off[x] = e;
                for (int32_t c = L.child_off[k]; c < L.child_off[k + 1]; c++) D.kid[e++] = perm[c];
            } else {
                D.kid_off[x] = L.child_off[k];
            }
        }
        D.kid_off[N] = pub ? e : L.child_off[N];
        // update groups in device information-set order, never spanning two depths
        D.group_cap = group_members(group_actions > L.max_actions ? group_actions : L.max_actions, fp64);
        cfr_status gst = set_update_groups(D, group_sets, err);
        if (gst != CFR_OK) return gst;
        // internal chance nodes by depth
        D.chance_off.assign((size_t)md + 2, 0);
        D.bigc_off.assign((size_t)md + 2, 0);
        D.chance_node.clear();
        D.bigc_node.clear();
        for (int d = 0; d <= md; d++) {
            for (int32_t x = D.depth_off[d]; x < D.int_end[d]; x++) {
                if (L.node_type[inv[x]] != CFR_NODE_CHANCE) continue;
                const int32_t k = D.kid_off[x + 1] - D.kid_off[x];
                if (k > BIG_FANOUT) D.bigc_node.push_back(x);
                else if (k > 0) D.chance_node.push_back(x);
            }
            D.chance_off[d + 1] = (int32_t)D.chance_node.size();
            D.bigc_off[d + 1] = (int32_t)D.bigc_node.size();
        }
        // single-game forest metadata
        D.n_games = 1;
        D.game_root.assign(1, 0);
        D.game_slot_base = {0, (int64_t)A};
        D.game_depth.assign(1, md);
        D.game_range.assign((size_t)(md + 1) * GR_FIELDS, 0);
        for (int d = 0; d <= md; d++) {
            int32_t *r = &D.game_range[(size_t)d * GR_FIELDS];
            r[0] = D.depth_off[d]; r[1] = D.depth_off[d + 1];
            r[2] = D.grp_depth_off[d]; r[3] = D.grp_depth_off[d + 1];
            r[4] = D.chance_off[d]; r[5] = D.chance_off[d + 1];
            r[6] = D.bigc_off[d]; r[7] = D.bigc_off[d + 1];
        }
        return CFR_OK;
    } catch (const std::bad_alloc &) {
        err = "host allocation failed while building the device layout";
        return CFR_ENOMEM;
    }
}

bool slot_child_offsets(const DeviceLayout &D, std::vector<int32_t> &koff) {
    koff.clear();
    if (!D.explicit_kids) return false;
    const int64_t I = (int64_t)D.slot_off.size() - 1;
    std::vector<int32_t> out((size_t)(I > 0 ? D.slot_off[I] : 0), 0);
    for (int64_t i = 0; i < I; i++) {
        const int32_t s0 = D.slot_off[i], nA = D.slot_off[i + 1] - s0;
        for (int32_t m = D.mem_off[i]; m < D.mem_off[i + 1]; m++) {
            const int32_t h = D.mem_node[m] & 0x7fffffff;
            if (D.kid_off[h + 1] - D.kid_off[h] != nA) return false;
            for (int32_t a = 0; a < nA; a++) {
                const int32_t d = D.kid[D.kid_off[h] + a] - h;
                if (m == D.mem_off[i]) out[s0 + a] = d;
                else if (out[s0 + a] != d) return false;
            }
        }
    }
    koff = std::move(out);
    return true;
}

bool plan_persistent(const std::vector<int64_t> &nodes, int32_t wg_nodes, int32_t max_w, int n_queues,
                     PersistentWork &P, std::string &err) {
    const int n = (int)nodes.size();
    if (n_queues < 1 || max_w < 1) { err = "bad persistent plan parameters"; return false; }
    if (wg_nodes <= 0) wg_nodes = 16384;
    std::vector<int> order((size_t)n);
    for (int s = 0; s < n; s++) order[(size_t)s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nodes[(size_t)a] > nodes[(size_t)b]; });
    for (;;) {
        int64_t wmax = 1;
        for (int s = 0; s < n; s++) wmax = std::max<int64_t>(wmax, (nodes[(size_t)s] + wg_nodes - 1) / wg_nodes);
        if (wmax <= max_w) break;
        if (wg_nodes >= (1 << 30)) { err = "a game needs more workgroups than one XCD holds"; return false; }
        wg_nodes *= 2;
    }
    P = PersistentWork();
    P.wg_nodes = wg_nodes;
    P.W.assign((size_t)n, 1);
    P.queue.assign((size_t)n, 0);
    P.load.assign((size_t)n_queues, 0);
    std::vector<std::vector<int>> qg((size_t)n_queues);
    for (int s : order) {
        const int64_t w = std::max<int64_t>(1, (nodes[(size_t)s] + wg_nodes - 1) / wg_nodes);
        P.W[(size_t)s] = (int32_t)w;
        P.max_W = std::max<int32_t>(P.max_W, (int32_t)w);
        int best = 0;
        for (int q = 1; q < n_queues; q++) if (P.load[(size_t)q] < P.load[(size_t)best]) best = q;
        P.queue[(size_t)s] = best;
        P.load[(size_t)best] += nodes[(size_t)s];
        qg[(size_t)best].push_back(s);
    }
    P.q_off.assign((size_t)n_queues + 1, 0);
    for (int q = 0; q < n_queues; q++) {
        for (int s : qg[(size_t)q])
            for (int32_t r = 0; r < P.W[(size_t)s]; r++) {
                P.ticket.push_back(s);
                P.ticket.push_back(r);
                P.ticket.push_back(P.W[(size_t)s]);
            }
        P.q_off[(size_t)q + 1] = (int32_t)(P.ticket.size() / 3);
    }
    return true;
}

cfr_status build_forest(std::vector<Layout> &Ls, std::vector<DeviceLayout> &Ds, DeviceLayout &F, std::string &err) {
    try {
        const int n = (int)Ds.size();
        if (n == 1) {
            F = std::move(Ds[0]);
            Ds.clear();
            return CFR_OK;
        }
        // the games share the kernels' LDS sizing: one group bound and capacity for all
        F.group_cap = Ds[0].group_cap;
        F.group_sets = Ds[0].group_sets;
        for (int s = 0; s < n; s++) {
            if (Ds[s].group_sets != F.group_sets || Ds[s].group_cap != F.group_cap) {
                err = "internal: the games of a batch differ in their update group bounds";
                return CFR_EINVAL;
            }
            F.groups_by_bound[0] += Ds[s].groups_by_bound[0];
            F.groups_by_bound[1] += Ds[s].groups_by_bound[1];
        }
        int MD = 0;
        for (int s = 0; s < n; s++) MD = std::max(MD, (int)Ds[s].depth_off.size() - 2);
        auto md_of = [&](int s) { return (int)Ds[s].depth_off.size() - 2; };
        auto cnt = [&](const std::vector<int32_t> &off, int s, int d) -> int32_t {
            return d <= md_of(s) ? off[d + 1] - off[d] : 0;
        };
        // node, set, group and chance bases per (depth, game)
        std::vector<int64_t> nb((size_t)(MD + 1) * n), ib((size_t)(MD + 1) * n), gb((size_t)(MD + 1) * n),
            cb((size_t)(MD + 1) * n), bb((size_t)(MD + 1) * n);
        F.depth_off.assign((size_t)MD + 2, 0);
        F.iset_depth_off.assign((size_t)MD + 2, 0);
        F.grp_depth_off.assign((size_t)MD + 2, 0);
        F.chance_off.assign((size_t)MD + 2, 0);
        F.bigc_off.assign((size_t)MD + 2, 0);
        int64_t N = 0, I = 0, G = 0, C = 0, B = 0;
        for (int d = 0; d <= MD; d++) {
            F.depth_off[d] = (int32_t)N; F.iset_depth_off[d] = (int32_t)I;
            F.grp_depth_off[d] = (int32_t)G; F.chance_off[d] = (int32_t)C; F.bigc_off[d] = (int32_t)B;
            for (int s = 0; s < n; s++) {
                const DeviceLayout &D = Ds[s];
                nb[(size_t)d * n + s] = N; ib[(size_t)d * n + s] = I;
                gb[(size_t)d * n + s] = G; cb[(size_t)d * n + s] = C; bb[(size_t)d * n + s] = B;
                N += cnt(D.depth_off, s, d); I += cnt(D.iset_depth_off, s, d);
                G += cnt(D.grp_depth_off, s, d); C += cnt(D.chance_off, s, d); B += cnt(D.bigc_off, s, d);
            }
        }
        F.depth_off[MD + 1] = (int32_t)N; F.iset_depth_off[MD + 1] = (int32_t)I;
        F.grp_depth_off[MD + 1] = (int32_t)G; F.chance_off[MD + 1] = (int32_t)C; F.bigc_off[MD + 1] = (int32_t)B;
        if (N > 0x7fffffffLL) { err = "batch too large"; return CFR_EINVAL; }
        // per game: depth of each node and of each set, to remap ids
        std::vector<std::vector<int8_t>> ndep(n), idep(n);
        std::vector<std::vector<int32_t>> slot_set(n);
        for (int s = 0; s < n; s++) {
            const DeviceLayout &D = Ds[s];
            ndep[s].resize(D.depth_off.back());
            for (int d = 0; d <= md_of(s); d++)
                for (int32_t x = D.depth_off[d]; x < D.depth_off[d + 1]; x++) ndep[s][x] = (int8_t)d;
            const int32_t Is = D.iset_depth_off.back();
            idep[s].resize(Is);
            for (int d = 0; d <= md_of(s); d++)
                for (int32_t i = D.iset_depth_off[d]; i < D.iset_depth_off[d + 1]; i++) idep[s][i] = (int8_t)d;
            slot_set[s].resize(D.slot_off.empty() ? 0 : D.slot_off.back());
            for (int32_t i = 0; i < Is; i++)
                for (int32_t q = D.slot_off[i]; q < D.slot_off[i + 1]; q++) slot_set[s][q] = i;
        }
        auto node = [&](int s, int32_t x) -> int32_t {
            const int d = ndep[s][x];
            return (int32_t)(nb[(size_t)d * n + s] + (x - Ds[s].depth_off[d]));
        };
        auto iset = [&](int s, int32_t i) -> int32_t {
            const int d = idep[s][i];
            return (int32_t)(ib[(size_t)d * n + s] + (i - Ds[s].iset_depth_off[d]));
        };
        // sets and slots in forest order
        F.slot_off.assign((size_t)I + 1, 0);
        F.iset_player.assign((size_t)I, 0);
        F.mem_off.assign((size_t)I + 1, 0);
        for (int s = 0; s < n; s++) {
            const DeviceLayout &D = Ds[s];
            for (int32_t i = 0; i + 1 < (int32_t)D.slot_off.size(); i++) {
                const int32_t fi = iset(s, i);
                F.slot_off[fi + 1] = D.slot_off[i + 1] - D.slot_off[i];
                F.mem_off[fi + 1] = D.mem_off[i + 1] - D.mem_off[i];
                F.iset_player[fi] = D.iset_player[i];
            }
        }
        for (int64_t i = 0; i < I; i++) { F.slot_off[i + 1] += F.slot_off[i]; F.mem_off[i + 1] += F.mem_off[i]; }
        auto slot = [&](int s, int32_t q) -> int32_t {
            const int32_t i = slot_set[s][q];
            return F.slot_off[iset(s, i)] + (q - Ds[s].slot_off[i]);
        };
        // node arrays
        int64_t E = 0;
        for (int s = 0; s < n; s++) E += Ds[s].kid_off.back() - Ds[s].kid_off.front();
        F.explicit_kids = true;
        F.up_parent.assign((size_t)N, -1);
        F.up_code.assign((size_t)N, 0);
        F.node_slot.assign((size_t)N, -1);
        F.node_iset.assign((size_t)N, -1);
        F.tmpl.assign((size_t)N, 0.0f);
        F.tmpl64.assign((size_t)N, 0.0);
        F.kid_off.assign((size_t)N + 1, 0);
        F.kid.assign((size_t)E, 0);
        std::vector<int32_t> nkids((size_t)N, 0);
        for (int s = 0; s < n; s++) {
            const DeviceLayout &D = Ds[s];
            const int32_t Ns = D.depth_off.back();
            for (int32_t x = 0; x < Ns; x++) {
                const int32_t fx = node(s, x);
                F.up_parent[fx] = D.up_parent[x] >= 0 ? node(s, D.up_parent[x]) : -1;
                int32_t code = D.up_code[x];
                const int owner = code & 3;
                if (owner) code = (int32_t)(((uint32_t)slot(s, (int32_t)((uint32_t)code >> 3)) << 3) | (uint32_t)(code & 7));
                F.up_code[fx] = code;
                if (D.node_iset[x] >= 0) {
                    F.node_iset[fx] = iset(s, D.node_iset[x]);
                    F.node_slot[fx] = F.slot_off[F.node_iset[fx]];
                }
                F.tmpl[fx] = D.tmpl[x];
                F.tmpl64[fx] = D.tmpl64[x];
                nkids[fx] = D.kid_off[x + 1] - D.kid_off[x];
            }
        }
        for (int64_t x = 0; x < N; x++) F.kid_off[x + 1] = F.kid_off[x] + nkids[x];
        for (int s = 0; s < n; s++) {
            const DeviceLayout &D = Ds[s];
            const int32_t Ns = D.depth_off.back();
            for (int32_t x = 0; x < Ns; x++) {
                const int32_t fx = node(s, x);
                int32_t e = F.kid_off[fx];
                for (int32_t k = D.kid_off[x]; k < D.kid_off[x + 1]; k++)
                    F.kid[e++] = node(s, D.explicit_kids ? D.kid[k] : k);
            }
        }
        // members (player tag kept), groups, chance nodes
        F.mem_node.assign((size_t)F.mem_off[I], 0);
        for (int s = 0; s < n; s++) {
            const DeviceLayout &D = Ds[s];
            for (int32_t i = 0; i + 1 < (int32_t)D.mem_off.size(); i++) {
                int32_t w = F.mem_off[iset(s, i)];
                for (int32_t k = D.mem_off[i]; k < D.mem_off[i + 1]; k++) {
                    const uint32_t tag = (uint32_t)D.mem_node[k] & 0x80000000u;
                    F.mem_node[w++] = (int32_t)((uint32_t)node(s, D.mem_node[k] & 0x7fffffff) | tag);
                }
            }
        }
        F.grp_iset_off.assign((size_t)G + 1, 0);
        F.chance_node.assign((size_t)C, 0);
        F.bigc_node.assign((size_t)B, 0);
        for (int d = 0; d <= MD; d++)
            for (int s = 0; s < n; s++) {
                const DeviceLayout &D = Ds[s];
                if (d > md_of(s)) continue;
                int64_t g = gb[(size_t)d * n + s];
                for (int32_t k = D.grp_depth_off[d]; k < D.grp_depth_off[d + 1]; k++, g++) {
                    F.grp_iset_off[g] = iset(s, D.grp_iset_off[k]);
                    // a group ends where the next starts; the last set of the game's depth ends it
                    const int32_t last = D.grp_iset_off[k + 1] - 1;
                    F.grp_iset_off[g + 1] = iset(s, last) + 1;
                }
                int64_t c = cb[(size_t)d * n + s];
                for (int32_t k = D.chance_off[d]; k < D.chance_off[d + 1]; k++) F.chance_node[c++] = node(s, D.chance_node[k]);
                int64_t b = bb[(size_t)d * n + s];
                for (int32_t k = D.bigc_off[d]; k < D.bigc_off[d + 1]; k++) F.bigc_node[b++] = node(s, D.bigc_node[k]);
            }
        F.int_end.assign((size_t)MD + 1, 0);
        for (int d = 0; d <= MD; d++) F.int_end[d] = F.depth_off[d + 1];  // terminals interleave across games
        // canonical slots at the ABI: game s's canonical slots follow game s-1's
        F.n_games = n;
        F.game_root.resize(n);
        F.game_depth.resize(n);
        F.game_slot_base.assign((size_t)n + 1, 0);
        for (int s = 0; s < n; s++) {
            F.game_root[s] = node(s, 0);
            F.game_depth[s] = md_of(s);
            F.game_slot_base[s + 1] = F.game_slot_base[s] + (int64_t)slot_set[s].size();
        }
        F.slot_canon_to_dev.assign((size_t)F.game_slot_base[n], 0);
        for (int s = 0; s < n; s++) {
            const DeviceLayout &D = Ds[s];
            const int64_t As = (int64_t)slot_set[s].size();
            for (int64_t c = 0; c < As; c++) {
                const int32_t q = D.slot_canon_to_dev.empty() ? (int32_t)c : D.slot_canon_to_dev[c];
                F.slot_canon_to_dev[F.game_slot_base[s] + c] = slot(s, q);
            }
        }
        F.game_range.assign((size_t)n * (MD + 1) * GR_FIELDS, 0);
        for (int s = 0; s < n; s++)
            for (int d = 0; d <= MD; d++) {
                int32_t *r = &F.game_range[((size_t)s * (MD + 1) + d) * GR_FIELDS];
                const size_t k = (size_t)d * n + s;
                r[0] = (int32_t)nb[k]; r[1] = (int32_t)(nb[k] + cnt(Ds[s].depth_off, s, d));
                r[2] = (int32_t)gb[k]; r[3] = (int32_t)(gb[k] + cnt(Ds[s].grp_depth_off, s, d));
                r[4] = (int32_t)cb[k]; r[5] = (int32_t)(cb[k] + cnt(Ds[s].chance_off, s, d));
                r[6] = (int32_t)bb[k]; r[7] = (int32_t)(bb[k] + cnt(Ds[s].bigc_off, s, d));
            }
        Ds.clear();
        Ls.clear();
        return CFR_OK;
    } catch (const std::bad_alloc &) {
        err = "host allocation failed while merging the batch";
        return CFR_ENOMEM;
    }
}

}  // namespace cfrx
