// runtime.hip -- handle, device memory, hipGraph capture/replay and the C ABI
// declared in include/cfr.h.
//
// One iteration is a fixed sequence of launches (paper Proposition 3 (iii):
// c1 + c2 D operations): D forward levels (the first also bumps the device
// iteration counter), D backward levels and one fused update.  The first
// cfr_iterate call runs one iteration with direct launches, then captures
// the body once into a hipGraph (k iterations per graph optional) and replays
// it (paper Section 4.3).  The pointers the graph bakes in are recorded at
// capture time and checked before every replay; a failed capture warns once
// and the handle keeps launching the same kernels directly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cfr.h"
#include "compiler.hpp"
#include "device.hpp"
#include "mlp.hpp"

using namespace cfrx;

namespace {
thread_local std::string g_err;

cfr_status fail(cfr_status s, const std::string &m) {
    g_err = m;
    return s;
}

}  // namespace

void cfrx::set_last_error(const std::string &m) { g_err = m; }

namespace {

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(CFR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)
}  // namespace

struct cfr_handle {
    cfr_options opt{};
    DevGame g{};
    // host copies of the schedule
    std::vector<int32_t> depth_off, int_end, iset_depth_off, grp_depth_off, chance_off, bigc_off;
    // the static launch schedule of one iteration: (kind, depth), kind 0 tick, 1 forward, 2 level,
    // plus HALF for the second (player 2) half of an alternating iteration
    std::vector<std::pair<int, int>> plan;
    std::vector<int32_t> slot_map;     // canonical slot -> device slot (empty: identity)
    // batches: number of games, canonical slot offsets, per-game depth and ranges, pots
    int32_t n_games = 1;
    std::vector<int64_t> game_slot_base;
    std::vector<int32_t> game_depth, game_range;
    std::vector<double> game_pot;
    // persistent schedule
    bool persistent = false;
    // set when a persistent launch stopped part-way (a barrier timed out): the state is partial, so
    // cfr_iterate refuses until cfr_reset starts over
    bool broken = false;
    // LDS-resident schedule (one tiny game, one workgroup): per-depth ranges on the device
    bool lds = false;
    int32_t *lds_range = nullptr;
    int32_t wg_nodes = 16384;
    PersistentPlan pp{};
    std::vector<void *> pp_allocs;
    hipGraph_t pgraph = nullptr;
    hipGraphExec_t pexec = nullptr;
    int64_t pgraph_n = -1;
    std::string device_name;
    int32_t D = 0;
    bool br_ok = true;
    int64_t E = 0, Z = 0;
    double pot = 1.0;
    int64_t device_bytes = 0;
    std::vector<double> perm_members;  // per depth: members of update groups listed in node order
    // batches: per-game activity (cfr_set_active); each depth's forward tiles (first tile per depth,
    // each tile's first and last game) and the lists of the work that still runs, per depth
    std::vector<int8_t> active;
    std::vector<int64_t> fwd_tile_base;
    std::vector<int2> fwd_games;
    std::vector<int64_t> fwd_off, grp_off, chance_off_l, bigc_off_l;
    bool any_inactive = false;
    int32_t node_order_groups = 0;
    int64_t node_order_members = 0;
    std::vector<void *> allocs;
    // graph state
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph1 = nullptr, graphk = nullptr;
    hipGraphExec_t exec1 = nullptr, execk = nullptr;
    bool captured = false, use_graph = true, warned = false;
    std::vector<const void *> pinned;  // pointers baked into the graph
    int64_t rebind[3] = {0, 0, 0};     // test hook offsets
    char *R_base = nullptr, *sigma_base = nullptr, *sbar_base = nullptr;
    size_t es = 4;                     // bytes per state element
    int64_t iters = 0;
    int64_t launches = 0;
    // algorithmic bytes per iteration of each kernel (traffic model, see model_bytes)
    double bytes_fwd = 0, bytes_lvl = 0;
    double method_fwd = 0, method_lvl = 0;   // per-unit byte figures of the method (see model_bytes)
    // canonical information sets of all games (rows of the warm-start network)
    int64_t I_canon = 0;
    int32_t *canon_off = nullptr;      // [I + 1] canonical slot offsets, global over the batch
    int8_t *canon_player = nullptr;    // [I]
    float *warm_z = nullptr;           // [I * 4] logits, allocated on first warm start
    float *warm_mag = nullptr;         // [I] regret unit of each set, written by cfr_features
    bool have_mag = false;
    // in-place re-solve (options.lifecycle): per terminal of every game, games in order
    std::vector<int64_t> lc_term_off;  // [n + 1] terminal records of game s
    std::vector<int64_t> lc_root_off;  // [n + 1] root children of game s (none when the root is not chance)
    std::vector<int64_t> lc_nodes;     // [n] input node count of game s
    int32_t *lc_node = nullptr;        // device node
    int32_t *lc_in = nullptr;          // input node id within its game
    int32_t *lc_branch = nullptr;      // root child above it, -1 when the root is not chance
    double *lc_u = nullptr;            // payoff
    double *lc_pic = nullptr;          // chance product below the root (the whole product without a chance root)
    double *lc_root = nullptr;         // root chance probabilities
    double *lc_stage = nullptr;        // staging for a game's payoff array
    // root hand map of each game (cfr_set_root_ranges): root child a of game s deals hands
    // (lc_hand1[k], lc_hand2[k]), k = lc_hand_off[s] + a; lc_nh1/lc_nh2 are the range lengths
    std::vector<int64_t> lc_hand_off;
    std::vector<int32_t> lc_hand1, lc_hand2, lc_nh1, lc_nh2;
    // canonical arrays of every game (options.keep_layout), for cfr_get_layout
    std::vector<Layout> layouts;
};

// fn(s) for s in [0, n) on up to 16 host threads (one game each at a time); fn must touch only game s.
template <typename F>
static void parallel_games(int n, F &&fn) {
    const int hw = (int)std::thread::hardware_concurrency();
    const int nt = std::max(1, std::min({n, hw > 0 ? hw : 1, 16}));
    if (nt == 1) {
        for (int s = 0; s < n; s++) fn(s);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    pool.reserve((size_t)nt);
    for (int k = 0; k < nt; k++)
        pool.emplace_back([&]() {
            for (int s = next.fetch_add(1); s < n; s = next.fetch_add(1)) fn(s);
        });
    for (auto &t : pool) t.join();
}

// The affine update's member list (mnode).  A group keeps its members in set-major order, unless
// listing them in node order makes a wave's 64 consecutive members touch at most half as many
// 32-node spans (cache lines of FP32 values) -- the case where the group's sets interleave, as a
// player-2 set's members, strided by the opponent's hand count, do.  Such a group is flagged in
// perm[g] and mpos gives each listed member's set-major position in its group (groups of several
// sets hold at most one staging chunk, so it fits 16 bits).  perm_members[d] counts the members of
// flagged groups of depth d (their extra position reads are design bytes).
static void member_lists(const DeviceLayout &D, std::vector<int32_t> &mnode, std::vector<uint16_t> &mpos,
                         std::vector<int8_t> &perm, std::vector<double> &perm_members) {
    const int64_t Ndec = (int64_t)D.mem_node.size();
    mnode = D.mem_node;
    mpos.assign((size_t)Ndec, 0);
    const int32_t G = (int32_t)D.grp_iset_off.size() - 1;
    perm.assign((size_t)std::max(G, 1), 0);
    constexpr int32_t SPAN = 4096;   // groups per task
    parallel_games((G + SPAN - 1) / SPAN, [&](int task) {
        std::vector<int32_t> idx;
        auto spans = [](const int32_t *nodes, int32_t n) {
            int64_t c = 0;
            for (int32_t w = 0; w < n; w += 64) {
                int32_t seen[64];
                int ns = 0;
                for (int32_t k = w; k < std::min(n, w + 64); k++) {
                    const int32_t line = (nodes[k] & MEMBER_NODE_MASK) >> 5;
                    bool dup = false;
                    for (int t = 0; t < ns && !dup; t++) dup = seen[t] == line;
                    if (!dup) seen[ns++] = line;
                }
                c += ns;
            }
            return c;
        };
        std::vector<int32_t> sorted_nodes;
        for (int32_t g = task * SPAN; g < std::min(G, (task + 1) * SPAN); g++) {
            const int32_t i0 = D.grp_iset_off[(size_t)g], i1 = D.grp_iset_off[(size_t)g + 1];
            const int32_t mb = D.mem_off[(size_t)i0], me = D.mem_off[(size_t)i1], n = me - mb;
            for (int32_t k = 0; k < n; k++) mpos[(size_t)(mb + k)] = (uint16_t)(k & 0xffff);
            if (i1 - i0 == 1) continue;
            const int32_t *list = D.mem_node.data() + mb;
            idx.resize((size_t)n);
            for (int32_t k = 0; k < n; k++) idx[(size_t)k] = k;
            std::sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
                return (list[x] & MEMBER_NODE_MASK) < (list[y] & MEMBER_NODE_MASK);
            });
            sorted_nodes.resize((size_t)n);
            for (int32_t k = 0; k < n; k++) sorted_nodes[(size_t)k] = list[idx[(size_t)k]];
            if (2 * spans(sorted_nodes.data(), n) > spans(list, n)) continue;
            perm[(size_t)g] = 1;
            for (int32_t k = 0; k < n; k++) {
                mnode[(size_t)(mb + k)] = sorted_nodes[(size_t)k];
                mpos[(size_t)(mb + k)] = (uint16_t)idx[(size_t)k];
            }
        }
    });
    const int md = (int)D.grp_depth_off.size() - 2;
    perm_members.assign((size_t)std::max(md + 1, 1), 0.0);
    for (int d = 0; d <= md; d++)
        for (int32_t g = D.grp_depth_off[(size_t)d]; g < D.grp_depth_off[(size_t)d + 1]; g++)
            if (perm[(size_t)g])
                perm_members[(size_t)d] += D.mem_off[(size_t)D.grp_iset_off[(size_t)g + 1]] - D.mem_off[(size_t)D.grp_iset_off[(size_t)g]];
}

// Per-launch event timing for cfr_profile: class 0 tick, 1 forward, 2 level.
struct LaunchTimer {
    std::vector<hipEvent_t> ev;   // pairs (before, after)
    std::vector<int> cls;
    size_t next = 0;
};

namespace {

template <typename T>
cfr_status dev_alloc(cfr_handle *h, T **p, int64_t count) {
    size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(CFR_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    h->allocs.push_back(q);
    h->device_bytes += (int64_t)bytes;
    *p = (T *)q;
    return CFR_OK;
}

template <typename T>
cfr_status upload(T *dst, const std::vector<T> &src) {
    if (src.empty()) return CFR_OK;
    HIP_TRY(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return CFR_OK;
}

// The addresses a captured graph bakes in.  The rebinding test hook shifts the reported
// address only; no kernel or copy ever sees a shifted pointer.
std::vector<const void *> persistent_ptrs(const cfr_handle *h) {
    return {h->R_base + h->rebind[0] * (int64_t)h->es, h->sbar_base + h->rebind[1] * 8,
            h->sigma_base + h->rebind[2] * (int64_t)h->es, h->g.v, h->g.reach, h->g.t, h->g.up, h->g.kid_off,
            h->g.mem};
}

// The launch schedule of one iteration (paper Proposition 3 (iii): a fixed sequence whose length
// depends on the depth only): the forward pass over depths 1..max_depth (depth 1 always launches,
// because its first thread advances the iteration counter), then the fused backward/update level
// over depths max_depth-1..0, skipping levels with nothing to do.  A single-node game only ticks.
constexpr int HALF = 10;

void build_plan(cfr_handle *h) {
    h->plan.clear();
    const DevGame &g = h->g;
    if (g.max_depth == 0) { h->plan.push_back({0, 0}); return; }
    const int halves = h->opt.order == CFR_ORDER_ALTERNATING ? 2 : 1;
    for (int half = 0; half < halves; half++) {
        for (int d = 1; d <= g.max_depth; d++)
            if (d == 1 || h->int_end[d] > h->depth_off[d]) h->plan.push_back({1 + HALF * half, d});
        for (int d = g.max_depth - 1; d >= 0; d--)
            if (h->grp_depth_off[d + 1] > h->grp_depth_off[d] || h->chance_off[d + 1] > h->chance_off[d] ||
                h->bigc_off[d + 1] > h->bigc_off[d])
                h->plan.push_back({2 + HALF * half, d});
    }
}

// one iteration, direct launches, in the plan's order; tm != nullptr brackets every launch with events
// flags (optional) replace the handle's rule for one simultaneous pass (the second half of an
// alternating plan is then skipped)
cfr_status enqueue_iteration(cfr_handle *h, hipStream_t s, int64_t *count, LaunchTimer *tm = nullptr,
                             const IterFlags *flags = nullptr) {
    const DevGame &g = h->g;
    const bool alt = h->opt.order == CFR_ORDER_ALTERNATING && !flags;
    int64_t n = 0;
    for (const auto &step : h->plan) {
        const int kind = step.first % HALF, half = step.first / HALF;
        if (half > 0 && !alt) continue;
        if (tm) {
            if (tm->next + 1 >= tm->ev.size()) return fail(CFR_EDEVICE, "profiling event pool exhausted");
            tm->cls.push_back(kind);
            HIP_TRY(hipEventRecord(tm->ev[tm->next++], s));
        }
        const int d = step.second;
        IterFlags f = flags ? *flags : IterFlags{h->opt.rule, h->opt.averaging == CFR_AVG_LINEAR ? 1 : 0, 3};
        if (alt) f.upd = 1 << half;
        if (kind == 0) HIP_TRY(launch_tick(g, s));
        else if (kind == 1)
            HIP_TRY(launch_forward(g, d, h->depth_off[d], h->int_end[d], d == 1 && half == 0 ? g.t : nullptr, s));
        else HIP_TRY(launch_level(g, d, f, s));
        if (tm) {
            tm->cls.push_back(-1);
            HIP_TRY(hipEventRecord(tm->ev[tm->next++], s));
        }
        n++;
    }
    if (count) *count = n;
    return CFR_OK;
}

// Algorithmic bytes of one iteration per kernel: every index, state and value element a
// kernel must touch in the device layout, counted once (sigma gathers count once per slot
// and pass).
void model_bytes(cfr_handle *h, const DeviceLayout &D) {
    const int md = (int)D.depth_off.size() - 2;
    const double es = (double)h->es;
    const double kb = D.explicit_kids ? 4.0 : 0.0;
    std::vector<double> Nr(md + 2, 0), Nint(md + 2, 0), Ad(md + 2, 0), Id(md + 2, 0), Md(md + 2, 0), Ed(md + 2, 0);
    for (int d = 0; d <= md; d++) {
        Nr[d] = D.int_end[d] - D.depth_off[d];
        for (int32_t n = D.depth_off[d]; n < D.int_end[d]; n++) Nint[d] += D.kid_off[n + 1] > D.kid_off[n];
        for (int32_t i = D.iset_depth_off[d]; i < D.iset_depth_off[d + 1]; i++) {
            const double nA = D.slot_off[i + 1] - D.slot_off[i], nm = D.mem_off[i + 1] - D.mem_off[i];
            Ad[d] += nA; Id[d] += 1; Md[d] += nm; Ed[d] += nm * nA;
        }
    }
    double f = 0, lv = 0;
    for (int d = 1; d <= md; d++) f += 8 * Nr[d] + 2 * es * Nint[d - 1] + 2 * es * Nint[d] + es * Ad[d - 1];
    for (int d = 0; d < md; d++) {
        // decision members: id, edge offset, value write, opponent reach; edges: child (index), value;
        // sets: member and slot offsets, player, own reach; slots: sigma read + write, R read + write,
        // sbar read + write
        // (affine layouts: a 4-byte member record, plus a 2-byte staging position in node-order
        // groups; no child index per edge, one offset per slot)
        if (h->g.affine)
            lv += (4 + 2 * es) * Md[d] + es * Ed[d] + (9 + es) * Id[d] + (4 * es + 20) * Ad[d] +
                  2.0 * ((size_t)d < h->perm_members.size() ? h->perm_members[(size_t)d] : 0.0);
        else lv += (8 + 2 * es) * Md[d] + (kb + es) * Ed[d] + (9 + es) * Id[d] + (4 * es + 16) * Ad[d];
        // chance nodes: list entry, edge offset, value write; edges: child (index), value
        for (int32_t j = D.chance_off[d]; j < D.chance_off[d + 1]; j++) {
            const int32_t x = D.chance_node[j];
            lv += 8 + es + (kb + es) * (D.kid_off[x + 1] - D.kid_off[x]);
        }
        for (int32_t j = D.bigc_off[d]; j < D.bigc_off[d + 1]; j++) {
            const int32_t x = D.bigc_node[j];
            lv += 8 + es + (kb + es) * (D.kid_off[x + 1] - D.kid_off[x]);
        }
    }
    const double halves = h->opt.order == CFR_ORDER_ALTERNATING ? 2.0 : 1.0;
    double pred_bytes = 0;   // PCFR+: the prediction written and read back by regret matching
    if (h->opt.rule == CFR_RULE_PCFR_PLUS)
        for (int d = 0; d < md; d++) pred_bytes += 2 * es * Ad[d];
    h->bytes_fwd = f * halves;
    h->bytes_lvl = (lv + pred_bytes) * halves;
    // The method's per-unit byte figures with 4-byte indices and state width es (FP64 strategy
    // sums): forward, per edge the parent index and edge code (8) and the two-lane reach write
    // (2 es), per internal parent the two-lane reach read (2 es); backward, per edge the child
    // value and pointer (es + 4), per terminal the template (es), per internal node the child
    // offset and value write (4 + es); regret, per decision edge the child value (es), per
    // decision node its id, value and both reaches (4 + 3 es), per set its offsets (4); per slot,
    // regrets read and written (2 es), strategy written and read twice (3 es), strategy sums read
    // and written (16) and the regret-matching read (2 es).
    std::vector<double> Zd(md + 2, 0), Nd(md + 2, 0);
    for (int d = 0; d <= md; d++) {
        Nd[d] = D.depth_off[d + 1] - D.depth_off[d];
        Zd[d] = Nd[d] - (double)(D.int_end[d] - D.depth_off[d]);
        if (!D.explicit_kids) {
            Zd[d] = 0;
            for (int32_t n = D.depth_off[d]; n < D.depth_off[d + 1]; n++) Zd[d] += D.kid_off[n + 1] == D.kid_off[n];
        }
    }
    double mf = 0, ml = 0;
    for (int d = 1; d <= md; d++) mf += (8 + 2 * es) * Nd[d] + 2 * es * Nint[d - 1];
    for (int d = 0; d < md; d++)
        ml += (es + 4) * Nd[d + 1] + es * Zd[d + 1] + (4 + es) * Nint[d] + es * Ed[d] + (4 + 3 * es) * Md[d] +
              4 * Id[d] + (7 * es + 16) * Ad[d];
    h->method_fwd = mf * halves;
    h->method_lvl = (ml + pred_bytes) * halves;
}

cfr_status capture(cfr_handle *h, int iters, hipGraph_t *graph, hipGraphExec_t *exec) {
    hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(CFR_EGRAPH, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    cfr_status st = CFR_OK;
    for (int k = 0; k < iters && st == CFR_OK; k++) st = enqueue_iteration(h, h->cap_stream, nullptr);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(h->cap_stream, &gr);
    if (st != CFR_OK) { if (gr) (void)hipGraphDestroy(gr); return st; }
    if (e != hipSuccess || !gr) return fail(CFR_EGRAPH, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(gr); return fail(CFR_EGRAPH, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)); }
    *graph = gr;
    *exec = ex;
    return CFR_OK;
}

// Destroy the captured iteration graphs; the next cfr_iterate captures them again.
void drop_graphs(cfr_handle *h) {
    if (h->exec1) (void)hipGraphExecDestroy(h->exec1);
    if (h->execk) (void)hipGraphExecDestroy(h->execk);
    if (h->graph1) (void)hipGraphDestroy(h->graph1);
    if (h->graphk) (void)hipGraphDestroy(h->graphk);
    h->exec1 = h->execk = nullptr;
    h->graph1 = h->graphk = nullptr;
    h->captured = false;
}

void free_handle(cfr_handle *h) {
    if (!h) return;
    if (h->exec1) (void)hipGraphExecDestroy(h->exec1);
    if (h->execk) (void)hipGraphExecDestroy(h->execk);
    if (h->graph1) (void)hipGraphDestroy(h->graph1);
    if (h->graphk) (void)hipGraphDestroy(h->graphk);
    if (h->pexec) (void)hipGraphExecDestroy(h->pexec);
    if (h->pgraph) (void)hipGraphDestroy(h->pgraph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (void *p : h->pp_allocs) (void)hipFree(p);
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
}

void fill_counts(const Layout &L, cfr_counts_t *c, double pot) {
    std::memset(c, 0, sizeof *c);
    c->nodes = L.N; c->edges = L.E; c->terminals = L.Z; c->decision_nodes = L.Ndec;
    c->infosets = L.I; c->slots = L.A; c->max_depth = L.max_depth; c->blocks = L.D;
    c->max_actions = L.max_actions; c->br_supported = L.br_ok ? 1 : 0; c->pot = pot;
}

template <typename T>
T *copy_out(const std::vector<T> &v) {
    T *p = (T *)std::malloc((v.size() ? v.size() : 1) * sizeof(T));
    if (p && !v.empty()) std::memcpy(p, v.data(), v.size() * sizeof(T));
    return p;
}

}  // namespace

extern "C" {

void cfr_default_options(cfr_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->rule = CFR_RULE_CFR_PLUS;
    o->averaging = CFR_AVG_LINEAR;
    o->order = CFR_ORDER_SIMULTANEOUS;
    o->iters_per_graph = 1;
    o->layout = CFR_LAYOUT_PUBLIC;
    o->use_graph = 1;
    o->device = 0;
    o->test_fail_capture = 0;
    o->precision = CFR_PRECISION_FP32;
    o->persistent = 0;
    o->wg_nodes = 0;
    o->lifecycle = 0;
    o->affine = 1;
}

const char *cfr_last_error(void) { return g_err.c_str(); }

static cfr_status layout_out(const Layout &L, double pot, cfr_layout *out);

cfr_status cfr_layout_host(const cfr_game_desc *game, cfr_layout *out) {
    if (!out) return fail(CFR_EINVAL, "out is NULL");
    std::memset(out, 0, sizeof *out);
    Layout L;
    std::string err;
    cfr_status st = build_layout(game, L, err);
    if (st != CFR_OK) return fail(st, err);
    return layout_out(L, game->pot, out);
}

cfr_status cfr_get_layout(cfr_handle *h, int32_t game, cfr_layout *out) {
    if (!h || !out) return fail(CFR_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof *out);
    if (game < 0 || game >= h->n_games) return fail(CFR_EINVAL, "game index out of range");
    if (h->layouts.empty()) return fail(CFR_ESTATE, "compile with options.keep_layout = 1 to keep the canonical arrays");
    cfr_status st = layout_out(h->layouts[(size_t)game], h->game_pot[(size_t)game], out);
    if (st != CFR_OK) return st;
    out->counts.device_bytes = h->device_bytes;
    out->counts.kernels_per_iteration = h->launches;
    return CFR_OK;
}

static cfr_status layout_out(const Layout &L, double pot, cfr_layout *out) {
    fill_counts(L, &out->counts, pot);
    out->depth_off = copy_out(L.depth_off);
    out->parent = copy_out(L.parent);
    out->child_off = copy_out(L.child_off);
    out->in_slot = copy_out(L.in_slot);
    out->node_infoset = copy_out(L.node_infoset);
    out->node_type = copy_out(L.node_type);
    out->tmpl = copy_out(L.tmpl);
    out->slot_off = copy_out(L.slot_off);
    out->mem_off = copy_out(L.mem_off);
    out->mem_node = copy_out(L.mem_node);
    out->iset_player = copy_out(L.iset_player);
    out->iset_key = copy_out(L.iset_key);
    if (!out->depth_off || !out->parent || !out->child_off || !out->in_slot || !out->node_infoset ||
        !out->node_type || !out->tmpl || !out->slot_off || !out->mem_off || !out->mem_node || !out->iset_player ||
        !out->iset_key) {
        cfr_layout_free(out);
        return fail(CFR_ENOMEM, "host allocation failed");
    }
    return CFR_OK;
}

void cfr_layout_free(cfr_layout *l) {
    if (!l) return;
    std::free(l->depth_off); std::free(l->parent); std::free(l->child_off); std::free(l->in_slot);
    std::free(l->node_infoset); std::free(l->node_type); std::free(l->tmpl); std::free(l->slot_off);
    std::free(l->mem_off); std::free(l->mem_node); std::free(l->iset_player); std::free(l->iset_key);
    std::memset(l, 0, sizeof *l);
}

// Work plan of the persistent launch (plan_persistent): per-XCD queues of (game, rank) tickets, each
// game's ranks at most a quarter of one XCD's resident workgroups, games balanced over the queues
// largest first.  The grid is the device's resident capacity for the kernel; workgroups claim tickets
// in order (see k_persistent).  At any time at most one game per queue is partly claimed, so with
// W <= max_w the launch keeps progressing whenever 8 (max_w - 1) + 1 workgroups -- a quarter of the
// device -- can be resident, whatever else holds the rest.
static cfr_status build_persistent_plan(cfr_handle *h, int32_t wg_nodes) {
    const DevGame &g = h->g;
    const int n = h->n_games;
    const int MD = g.max_depth;
    int per_cu = 0, cus = 0;
    HIP_TRY(persistent_occupancy(g, &per_cu));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, h->opt.device));
    cus = prop.multiProcessorCount;
    const int64_t capacity = (int64_t)per_cu * cus;
    if (capacity < PERSISTENT_QUEUES) return fail(CFR_EDEVICE, "persistent kernel cannot be resident");
    std::vector<int64_t> nodes((size_t)n, 0);
    for (int s = 0; s < n; s++)
        for (int d = 0; d <= MD; d++) {
            const int32_t *r = &h->game_range[((size_t)s * (MD + 1) + d) * GR_FIELDS];
            nodes[s] += r[1] - r[0];
        }
    PersistentWork P;
    std::string err;
    const int32_t max_w = (int32_t)std::max<int64_t>(1, capacity / PERSISTENT_QUEUES / 4);
    if (!plan_persistent(nodes, wg_nodes, max_w, PERSISTENT_QUEUES, P, err)) return fail(CFR_EUNSUPPORTED, err);
    std::vector<int4> table(P.ticket.size() / 3);
    for (size_t k = 0; k < table.size(); k++)
        table[k] = make_int4(P.ticket[3 * k], P.ticket[3 * k + 1], P.ticket[3 * k + 2], 0);
    // device copies (replacing any previous plan)
    for (void *p : h->pp_allocs) (void)hipFree(p);
    h->pp_allocs.clear();
    auto alloc = [&](void **p, size_t bytes) -> cfr_status {
        hipError_t e = hipMalloc(p, bytes ? bytes : 4);
        if (e != hipSuccess) return fail(CFR_ENOMEM, "hipMalloc for the persistent plan failed");
        h->pp_allocs.push_back(*p);
        return CFR_OK;
    };
    PersistentPlan &pp = h->pp;
    cfr_status st;
    if ((st = alloc((void **)&pp.tickets, table.size() * sizeof(int4))) != CFR_OK) return st;
    if ((st = alloc((void **)&pp.q_off, P.q_off.size() * sizeof(int32_t))) != CFR_OK) return st;
    if ((st = alloc((void **)&pp.game_range, h->game_range.size() * sizeof(int32_t))) != CFR_OK) return st;
    if ((st = alloc((void **)&pp.game_depth, (size_t)n * sizeof(int32_t))) != CFR_OK) return st;
    // barrier counters of the games, then the queues' claim counters (zeroed together per launch)
    if ((st = alloc((void **)&pp.barrier, ((size_t)n + PERSISTENT_QUEUES) * sizeof(int32_t))) != CFR_OK) return st;
    if ((st = alloc((void **)&pp.err, sizeof(int32_t))) != CFR_OK) return st;
    pp.claim = pp.barrier + n;
    HIP_TRY(hipMemcpy(pp.tickets, table.data(), table.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(pp.q_off, P.q_off.data(), P.q_off.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(pp.game_range, h->game_range.data(), h->game_range.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(pp.game_depth, h->game_depth.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(pp.err, 0, sizeof(int32_t)));
    {
        int khz = 0;  // rate of the constant clock wall_clock64() reads
        HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->opt.device));
        if (khz <= 0) return fail(CFR_EDEVICE, "device reports no wall-clock rate");
        pp.timeout_ticks = (int64_t)(BARRIER_TIMEOUT_S * 1000.0 * khz);
    }
    pp.n_tickets = (int32_t)table.size();
    pp.blocks = (int32_t)std::min<int64_t>(capacity, ((int64_t)pp.n_tickets + PERSISTENT_QUEUES - 1) /
                                                         PERSISTENT_QUEUES * PERSISTENT_QUEUES);
    pp.n_games = n;
    pp.max_depth = MD;
    pp.wg_nodes = P.wg_nodes;
    pp.max_W = P.max_W;
    h->wg_nodes = P.wg_nodes;
    if (h->pexec) { (void)hipGraphExecDestroy(h->pexec); h->pexec = nullptr; }
    if (h->pgraph) { (void)hipGraphDestroy(h->pgraph); h->pgraph = nullptr; }
    h->pgraph_n = -1;
    return CFR_OK;
}

// One launch (captured once per n) that runs all n iterations: the persistent or the LDS schedule.
static cfr_status persistent_iterate(cfr_handle *h, int64_t n, hipStream_t s) {
    if (n > 0x7fffffffLL) return fail(CFR_EINVAL, "n too large for one persistent launch");
    const IterFlags f{h->opt.rule, h->opt.averaging == CFR_AVG_LINEAR ? 1 : 0, 3};
    const int alt = h->opt.order == CFR_ORDER_ALTERNATING ? 1 : 0;
    if (h->use_graph && h->pgraph_n != n) {
        if (h->pexec) { (void)hipGraphExecDestroy(h->pexec); h->pexec = nullptr; }
        if (h->pgraph) { (void)hipGraphDestroy(h->pgraph); h->pgraph = nullptr; }
        h->pgraph_n = -1;
        hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = h->lds ? launch_lds(h->g, h->lds_range, (int32_t)n, f, alt, h->cap_stream)
                                   : launch_persistent(h->g, h->pp, (int32_t)n, f, alt, h->cap_stream);
            hipGraph_t gr = nullptr;
            e = hipStreamEndCapture(h->cap_stream, &gr);
            if (le == hipSuccess && e == hipSuccess && gr) {
                hipGraphExec_t ex = nullptr;
                if (hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) == hipSuccess) {
                    h->pgraph = gr; h->pexec = ex; h->pgraph_n = n;
                } else {
                    (void)hipGraphDestroy(gr);
                }
            } else if (gr) {
                (void)hipGraphDestroy(gr);
            }
        }
    }
    if (h->pexec && h->pgraph_n == n) {
        hipError_t e = hipGraphLaunch(h->pexec, s);
        if (e != hipSuccess) return fail(CFR_EGRAPH, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    } else if (h->lds) {
        HIP_TRY(launch_lds(h->g, h->lds_range, (int32_t)n, f, alt, s));
    } else {
        HIP_TRY(launch_persistent(h->g, h->pp, (int32_t)n, f, alt, s));
    }
    if (h->lds) {   // no barriers, no error flag to read back
        h->iters += n;
        return CFR_OK;
    }
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, h->pp.err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err) {
        h->broken = true;
        return fail(CFR_EDEVICE, "a per-game barrier of the persistent launch timed out; the solver state is "
                                 "partial (call cfr_reset)");
    }
    h->iters += n;
    return CFR_OK;
}

// Per-terminal records of the in-place re-solve: device node (of the game's own device layout
// until the forest renumbers it), input id, payoff, chance product below the root, root branch.
struct LifecycleHost {
    std::vector<int64_t> term_off{0}, root_off{0}, nodes;
    std::vector<int32_t> node, in, branch, depth;
    std::vector<double> u, pic, root;
    std::vector<std::vector<int32_t>> depth_off;   // per game
};

static void lifecycle_records(const cfr_game_desc &g, const Layout &L, const DeviceLayout &D, LifecycleHost &lc) {
    const int64_t N = L.N;
    const bool chance_root = L.node_type[0] == CFR_NODE_CHANCE;
    std::vector<double> pic((size_t)N, 1.0);
    std::vector<int32_t> br((size_t)N, -1);
    for (int64_t k = 0; k < N; k++) {
        const int32_t h = L.input_id[(size_t)k];
        for (int32_t c = L.child_off[k]; c < L.child_off[k + 1]; c++) {
            const int32_t a = c - L.child_off[k];
            if (k == 0 && chance_root) {
                br[c] = a;
                pic[c] = 1.0;
            } else {
                br[c] = br[k];
                pic[c] = L.node_type[k] == CFR_NODE_CHANCE ? pic[k] * g.chance_prob[g.child_begin[h] + a] : pic[k];
            }
        }
    }
    int d = 0;
    for (int64_t k = 0; k < N; k++) {
        while (k >= L.depth_off[d + 1]) d++;
        if (L.node_type[k] != CFR_NODE_TERMINAL) continue;
        const int32_t h = L.input_id[(size_t)k];
        lc.node.push_back(D.node_dev[(size_t)k]);
        lc.in.push_back(h);
        lc.branch.push_back(br[k]);
        lc.depth.push_back(d);
        lc.u.push_back(g.payoff[h]);
        lc.pic.push_back(pic[k]);
    }
    if (chance_root)
        for (int32_t a = 0; a < g.num_children[g.root]; a++) lc.root.push_back(g.chance_prob[g.child_begin[g.root] + a]);
    lc.term_off.push_back((int64_t)lc.node.size());
    lc.root_off.push_back((int64_t)lc.root.size());
    lc.nodes.push_back(g.num_nodes);
    lc.depth_off.push_back(L.depth_off);
}

// Compile one game or a batch of independent games (a depth-major forest, see build_forest).
static cfr_status compile_games(const cfr_game_desc *games, int n, const cfr_options *opt, cfr_handle **out) {
    if (!out) return fail(CFR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!games || n <= 0) return fail(CFR_EINVAL, "no games");
    cfr_options o;
    cfr_default_options(&o);
    if (opt) o = *opt;
    if (o.rule < CFR_RULE_CFR_PLUS || o.rule > CFR_RULE_PCFR_PLUS) return fail(CFR_EINVAL, "unknown rule");
    if (o.averaging != CFR_AVG_LINEAR && o.averaging != CFR_AVG_UNIFORM) return fail(CFR_EINVAL, "unknown averaging");
    if (o.order != CFR_ORDER_SIMULTANEOUS && o.order != CFR_ORDER_ALTERNATING) return fail(CFR_EINVAL, "unknown order");
    if (o.layout != CFR_LAYOUT_BFS && o.layout != CFR_LAYOUT_PUBLIC) return fail(CFR_EINVAL, "unknown layout");
    if (o.iters_per_graph < 1 || o.iters_per_graph > 1000) return fail(CFR_EINVAL, "iters_per_graph must be in [1, 1000]");
    if (o.precision != CFR_PRECISION_FP32 && o.precision != CFR_PRECISION_FP64) return fail(CFR_EINVAL, "unknown precision");
    if (o.persistent < CFR_SCHEDULE_LEVEL || o.persistent > CFR_SCHEDULE_LDS) return fail(CFR_EINVAL, "unknown schedule");
    if (o.group_sets != 0 && o.group_sets != 128 && o.group_sets != GROUP_SETS_MAX)
        return fail(CFR_EINVAL, "group_sets must be 0, 128 or 256");
    std::string err;
    cfr_status st = CFR_OK;
    // canonical layouts first: the update groups of every game are sized for the batch's action bound
    std::vector<Layout> Ls((size_t)n);
    int64_t N = 0, E = 0, Z = 0, Ndec = 0, I = 0, A = 0;
    int max_actions = 0, max_depth = 0, blocks = 0;
    std::vector<int32_t> canon_off;
    std::vector<int8_t> canon_player;
    std::vector<int64_t> hand_off{0};
    std::vector<int32_t> hand1, hand2, nh1, nh2;
    // the games of a batch compile independently: their canonical layouts on several host threads
    std::vector<cfr_status> sts((size_t)n, CFR_OK);
    std::vector<std::string> errs((size_t)n);
    for (int s = 0; s < n; s++) Ls[s].keep_maps = o.lifecycle != 0;
    parallel_games(n, [&](int s) {
        try {
            sts[s] = build_layout(&games[s], Ls[s], errs[s]);
        } catch (...) {
            sts[s] = CFR_ENOMEM;
            errs[s] = "host compile failed";
        }
    });
    for (int s = 0; s < n; s++) {
        st = sts[s];
        if (st != CFR_OK) return fail(st, n > 1 ? "game " + std::to_string(s) + ": " + errs[s] : errs[s]);
        const cfr_game_desc &gd = games[s];
        if (gd.root_hand1 || gd.root_hand2) {
            const std::string pre = n > 1 ? "game " + std::to_string(s) + ": " : "";
            if (!gd.root_hand1 || !gd.root_hand2) return fail(CFR_EINVAL, pre + "root_hand1 and root_hand2 go together");
            if (gd.node_type[gd.root] != CFR_NODE_CHANCE)
                return fail(CFR_EINVAL, pre + "a root hand map needs a chance root");
            if (gd.num_hands1 <= 0 || gd.num_hands2 <= 0) return fail(CFR_EINVAL, pre + "num_hands1/2 must be positive");
            for (int32_t a = 0; a < gd.num_children[gd.root]; a++) {
                const int32_t x = gd.root_hand1[a], y = gd.root_hand2[a];
                if (x < 0 || x >= gd.num_hands1 || y < 0 || y >= gd.num_hands2)
                    return fail(CFR_EINVAL, pre + "root hand index out of range at root child " + std::to_string(a));
                hand1.push_back(x);
                hand2.push_back(y);
            }
            nh1.push_back(gd.num_hands1);
            nh2.push_back(gd.num_hands2);
        } else {
            nh1.push_back(0);
            nh2.push_back(0);
        }
        hand_off.push_back((int64_t)hand1.size());
        if (!Ls[s].br_ok)
            return fail(CFR_EUNSUPPORTED, "an information set has members at different depths; the level-fused "
                                          "update needs every set on one depth");
        for (int64_t i = 0; i < Ls[s].I; i++) {
            canon_off.push_back((int32_t)(A + Ls[s].slot_off[(size_t)i]));
            canon_player.push_back(Ls[s].iset_player[(size_t)i]);
        }
        N += Ls[s].N; E += Ls[s].E; Z += Ls[s].Z; Ndec += Ls[s].Ndec; I += Ls[s].I; A += Ls[s].A;
        max_actions = std::max(max_actions, Ls[s].max_actions);
        max_depth = std::max(max_depth, Ls[s].max_depth);
        blocks = std::max(blocks, Ls[s].D);
    }
    if (N > 0x7fffffffLL || A > (1LL << 28)) return fail(CFR_EINVAL, "batch too large");
    canon_off.push_back((int32_t)A);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(CFR_EDEVICE, "no HIP device available");
    if (o.device < 0 || o.device >= ndev) return fail(CFR_EINVAL, "device ordinal out of range");
    HIP_TRY(hipSetDevice(o.device));

    DeviceLayout DL;
    LifecycleHost lc;
    std::vector<Layout> kept;
    {
        std::vector<DeviceLayout> Ds((size_t)n);
        parallel_games(n, [&](int s) {
            try {
                sts[s] = build_device_layout(Ls[s], o.layout, max_actions, o.precision == CFR_PRECISION_FP64,
                                             o.group_sets, Ds[s], errs[s]);
            } catch (...) {
                sts[s] = CFR_ENOMEM;
                errs[s] = "host compile failed";
            }
        });
        for (int s = 0; s < n; s++) {
            if (sts[s] != CFR_OK) return fail(sts[s], n > 1 ? "game " + std::to_string(s) + ": " + errs[s] : errs[s]);
            if (o.lifecycle) lifecycle_records(games[s], Ls[s], Ds[s], lc);
            if (n > 1 && !o.keep_layout) Ls[s] = Layout();  // free the canonical arrays early
        }
        if (n > 1 && o.group_sets == 0) {
            // one set bound for the batch, chosen from its group counts as a whole
            int64_t g128 = 0, g256 = 0;
            for (int s = 0; s < n; s++) {
                g128 += Ds[s].groups_by_bound[0];
                g256 += Ds[s].groups_by_bound[1];
            }
            const int32_t gs = choose_group_sets(g128, g256);
            for (int s = 0; s < n; s++) {
                if (Ds[s].group_sets == gs) continue;
                st = set_update_groups(Ds[s], gs, err);
                if (st != CFR_OK) return fail(st, "game " + std::to_string(s) + ": " + err);
            }
        }
        if (o.keep_layout) kept.swap(Ls);   // the merge releases the canonical arrays it is given
        st = build_forest(Ls, Ds, DL, err);
        if (st != CFR_OK) return fail(st, err);
    }
    if (o.lifecycle && n > 1) {
        // device ids of each game -> forest ids: the game's depth-d nodes start at its range lo
        const int MD = max_depth;
        for (int s = 0; s < n; s++)
            for (int64_t j = lc.term_off[s]; j < lc.term_off[s + 1]; j++) {
                const int d = lc.depth[(size_t)j];
                const int32_t lo = DL.game_range[((size_t)s * (MD + 1) + d) * GR_FIELDS];
                lc.node[(size_t)j] = lo + (lc.node[(size_t)j] - lc.depth_off[s][(size_t)d]);
            }
    }
    cfr_handle *h = new cfr_handle();
    h->opt = o;
    h->use_graph = o.use_graph != 0;
    h->depth_off = DL.depth_off;
    h->int_end = DL.int_end;
    h->iset_depth_off = DL.iset_depth_off;
    h->slot_map = DL.slot_canon_to_dev;
    h->grp_depth_off = DL.grp_depth_off;
    h->chance_off = DL.chance_off;
    h->bigc_off = DL.bigc_off;
    h->n_games = DL.n_games;
    h->game_slot_base = DL.game_slot_base;
    h->game_depth = DL.game_depth;
    h->game_range = DL.game_range;
    for (int s = 0; s < n; s++) h->game_pot.push_back(games[s].pot);
    h->lc_hand_off = std::move(hand_off);
    h->lc_hand1 = std::move(hand1);
    h->lc_hand2 = std::move(hand2);
    h->lc_nh1 = std::move(nh1);
    h->lc_nh2 = std::move(nh2);
    h->D = blocks;
    h->br_ok = true;
    h->E = E; h->Z = Z; h->pot = games[0].pot;
    DevGame &g = h->g;
    g.N = (int32_t)N; g.I = (int32_t)I; g.A = (int32_t)A; g.Ndec = (int32_t)Ndec;
    g.max_depth = max_depth; g.max_actions = max_actions;
    g.fp64 = o.precision == CFR_PRECISION_FP64 ? 1 : 0;
    g.rule = o.rule;
    g.explicit_kids = DL.explicit_kids ? 1 : 0;
    h->es = g.fp64 ? 8 : 4;
    std::vector<int32_t> koff;
    g.affine = o.affine && slot_child_offsets(DL, koff) ? 1 : 0;
    g.group_sets = DL.group_sets;

    std::vector<int2> up((size_t)N);
    for (int64_t k = 0; k < N; k++) up[k] = make_int2(DL.up_parent[k], DL.up_code[k]);
    DL.up_parent = std::vector<int32_t>();
    DL.up_code = std::vector<int32_t>();

#define ALLOC(ptr, cnt) do { st = dev_alloc(h, &(ptr), (cnt)); if (st != CFR_OK) { free_handle(h); return st; } } while (0)
    ALLOC(g.up, N);
    ALLOC(g.kid_off, N + 1);
    if (g.explicit_kids) ALLOC(g.kid, E);
    if (!h->slot_map.empty()) ALLOC(g.slot_map, A);
    ALLOC(g.node_slot, N);
    ALLOC(g.node_iset, N);
    ALLOC(g.slot_off, I + 1);
    ALLOC(g.mem_off, I + 1);
    ALLOC(g.mem, Ndec);
    if (g.affine) {
        ALLOC(g.koff, A > 0 ? A : 1);
        ALLOC(g.mnode, Ndec > 0 ? Ndec : 1);
        ALLOC(g.mpos, Ndec > 0 ? Ndec : 1);
        ALLOC(g.grp_perm, std::max<int64_t>((int64_t)DL.grp_iset_off.size() - 1, 1));
    }
    ALLOC(g.iset_player, I);
    g.G = (int32_t)DL.grp_iset_off.size() - 1;
    ALLOC(g.grp_iset_off, (int64_t)DL.grp_iset_off.size());
    ALLOC(g.chance_node, (int64_t)DL.chance_node.size());
    ALLOC(g.bigc_node, (int64_t)DL.bigc_node.size());
    g.grp_depth_off = h->grp_depth_off.data();
    g.chance_off = h->chance_off.data();
    g.bigc_off = h->bigc_off.data();
    {
        char *pv = nullptr, *pr = nullptr, *ps = nullptr, *pR = nullptr;
        ALLOC(pv, N * (int64_t)h->es);
        ALLOC(pr, 2 * N * (int64_t)h->es);
        ALLOC(ps, (A > 0 ? A : 1) * (int64_t)h->es);
        ALLOC(pR, (A > 0 ? A : 1) * (int64_t)h->es);
        g.v = pv; g.reach = pr; g.sigma = ps; g.R = pR;
        if (o.rule == CFR_RULE_PCFR_PLUS) {
            char *pp = nullptr;
            ALLOC(pp, (A > 0 ? A : 1) * (int64_t)h->es);
            g.pred = pp;
        }
    }
    ALLOC(g.sbar, A);
    ALLOC(g.t, 1);
    ALLOC(g.vbr, N);
    ALLOC(g.qbr, N);
    ALLOC(g.sigbar, A);
    ALLOC(g.astar, I);
    ALLOC(g.out, A);
    ALLOC(g.out2, A);
    ALLOC(h->canon_off, I + 1);
    ALLOC(h->canon_player, I);
    ALLOC(h->warm_mag, I);
#undef ALLOC
    h->I_canon = I;
    h->R_base = (char *)g.R; h->sbar_base = (char *)g.sbar; h->sigma_base = (char *)g.sigma;
#define UP(dst, src) do { st = upload(dst, src); if (st != CFR_OK) { free_handle(h); return st; } } while (0)
    UP(g.up, up);
    UP(g.kid_off, DL.kid_off);
    if (g.explicit_kids) UP(g.kid, DL.kid);
    if (g.slot_map) UP(g.slot_map, h->slot_map);
    UP(g.node_slot, DL.node_slot);
    UP(g.node_iset, DL.node_iset);
    UP(g.slot_off, DL.slot_off);
    UP(g.mem_off, DL.mem_off);
    {
        std::vector<int2> mem((size_t)Ndec);
        for (int64_t k = 0; k < Ndec; k++)
            mem[k] = make_int2(DL.mem_node[k], DL.kid_off[DL.mem_node[k] & MEMBER_NODE_MASK]);
        UP(g.mem, mem);
    }
    if (g.affine) {
        UP(g.koff, koff);
        std::vector<int32_t> mnode;
        std::vector<uint16_t> mpos;
        std::vector<int8_t> perm;
        member_lists(DL, mnode, mpos, perm, h->perm_members);
        for (int8_t f : perm) h->node_order_groups += f;
        for (double m : h->perm_members) h->node_order_members += (int64_t)m;
        UP(g.mnode, mnode);
        UP(g.mpos, mpos);
        UP(g.grp_perm, perm);
    }
    UP(g.iset_player, DL.iset_player);
    UP(g.grp_iset_off, DL.grp_iset_off);
    UP(g.chance_node, DL.chance_node);
    UP(g.bigc_node, DL.bigc_node);
    if (DL.n_games > 1) {
        // the first and last game of every forward tile (BLOCK * 4 nodes of one depth) and room for the
        // lists of the work that still runs once games retire (cfr_set_active)
        const int ng = DL.n_games, MD = (int)DL.depth_off.size() - 2;
        auto range = [&](int s_, int d, int f) { return DL.game_range[((size_t)s_ * (MD + 1) + d) * GR_FIELDS + f]; };
        constexpr int32_t TILE = 1024;   // k_forward's nodes per workgroup
        h->fwd_tile_base.assign((size_t)MD + 2, 0);
        h->fwd_games.clear();
        for (int d = 0; d <= MD; d++) {
            h->fwd_tile_base[(size_t)d] = (int64_t)h->fwd_games.size();
            const int32_t lo = DL.depth_off[(size_t)d], hi = DL.int_end[(size_t)d];
            int s_ = 0;
            for (int32_t a0 = lo; a0 < hi; a0 += TILE) {
                const int32_t a1 = std::min(hi, a0 + TILE) - 1;
                while (s_ + 1 < ng && range(s_, d, 1) <= a0) s_++;
                int e_ = s_;
                while (e_ + 1 < ng && range(e_, d, 1) <= a1) e_++;
                h->fwd_games.push_back(make_int2(s_, e_));
            }
        }
        h->fwd_tile_base[(size_t)MD + 1] = (int64_t)h->fwd_games.size();
        h->active.assign((size_t)ng, 1);
        for (auto *v : {&h->fwd_off, &h->grp_off, &h->chance_off_l, &h->bigc_off_l}) v->assign((size_t)MD + 2, 0);
#define BA(ptr, cnt) do { st = dev_alloc(h, &(ptr), (cnt)); if (st != CFR_OK) { free_handle(h); return st; } } while (0)
        BA(g.fwd_list, std::max<int64_t>((int64_t)h->fwd_games.size(), 1));
        BA(g.grp_list, std::max<int64_t>(g.G, 1));
        BA(g.chance_list, std::max<int64_t>((int64_t)DL.chance_node.size(), 1));
        BA(g.bigc_list, std::max<int64_t>((int64_t)DL.bigc_node.size(), 1));
#undef BA
        g.fwd_off = h->fwd_off.data();
        g.grp_off = h->grp_off.data();
        g.chance_off_l = h->chance_off_l.data();
        g.bigc_off_l = h->bigc_off_l.data();
    }
    UP(h->canon_off, canon_off);
    UP(h->canon_player, canon_player);
    if (o.lifecycle) {
        const int64_t nt = (int64_t)lc.node.size(), nr = (int64_t)lc.root.size();
        int64_t maxn = 1;
        for (int64_t v : lc.nodes) maxn = std::max(maxn, v);
#define LA(ptr, cnt) do { st = dev_alloc(h, &(ptr), (cnt)); if (st != CFR_OK) { free_handle(h); return st; } } while (0)
        LA(h->lc_node, nt); LA(h->lc_in, nt); LA(h->lc_branch, nt); LA(h->lc_u, nt); LA(h->lc_pic, nt);
        LA(h->lc_root, nr); LA(h->lc_stage, maxn);
#undef LA
        UP(h->lc_node, lc.node); UP(h->lc_in, lc.in); UP(h->lc_branch, lc.branch); UP(h->lc_u, lc.u);
        UP(h->lc_pic, lc.pic); UP(h->lc_root, lc.root);
        h->lc_term_off = lc.term_off;
        h->lc_root_off = lc.root_off;
        h->lc_nodes = lc.nodes;
    }
    if (g.fp64) { UP((double *)g.v, DL.tmpl64); } else { UP((float *)g.v, DL.tmpl); }
    UP(g.vbr, DL.tmpl64);
    {
        // roots (the first n nodes) have reach 1 in both lanes and in the best-response lane;
        // written once, never overwritten
        std::vector<float> onef((size_t)n, 1.0f);
        std::vector<double> oned((size_t)n, 1.0);
        char *r = (char *)g.reach;
        const void *src = g.fp64 ? (const void *)oned.data() : (const void *)onef.data();
        hipError_t e = hipMemcpy(r, src, h->es * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(r + N * (int64_t)h->es, src, h->es * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(g.qbr, oned.data(), sizeof(double) * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) { free_handle(h); return fail(CFR_EDEVICE, std::string("setup: ") + hipGetErrorString(e)); }
    }
#undef UP
    build_plan(h);
    h->launches = (int64_t)h->plan.size();
    model_bytes(h, DL);
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, o.device) == hipSuccess) h->device_name = prop.gcnArchName;
    }
    if (o.persistent != CFR_SCHEDULE_LEVEL) {
        st = cfr_set_schedule(h, o.persistent, o.wg_nodes);
        if (st != CFR_OK) { free_handle(h); return st; }
    }
    st = cfr_reset(h);
    if (st != CFR_OK) { free_handle(h); return st; }
    if (o.keep_layout) h->layouts = std::move(kept);
    *out = h;
    return CFR_OK;
}

cfr_status cfr_compile(const cfr_game_desc *game, const cfr_options *opt, cfr_handle **out) {
    if (!game) return fail(CFR_EINVAL, "game description is NULL");
    return compile_games(game, 1, opt, out);
}

cfr_status cfr_compile_batch(const cfr_game_desc *games, int32_t n, const cfr_options *opt, cfr_handle **out) {
    return compile_games(games, n, opt, out);
}

cfr_status cfr_batch_size(cfr_handle *h, int32_t *n_games, int64_t *slot_base) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (n_games) *n_games = h->n_games;
    if (slot_base)
        for (int s = 0; s <= h->n_games; s++) slot_base[s] = h->game_slot_base[(size_t)s];
    return CFR_OK;
}

cfr_status cfr_reset(cfr_handle *h) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    HIP_TRY(hipSetDevice(h->opt.device));
    // iterations may still be queued on a caller's stream: finish them before clearing
    HIP_TRY(hipDeviceSynchronize());
    const DevGame &g = h->g;
    hipStream_t s = h->cap_stream;
    HIP_TRY(hipMemsetAsync(g.R, 0, (size_t)(g.A > 0 ? g.A : 1) * h->es, s));
    if (g.pred) HIP_TRY(hipMemsetAsync(g.pred, 0, (size_t)(g.A > 0 ? g.A : 1) * h->es, s));
    HIP_TRY(hipMemsetAsync(g.sbar, 0, (size_t)(g.A > 0 ? g.A : 1) * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(g.t, 0, sizeof(int32_t), s));
    if (h->pp.err) HIP_TRY(hipMemsetAsync(h->pp.err, 0, sizeof(int32_t), s));
    if (h->any_inactive) {
        // a fresh solve iterates every game again (the graphs are captured anew)
        h->active.assign(h->active.size(), 1);
        h->any_inactive = false;
        h->g.use_lists = 0;
        drop_graphs(h);
    }
    HIP_TRY(launch_regret_matching(g, s));
    HIP_TRY(hipStreamSynchronize(s));
    h->iters = 0;
    h->broken = false;
    return CFR_OK;
}

cfr_status cfr_set_active(cfr_handle *h, const uint8_t *active, int32_t n, void *stream) {
    if (!h || !active) return fail(CFR_EINVAL, "NULL argument");
    if (n != h->n_games) return fail(CFR_EINVAL, "n must equal the number of games " + std::to_string(h->n_games));
    if (h->n_games == 1) {
        if (!active[0]) return fail(CFR_EUNSUPPORTED, "a single game cannot be retired (do not iterate it)");
        return CFR_OK;
    }
    bool any = false;
    for (int32_t s_ = 0; s_ < n; s_++) any |= active[s_] == 0;
    if (any && (h->persistent || h->lds))
        return fail(CFR_EUNSUPPORTED, "retiring games needs the level-synchronous schedule (cfr_set_schedule)");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    // queued iterations read the lists and graphs replaced below
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipDeviceSynchronize());
    for (int32_t s_ = 0; s_ < n; s_++) h->active[(size_t)s_] = active[s_] ? 1 : 0;
    if (any) {
        // per depth, the forward tiles with an active game and the active games' update groups, chance
        // nodes and big chance nodes
        const int MD = (int)h->fwd_off.size() - 2;
        const int ng = h->n_games;
        auto range = [&](int s_, int d, int f) { return h->game_range[((size_t)s_ * (MD + 1) + d) * GR_FIELDS + f]; };
        std::vector<int32_t> fl, gl, cl, bl;
        for (int d = 0; d <= MD; d++) {
            h->fwd_off[(size_t)d] = (int64_t)fl.size();
            h->grp_off[(size_t)d] = (int64_t)gl.size();
            h->chance_off_l[(size_t)d] = (int64_t)cl.size();
            h->bigc_off_l[(size_t)d] = (int64_t)bl.size();
            for (int64_t t = h->fwd_tile_base[(size_t)d]; t < h->fwd_tile_base[(size_t)d + 1]; t++) {
                const int2 gr = h->fwd_games[(size_t)t];
                bool on = false;
                for (int q = gr.x; q <= gr.y && !on; q++) on = h->active[(size_t)q] != 0;
                if (on) fl.push_back((int32_t)(t - h->fwd_tile_base[(size_t)d]));
            }
            for (int s_ = 0; s_ < ng; s_++) {
                if (!h->active[(size_t)s_]) continue;
                for (int32_t x = range(s_, d, 2); x < range(s_, d, 3); x++) gl.push_back(x);
                for (int32_t x = range(s_, d, 4); x < range(s_, d, 5); x++) cl.push_back(x);
                for (int32_t x = range(s_, d, 6); x < range(s_, d, 7); x++) bl.push_back(x);
            }
        }
        h->fwd_off[(size_t)MD + 1] = (int64_t)fl.size();
        h->grp_off[(size_t)MD + 1] = (int64_t)gl.size();
        h->chance_off_l[(size_t)MD + 1] = (int64_t)cl.size();
        h->bigc_off_l[(size_t)MD + 1] = (int64_t)bl.size();
        if (!fl.empty()) HIP_TRY(hipMemcpy(h->g.fwd_list, fl.data(), fl.size() * 4, hipMemcpyHostToDevice));
        if (!gl.empty()) HIP_TRY(hipMemcpy(h->g.grp_list, gl.data(), gl.size() * 4, hipMemcpyHostToDevice));
        if (!cl.empty()) HIP_TRY(hipMemcpy(h->g.chance_list, cl.data(), cl.size() * 4, hipMemcpyHostToDevice));
        if (!bl.empty()) HIP_TRY(hipMemcpy(h->g.bigc_list, bl.data(), bl.size() * 4, hipMemcpyHostToDevice));
    }
    if (any || h->any_inactive) drop_graphs(h);   // the launch shapes change: capture again
    h->g.use_lists = any ? 1 : 0;
    h->any_inactive = any;
    return CFR_OK;
}

cfr_status cfr_iterate(cfr_handle *h, int64_t n, void *stream) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (n < 0) return fail(CFR_EINVAL, "n must be >= 0");
    if (n == 0) return CFR_OK;
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    if (h->broken) return fail(CFR_ESTATE, "a persistent launch stopped part-way; call cfr_reset first");
    if (h->any_inactive && (h->persistent || h->lds))
        return fail(CFR_ESTATE, "retired games need the level-synchronous schedule; reactivate them first");
    if (h->persistent || h->lds) return persistent_iterate(h, n, s);
    if (h->captured && h->pinned != persistent_ptrs(h))
        return fail(CFR_ESTATE, "a persistent buffer changed since graph capture; refusing to replay");
    if (!h->use_graph) {
        for (int64_t k = 0; k < n; k++) {
            cfr_status st = enqueue_iteration(h, s, nullptr);
            if (st != CFR_OK) return st;
            h->iters++;
        }
        return CFR_OK;
    }
    if (!h->captured) {
        // one direct iteration first (loads every kernel), then capture
        cfr_status st = enqueue_iteration(h, s, nullptr);
        if (st != CFR_OK) return st;
        h->iters++;
        n--;
        if (h->opt.test_fail_capture) st = fail(CFR_EGRAPH, "capture failure injected by test hook");
        else st = capture(h, 1, &h->graph1, &h->exec1);
        if (st == CFR_OK && h->opt.iters_per_graph > 1) st = capture(h, h->opt.iters_per_graph, &h->graphk, &h->execk);
        if (st != CFR_OK) {
            if (!h->warned) {
                std::fprintf(stderr, "cfr: graph capture failed (%s); launching the same kernels directly\n",
                             g_err.c_str());
                h->warned = true;
            }
            h->use_graph = false;
            return cfr_iterate(h, n, stream);
        }
        h->captured = true;
        h->pinned = persistent_ptrs(h);
    }
    const int64_t k = h->opt.iters_per_graph;
    while (k > 1 && n >= k) {
        hipError_t e = hipGraphLaunch(h->execk, s);
        if (e != hipSuccess) return fail(CFR_EGRAPH, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        h->iters += k;
        n -= k;
    }
    for (; n > 0; n--) {
        hipError_t e = hipGraphLaunch(h->exec1, s);
        if (e != hipSuccess) return fail(CFR_EGRAPH, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        h->iters++;
    }
    return CFR_OK;
}

cfr_status cfr_iterations(cfr_handle *h, int64_t *t) {
    if (!h || !t) return fail(CFR_EINVAL, "NULL argument");
    *t = h->iters;
    return CFR_OK;
}

cfr_status cfr_strategy(cfr_handle *h, int which, float *dst, int64_t len, int dst_on_device, void *stream) {
    if (!h || (!dst && len > 0)) return fail(CFR_EINVAL, "NULL argument");
    if (len != h->g.A) return fail(CFR_EINVAL, "len must equal the slot count " + std::to_string(h->g.A));
    if (which != CFR_STRATEGY_CURRENT && which != CFR_STRATEGY_AVERAGE) return fail(CFR_EINVAL, "unknown strategy kind");
    if (len == 0) return CFR_OK;
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    const float *src = h->g.out;
    if (which == CFR_STRATEGY_AVERAGE) {
        HIP_TRY(launch_average(h->g, s));                    // device order into out2
        HIP_TRY(launch_gather_float(h->g, h->g.out2, h->g.out, s));
    } else {
        HIP_TRY(launch_sigma_to_float(h->g, h->g.out, s));   // gathers into canonical order
    }
    HIP_TRY(hipMemcpyAsync(dst, src, (size_t)len * sizeof(float),
                           dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!dst_on_device) HIP_TRY(hipStreamSynchronize(s));
    return CFR_OK;
}

cfr_status cfr_get_state(cfr_handle *h, double *regrets, double *strategy_sum, int64_t len, void *stream) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (len != h->g.A) return fail(CFR_EINVAL, "len must equal the slot count " + std::to_string(h->g.A));
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    if (len == 0) return CFR_OK;
    std::vector<double> rd((size_t)len), sd((size_t)len);
    std::vector<float> rf;
    if (regrets) {
        if (h->g.fp64) {
            HIP_TRY(hipMemcpyAsync(rd.data(), h->g.R, (size_t)len * 8, hipMemcpyDeviceToHost, s));
        } else {
            rf.resize((size_t)len);
            HIP_TRY(hipMemcpyAsync(rf.data(), h->g.R, (size_t)len * 4, hipMemcpyDeviceToHost, s));
        }
    }
    if (strategy_sum)
        HIP_TRY(hipMemcpyAsync(sd.data(), h->g.sbar, (size_t)len * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const bool ident = h->slot_map.empty();
    for (int64_t q = 0; q < len; q++) {
        const size_t dq = ident ? (size_t)q : (size_t)h->slot_map[(size_t)q];
        if (regrets) regrets[q] = h->g.fp64 ? rd[dq] : (double)rf[dq];
        if (strategy_sum) strategy_sum[q] = sd[dq];
    }
    return CFR_OK;
}

cfr_status cfr_set_regrets(cfr_handle *h, const float *r0, int64_t len, int src_on_device, void *stream) {
    if (!h || (!r0 && len > 0)) return fail(CFR_EINVAL, "NULL argument");
    if (len != h->g.A) return fail(CFR_EINVAL, "len must equal the slot count " + std::to_string(h->g.A));
    if (len == 0) return CFR_OK;
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(h->g.out, r0, (size_t)len * sizeof(float),
                           src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (h->g.pred) HIP_TRY(hipMemsetAsync(h->g.pred, 0, (size_t)len * h->es, s));
    HIP_TRY(launch_regrets_from_float(h->g, h->g.out, s));
    HIP_TRY(launch_regret_matching(h->g, s));
    if (!src_on_device) HIP_TRY(hipStreamSynchronize(s));
    return CFR_OK;
}

cfr_status cfr_set_state(cfr_handle *h, const double *regrets, const double *strategy_sum, const double *prediction,
                         int64_t len, int64_t t, void *stream) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (len != h->g.A) return fail(CFR_EINVAL, "len must equal the slot count " + std::to_string(h->g.A));
    if (t < 0 || t > 0x7fffffffLL) return fail(CFR_EINVAL, "t must be in [0, 2^31)");
    if (prediction && !h->g.pred) return fail(CFR_EINVAL, "only PCFR+ keeps a prediction");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    const DevGame &g = h->g;
    // every array goes through the FP64 evaluation scratch (sigbar, A doubles) and is scattered to
    // device slot order in the state type; the stream is synchronised before the staging is reused
    auto put = [&](const double *src, void *dst, bool state_type) -> cfr_status {
        HIP_TRY(hipMemcpyAsync(g.sigbar, src, (size_t)len * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(launch_scatter_double(g, g.sigbar, dst, state_type, s));
        HIP_TRY(hipStreamSynchronize(s));
        return CFR_OK;
    };
    cfr_status st = CFR_OK;
    if (len > 0) {
        if (regrets && (st = put(regrets, g.R, true)) != CFR_OK) return st;
        if (strategy_sum && (st = put(strategy_sum, g.sbar, false)) != CFR_OK) return st;
        if (g.pred) {
            if (prediction) {
                if ((st = put(prediction, g.pred, true)) != CFR_OK) return st;
            } else {
                HIP_TRY(launch_fill_state(g, g.pred, s));
            }
        }
    }
    const int32_t t32 = (int32_t)t;
    HIP_TRY(hipMemcpyAsync(g.t, &t32, sizeof t32, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_regret_matching(g, s));
    HIP_TRY(hipStreamSynchronize(s));
    h->iters = t;
    h->broken = false;
    return CFR_OK;
}

cfr_status cfr_get_game_state(cfr_handle *h, int32_t game, double *regrets, double *strategy_sum,
                              double *prediction, int64_t len, void *stream) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (game < 0 || game >= h->n_games) return fail(CFR_EINVAL, "game out of range");
    const int64_t b = h->game_slot_base[(size_t)game], e = h->game_slot_base[(size_t)game + 1];
    if (len != e - b) return fail(CFR_EINVAL, "len must equal the game's slot count " + std::to_string(e - b));
    if (prediction && !h->g.pred) return fail(CFR_EINVAL, "only PCFR+ keeps a prediction");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    if (len == 0) return CFR_OK;
    // the game's device slots, sorted, copied run by run (a game's sets are contiguous per depth)
    const bool ident = h->slot_map.empty();
    std::vector<int32_t> dev((size_t)len);
    for (int64_t q = b; q < e; q++) dev[(size_t)(q - b)] = ident ? (int32_t)q : h->slot_map[(size_t)q];
    std::vector<int32_t> sorted(dev);
    std::sort(sorted.begin(), sorted.end());
    const size_t es = h->es;
    std::vector<unsigned char> rb(regrets ? (size_t)len * es : 0), pb(prediction ? (size_t)len * es : 0);
    std::vector<double> sb(strategy_sum ? (size_t)len : 0);
    for (size_t k0 = 0; k0 < sorted.size();) {
        size_t k1 = k0 + 1;
        while (k1 < sorted.size() && sorted[k1] == sorted[k1 - 1] + 1) k1++;
        const size_t x0 = (size_t)sorted[k0], n = k1 - k0;
        if (regrets)
            HIP_TRY(hipMemcpyAsync(rb.data() + k0 * es, (const unsigned char *)h->g.R + x0 * es, n * es,
                                   hipMemcpyDeviceToHost, s));
        if (strategy_sum)
            HIP_TRY(hipMemcpyAsync(sb.data() + k0, h->g.sbar + x0, n * sizeof(double), hipMemcpyDeviceToHost, s));
        if (prediction)
            HIP_TRY(hipMemcpyAsync(pb.data() + k0 * es, (const unsigned char *)h->g.pred + x0 * es, n * es,
                                   hipMemcpyDeviceToHost, s));
        k0 = k1;
    }
    HIP_TRY(hipStreamSynchronize(s));
    auto val = [&](const std::vector<unsigned char> &v, size_t k) {
        if (h->g.fp64) { double x; std::memcpy(&x, v.data() + k * 8, 8); return x; }
        float x; std::memcpy(&x, v.data() + k * 4, 4); return (double)x;
    };
    for (int64_t q = 0; q < len; q++) {
        const size_t k = (size_t)(std::lower_bound(sorted.begin(), sorted.end(), dev[(size_t)q]) - sorted.begin());
        if (regrets) regrets[q] = val(rb, k);
        if (strategy_sum) strategy_sum[q] = sb[k];
        if (prediction) prediction[q] = val(pb, k);
    }
    return CFR_OK;
}

cfr_status cfr_get_prediction(cfr_handle *h, double *prediction, int64_t len, void *stream) {
    if (!h || (!prediction && len > 0)) return fail(CFR_EINVAL, "NULL argument");
    if (len != h->g.A) return fail(CFR_EINVAL, "len must equal the slot count " + std::to_string(h->g.A));
    if (!h->g.pred) return fail(CFR_EINVAL, "only PCFR+ keeps a prediction");
    if (len == 0) return CFR_OK;
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> pd((size_t)len);
    std::vector<float> pf;
    if (h->g.fp64) {
        HIP_TRY(hipMemcpyAsync(pd.data(), h->g.pred, (size_t)len * 8, hipMemcpyDeviceToHost, s));
    } else {
        pf.resize((size_t)len);
        HIP_TRY(hipMemcpyAsync(pf.data(), h->g.pred, (size_t)len * 4, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    const bool ident = h->slot_map.empty();
    for (int64_t q = 0; q < len; q++) {
        const size_t dq = ident ? (size_t)q : (size_t)h->slot_map[(size_t)q];
        prediction[q] = h->g.fp64 ? pd[dq] : (double)pf[dq];
    }
    return CFR_OK;
}

// Best responses of every game of the handle: vals[k][s] for k = best responder 1, 2 and the
// average-profile value (k = 0), read at each game's root.
static cfr_status best_responses(cfr_handle *h, hipStream_t s, std::vector<double> vals[3]) {
    if (!h->br_ok) return fail(CFR_EUNSUPPORTED, "an information set spans several depths; the level-synchronous best response needs one depth per set");
    HIP_TRY(hipSetDevice(h->opt.device));
    const DevGame &g = h->g;
    const int n = h->n_games;
    HIP_TRY(launch_average(g, s));
    const int order[3] = {1, 2, 0};
    for (int k = 0; k < 3; k++) {
        const int br = order[k];
        if (br != 0)
            for (int d = 1; d <= g.max_depth; d++) HIP_TRY(launch_br_forward(g, h->depth_off[d], h->int_end[d], br, s));
        for (int d = g.max_depth - 1; d >= 0; d--) {
            if (br != 0) HIP_TRY(launch_br_argmax(g, h->iset_depth_off[d], h->iset_depth_off[d + 1], br, s));
            HIP_TRY(launch_br_backward(g, h->depth_off[d], h->int_end[d], br, s));
        }
        vals[br].assign((size_t)n, 0.0);
        HIP_TRY(hipMemcpyAsync(vals[br].data(), g.vbr, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return CFR_OK;
}

cfr_status cfr_exploitability(cfr_handle *h, void *stream, double *expl, double *br1, double *br2,
                              double *value_avg) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (h->n_games != 1) return fail(CFR_EINVAL, "handle holds a batch; use cfr_batch_exploitability");
    std::vector<double> vals[3];
    cfr_status st = best_responses(h, (hipStream_t)stream, vals);
    if (st != CFR_OK) return st;
    double b1 = vals[1][0], b2 = -vals[2][0];
    if (br1) *br1 = b1;
    if (br2) *br2 = b2;
    if (value_avg) *value_avg = vals[0][0];
    if (expl) *expl = 0.5 * (b1 + b2);
    return CFR_OK;
}

cfr_status cfr_batch_exploitability(cfr_handle *h, void *stream, double *expl, double *br1, double *br2,
                                    double *value_avg, int32_t n) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (n != h->n_games) return fail(CFR_EINVAL, "n must equal the number of games " + std::to_string(h->n_games));
    std::vector<double> vals[3];
    cfr_status st = best_responses(h, (hipStream_t)stream, vals);
    if (st != CFR_OK) return st;
    for (int s = 0; s < n; s++) {
        const double b1 = vals[1][(size_t)s], b2 = -vals[2][(size_t)s];
        if (br1) br1[s] = b1;
        if (br2) br2[s] = b2;
        if (value_avg) value_avg[s] = vals[0][(size_t)s];
        if (expl) expl[s] = 0.5 * (b1 + b2);
    }
    return CFR_OK;
}

cfr_status cfr_counts(cfr_handle *h, cfr_counts_t *c) {
    if (!h || !c) return fail(CFR_EINVAL, "NULL argument");
    std::memset(c, 0, sizeof *c);
    c->nodes = h->g.N; c->edges = h->E; c->terminals = h->Z; c->decision_nodes = h->g.Ndec;
    c->infosets = h->g.I; c->slots = h->g.A; c->max_depth = h->g.max_depth; c->blocks = h->D;
    c->max_actions = h->g.max_actions; c->br_supported = h->br_ok ? 1 : 0;
    c->device_bytes = h->device_bytes; c->kernels_per_iteration = h->launches; c->pot = h->pot;
    c->child_addressing = h->g.affine ? 2 : h->g.explicit_kids ? 1 : 0;
    c->node_order_groups = h->node_order_groups;
    c->node_order_members = h->node_order_members;
    c->group_sets = h->g.group_sets;
    c->update_groups = h->g.G;
    return CFR_OK;
}

cfr_status cfr_profile(cfr_handle *h, int64_t n, void *stream, cfr_kernel_stat *out, int32_t max_out,
                       int32_t *n_out) {
    if (!h || !out || !n_out || n <= 0 || max_out < 0) return fail(CFR_EINVAL, "bad argument");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    LaunchTimer tm;
    tm.ev.resize((size_t)(2 * h->launches * n + 2));
    for (auto &e : tm.ev) HIP_TRY(hipEventCreate(&e));
    cfr_status st = CFR_OK;
    for (int64_t k = 0; k < n && st == CFR_OK; k++) {
        st = enqueue_iteration(h, s, nullptr, &tm);
        if (st == CFR_OK) h->iters++;
    }
    hipError_t e = hipStreamSynchronize(s);
    double ms[4] = {0, 0, 0, 0};
    int64_t cnt[4] = {0, 0, 0, 0};
    if (st == CFR_OK && e == hipSuccess) {
        for (size_t i = 0; i + 1 < tm.next; i += 2) {
            float x = 0.0f;
            e = hipEventElapsedTime(&x, tm.ev[i], tm.ev[i + 1]);
            if (e != hipSuccess) break;
            ms[tm.cls[i]] += x;
            cnt[tm.cls[i]]++;
        }
    }
    for (auto &ev : tm.ev) (void)hipEventDestroy(ev);
    if (st != CFR_OK) return st;
    if (e != hipSuccess) return fail(CFR_EDEVICE, std::string("profiling events: ") + hipGetErrorString(e));
    const char *names[4] = {"k_tick", "k_forward", "k_level", ""};
    const double bytes[4] = {0.0, h->bytes_fwd, h->bytes_lvl, 0.0};
    const double method[4] = {0.0, h->method_fwd, h->method_lvl, 0.0};
    int32_t k = 0;
    for (int c = 0; c < 4; c++) {
        if (cnt[c] == 0) continue;
        if (k < max_out) {
            cfr_kernel_stat &o = out[k];
            std::memset(&o, 0, sizeof o);
            std::snprintf(o.name, sizeof o.name, "%s", names[c]);
            o.launches_per_iteration = cnt[c] / n;
            o.bytes_per_iteration = bytes[c];
            o.method_bytes_per_iteration = method[c];
            o.ms_per_iteration = ms[c] / (double)n;
        }
        k++;
    }
    *n_out = k < max_out ? k : max_out;
    return CFR_OK;
}

// The LDS-resident schedule: one game whose state fits in the device's LDS per workgroup and
// whose sets have at most 16 actions.
static cfr_status set_lds_schedule(cfr_handle *h) {
    if (h->n_games != 1) return fail(CFR_EINVAL, "the LDS schedule runs one standalone game, not a batch");
    size_t bytes = lds_schedule_bytes(h->g.N, h->g.A, h->g.fp64, h->g.pred != nullptr);
    int limit = 0;
    HIP_TRY(hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, h->opt.device));
    if (bytes > (size_t)limit)
        return fail(CFR_EINVAL, "the game needs " + std::to_string(bytes) + " bytes of LDS for the LDS schedule; "
                                "a workgroup has " + std::to_string(limit));
    if (prepare_lds(h->g, h->opt.rule, &bytes) != hipSuccess)
        return fail(CFR_EINVAL, "the LDS schedule supports at most 16 actions per information set");
    if (!h->lds_range) {
        cfr_status st = dev_alloc(h, &h->lds_range, (int64_t)h->game_range.size());
        if (st != CFR_OK) return st;
        st = upload(h->lds_range, h->game_range);
        if (st != CFR_OK) return st;
    }
    if (h->pexec) { (void)hipGraphExecDestroy(h->pexec); h->pexec = nullptr; }
    if (h->pgraph) { (void)hipGraphDestroy(h->pgraph); h->pgraph = nullptr; }
    h->pgraph_n = -1;
    return CFR_OK;
}

cfr_status cfr_persistent_plan_host(const int64_t *nodes, int32_t n, int32_t wg_nodes, int32_t max_w, int32_t *W,
                                    int32_t *queue, int32_t *q_off, int32_t *wg_nodes_used) {
    if (n < 0 || (n > 0 && (!nodes || !W || !queue)) || !q_off || !wg_nodes_used || max_w < 1)
        return fail(CFR_EINVAL, "bad argument");
    std::vector<int64_t> nv(nodes, nodes + n);
    for (int64_t x : nv)
        if (x < 0) return fail(CFR_EINVAL, "negative node count");
    PersistentWork P;
    std::string err;
    if (!plan_persistent(nv, wg_nodes, max_w, PERSISTENT_QUEUES, P, err)) return fail(CFR_EUNSUPPORTED, err);
    for (int s = 0; s < n; s++) {
        W[s] = P.W[(size_t)s];
        queue[s] = P.queue[(size_t)s];
    }
    for (int q = 0; q <= PERSISTENT_QUEUES; q++) q_off[q] = P.q_off[(size_t)q];
    *wg_nodes_used = P.wg_nodes;
    return CFR_OK;
}

cfr_status cfr_set_schedule(cfr_handle *h, int32_t persistent, int32_t wg_nodes) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (persistent < CFR_SCHEDULE_LEVEL || persistent > CFR_SCHEDULE_LDS) return fail(CFR_EINVAL, "unknown schedule");
    if (persistent != CFR_SCHEDULE_LEVEL && h->any_inactive)
        return fail(CFR_ESTATE, "some games are retired: the persistent and LDS schedules iterate every game");
    HIP_TRY(hipSetDevice(h->opt.device));
    HIP_TRY(hipDeviceSynchronize());
    if (persistent == CFR_SCHEDULE_PERSISTENT) {
        cfr_status st = build_persistent_plan(h, wg_nodes);
        if (st != CFR_OK) return st;
    } else if (persistent == CFR_SCHEDULE_LDS) {
        cfr_status st = set_lds_schedule(h);
        if (st != CFR_OK) return st;
    }
    h->persistent = persistent == CFR_SCHEDULE_PERSISTENT;
    h->lds = persistent == CFR_SCHEDULE_LDS;
    return CFR_OK;
}

static std::string tune_key(const cfr_handle *h) {
    return h->device_name + " fp" + (h->g.fp64 ? "64" : "32") + " games=" + std::to_string(h->n_games) +
           " nodes=" + std::to_string(h->g.N) + " slots=" + std::to_string(h->g.A) +
           " depth=" + std::to_string(h->g.max_depth);
}

cfr_status cfr_autotune(cfr_handle *h, int64_t iters, void *stream, const char *cache_path, cfr_tune_result *out) {
    if (!h || iters <= 0) return fail(CFR_EINVAL, "bad argument");
    if (h->any_inactive) return fail(CFR_ESTATE, "some games are retired: reactivate them (or cfr_reset) first");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    const std::string key = tune_key(h);
    cfr_tune_result best{};
    best.ms_per_iteration = -1.0;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[512];
            while (std::fgets(line, sizeof line, f)) {
                int pers = 0, wg = 0;
                double ms = 0;
                char k[400];
                if (std::sscanf(line, "%d %d %lf %399[^\n]", &pers, &wg, &ms, k) == 4 && key == k) {
                    best.persistent = pers; best.wg_nodes = wg; best.ms_per_iteration = ms;
                }
            }
            std::fclose(f);
        }
    }
    int candidates = 0, failed = 0;
    if (best.ms_per_iteration < 0) {
        std::vector<std::pair<int, int>> cand = {{CFR_SCHEDULE_LEVEL, 0}};
        for (int wg : {1024, 4096, 16384, 65536, 262144}) cand.push_back({CFR_SCHEDULE_PERSISTENT, wg});
        if (h->n_games == 1) cand.push_back({CFR_SCHEDULE_LDS, 0});   // skipped unless the game fits in LDS
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        int32_t last_wg = -1;
        for (auto c : cand) {
            cfr_status st = cfr_set_schedule(h, c.first, c.second);
            if (st != CFR_OK) continue;
            const bool pers = c.first == CFR_SCHEDULE_PERSISTENT;
            if (pers && h->pp.wg_nodes == last_wg) continue;  // same plan as the previous size
            if (pers) last_wg = h->pp.wg_nodes;
            st = cfr_iterate(h, iters, stream);            // warm-up (capture)
            if (st == CFR_OK) HIP_TRY(hipEventRecord(e0, s));
            if (st == CFR_OK) st = cfr_iterate(h, iters, stream);
            if (st == CFR_EDEVICE && pers) {
                // a per-game barrier of this launch shape timed out (its blocks were not all
                // resident): drop the candidate; the next plan build clears the error flag
                std::fprintf(stderr, "cfr: autotune dropped persistent schedule wg_nodes=%d (%s)\n", h->wg_nodes,
                             g_err.c_str());
                failed++;
                st = cfr_reset(h);   // the failed launch left a partial state behind
                if (st != CFR_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return st; }
                continue;
            }
            if (st != CFR_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return st; }
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            const double per = ms / (double)iters;
            candidates++;
            if (best.ms_per_iteration < 0 || per < best.ms_per_iteration) {
                best.persistent = c.first; best.wg_nodes = pers ? h->wg_nodes : 0; best.ms_per_iteration = per;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (best.ms_per_iteration < 0) return fail(CFR_EDEVICE, "no schedule could run");
        if (cache_path) {
            if (FILE *f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "%d %d %.6f %s\n", best.persistent, best.wg_nodes, best.ms_per_iteration, key.c_str());
                std::fclose(f);
            }
        }
    }
    cfr_status st = cfr_set_schedule(h, best.persistent, best.wg_nodes);
    if (st != CFR_OK) return st;
    st = cfr_reset(h);
    if (st != CFR_OK) return st;
    best.blocks = h->persistent ? h->pp.blocks : h->lds ? 1 : 0;
    best.candidates = candidates;
    best.failed = failed;
    if (out) *out = best;
    return CFR_OK;
}

cfr_status cfr_debug_rebind(cfr_handle *h, int which, int64_t delta) {
    if (!h || which < 0 || which > 2) return fail(CFR_EINVAL, "bad argument");
    h->rebind[which] = delta;
    return CFR_OK;
}

static cfr_status lifecycle_check(cfr_handle *h, int32_t game) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (!h->lc_node) return fail(CFR_ESTATE, "compile with options.lifecycle = 1 to rewrite payoffs or root chance");
    if (game < 0 || game >= h->n_games) return fail(CFR_EINVAL, "game index out of range");
    return CFR_OK;
}

static cfr_status lifecycle_template(cfr_handle *h, int32_t game, hipStream_t s) {
    const int64_t lo = h->lc_term_off[(size_t)game], hi = h->lc_term_off[(size_t)game + 1];
    const bool has_root = h->lc_root_off[(size_t)game + 1] > h->lc_root_off[(size_t)game];
    HIP_TRY(launch_template(h->g, lo, hi, h->lc_node, h->lc_branch, h->lc_u, h->lc_pic,
                            has_root ? h->lc_root + h->lc_root_off[(size_t)game] : nullptr, s));
    return CFR_OK;
}

cfr_status cfr_set_payoffs(cfr_handle *h, int32_t game, const double *payoff, int64_t num_nodes, void *stream) {
    cfr_status st = lifecycle_check(h, game);
    if (st != CFR_OK) return st;
    if (!payoff) return fail(CFR_EINVAL, "payoff is NULL");
    if (num_nodes != h->lc_nodes[(size_t)game]) return fail(CFR_EINVAL, "num_nodes differs from the compiled game");
    for (int64_t k = 0; k < num_nodes; k++)
        if (!std::isfinite(payoff[k])) return fail(CFR_EINVAL, "non-finite payoff");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(h->lc_stage, payoff, (size_t)num_nodes * sizeof(double), hipMemcpyHostToDevice, s));
    const int64_t lo = h->lc_term_off[(size_t)game], hi = h->lc_term_off[(size_t)game + 1];
    HIP_TRY(launch_gather_payoffs(lo, hi, h->lc_in, h->lc_stage, h->lc_u, s));
    st = lifecycle_template(h, game, s);
    if (st != CFR_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));   // the staging buffer is reused by the next call
    return CFR_OK;
}

// Root chance of `game` <- prob[n] (validated by the caller) and the game's template rewritten.
static cfr_status write_root_chance(cfr_handle *h, int32_t game, const double *prob, int64_t n, hipStream_t s) {
    const int64_t r0 = h->lc_root_off[(size_t)game];
    HIP_TRY(hipSetDevice(h->opt.device));
    HIP_TRY(hipMemcpyAsync(h->lc_root + r0, prob, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    cfr_status st = lifecycle_template(h, game, s);
    if (st != CFR_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));
    return CFR_OK;
}

cfr_status cfr_set_root_chance(cfr_handle *h, int32_t game, const double *prob, int64_t n, void *stream) {
    cfr_status st = lifecycle_check(h, game);
    if (st != CFR_OK) return st;
    const int64_t r0 = h->lc_root_off[(size_t)game], r1 = h->lc_root_off[(size_t)game + 1];
    if (r1 == r0) return fail(CFR_EINVAL, "the game's root is not a chance node");
    if (!prob || n != r1 - r0) return fail(CFR_EINVAL, "prob must hold one probability per root child");
    double sum = 0.0;
    for (int64_t a = 0; a < n; a++) {
        if (!(prob[a] >= 0.0) || !std::isfinite(prob[a])) return fail(CFR_EINVAL, "invalid chance probability");
        sum += prob[a];
    }
    if (std::fabs(sum - 1.0) > 1e-9) return fail(CFR_EINVAL, "root chance probabilities do not sum to 1");
    return write_root_chance(h, game, prob, n, (hipStream_t)stream);
}

cfr_status cfr_set_root_ranges(cfr_handle *h, int32_t game, const double *r1, int64_t n1, const double *r2, int64_t n2,
                               void *stream) {
    cfr_status st = lifecycle_check(h, game);
    if (st != CFR_OK) return st;
    const int64_t k0 = h->lc_hand_off[(size_t)game], k1 = h->lc_hand_off[(size_t)game + 1];
    if (k1 == k0) return fail(CFR_ESTATE, "the game was compiled without a root hand map (root_hand1/root_hand2)");
    if (!r1 || !r2) return fail(CFR_EINVAL, "NULL range");
    if (n1 != h->lc_nh1[(size_t)game] || n2 != h->lc_nh2[(size_t)game])
        return fail(CFR_EINVAL, "range lengths must equal num_hands1 and num_hands2 of the description");
    for (int64_t i = 0; i < n1; i++)
        if (!(r1[i] >= 0.0) || !std::isfinite(r1[i])) return fail(CFR_EINVAL, "invalid range weight for player 1");
    for (int64_t i = 0; i < n2; i++)
        if (!(r2[i] >= 0.0) || !std::isfinite(r2[i])) return fail(CFR_EINVAL, "invalid range weight for player 2");
    // p(a) = r1(h1(a)) r2(h2(a)) / W, W the sum of the products over the root's children in child order
    const int64_t n = k1 - k0;
    std::vector<double> prob((size_t)n);
    double W = 0.0;
    for (int64_t a = 0; a < n; a++) W += r1[h->lc_hand1[(size_t)(k0 + a)]] * r2[h->lc_hand2[(size_t)(k0 + a)]];
    if (!(W > 0.0) || !std::isfinite(W)) return fail(CFR_EINVAL, "the ranges give no dealt pair a positive weight");
    for (int64_t a = 0; a < n; a++)
        prob[(size_t)a] = r1[h->lc_hand1[(size_t)(k0 + a)]] * r2[h->lc_hand2[(size_t)(k0 + a)]] / W;
    return write_root_chance(h, game, prob.data(), n, (hipStream_t)stream);
}

cfr_status cfr_num_infosets(cfr_handle *h, int64_t *count) {
    if (!h || !count) return fail(CFR_EINVAL, "NULL argument");
    *count = h->I_canon;
    return CFR_OK;
}

cfr_status cfr_features(cfr_handle *h, const int16_t *bucket, const int16_t *history, const float *scalars,
                        int32_t probe_iters, void *x, int64_t rows, void *stream) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (probe_iters < 0) return fail(CFR_EINVAL, "probe_iters must be >= 0");
    if (rows != h->I_canon) return fail(CFR_EINVAL, "rows must equal the information-set count " + std::to_string(h->I_canon));
    if (rows > 0 && (!bucket || !history || !scalars || !x)) return fail(CFR_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    const DevGame &g = h->g;
    auto clear = [&]() -> cfr_status {
        HIP_TRY(hipMemsetAsync(g.R, 0, (size_t)(g.A > 0 ? g.A : 1) * h->es, s));
        if (g.pred) HIP_TRY(hipMemsetAsync(g.pred, 0, (size_t)(g.A > 0 ? g.A : 1) * h->es, s));
        HIP_TRY(hipMemsetAsync(g.sbar, 0, (size_t)(g.A > 0 ? g.A : 1) * sizeof(double), s));
        HIP_TRY(hipMemsetAsync(g.t, 0, sizeof(int32_t), s));
        HIP_TRY(launch_regret_matching(g, s));
        return CFR_OK;
    };
    cfr_status st = clear();
    if (st != CFR_OK) return st;
    // one plain iteration from zero regrets: R becomes the instantaneous regrets of the uniform strategy
    const IterFlags plain{CFR_RULE_CFR, 0, 3};
    st = enqueue_iteration(h, s, nullptr, nullptr, &plain);
    if (st != CFR_OK) return st;
    FeatureArgs f{};
    f.canon_off = h->canon_off; f.player = h->canon_player; f.slot_map = g.slot_map;
    f.bucket = bucket; f.history = history; f.scalars = scalars; f.I = rows; f.X = (uint16_t *)x;
    f.mag = h->warm_mag;
    HIP_TRY(launch_features(f, g.R, g.fp64 != 0, s));
    st = clear();
    if (st != CFR_OK) return st;
    h->iters = 0;
    h->have_mag = true;
    if (probe_iters > 0) {
        // the first probe_iters iterations of the solve itself; their strategies become columns 120-127
        st = cfr_iterate(h, probe_iters, stream);
        if (st != CFR_OK) return st;
        HIP_TRY(launch_features_probe(f, g.sigma, g.sbar, g.fp64 != 0, s));
    }
    return CFR_OK;
}

cfr_status cfr_regret_unit(cfr_handle *h, float *unit, int64_t rows, void *stream) {
    if (!h) return fail(CFR_EINVAL, "handle is NULL");
    if (rows != h->I_canon) return fail(CFR_EINVAL, "rows must equal the information-set count " + std::to_string(h->I_canon));
    if (!h->have_mag) return fail(CFR_ESTATE, "call cfr_features first: it records the regret unit of every set");
    if (rows == 0) return CFR_OK;
    if (!unit) return fail(CFR_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(h->opt.device));
    HIP_TRY(hipMemcpyAsync(unit, h->warm_mag, (size_t)rows * sizeof(float), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return CFR_OK;
}

cfr_status cfr_warm_start(cfr_handle *h, cfr_mlp *n, const void *x, int64_t rows, float scale, int32_t add,
                          void *stream) {
    if (!h || !n) return fail(CFR_EINVAL, "NULL argument");
    if (rows != h->I_canon) return fail(CFR_EINVAL, "rows must equal the information-set count " + std::to_string(h->I_canon));
    if (mlp_in_dim(n) != CFR_FEATURES) return fail(CFR_EINVAL, "the network's in_dim must be CFR_FEATURES");
    if (mlp_device(n) != h->opt.device) return fail(CFR_EINVAL, "network and handle live on different devices");
    if (!(scale >= 0.f) || !std::isfinite(scale)) return fail(CFR_EINVAL, "scale must be finite and >= 0");
    if (rows > 0 && !x) return fail(CFR_EINVAL, "NULL argument");
    if (!h->have_mag) return fail(CFR_ESTATE, "call cfr_features first: it records the regret unit of every set");
    HIP_TRY(hipSetDevice(h->opt.device));
    hipStream_t s = (hipStream_t)stream;
    if (rows == 0) return CFR_OK;
    if (!h->warm_z) {
        cfr_status st = dev_alloc(h, &h->warm_z, rows * 4);
        if (st != CFR_OK) return st;
    }
    cfr_status st = mlp_forward_internal(n, x, rows, h->warm_z, s);
    if (st != CFR_OK) return st;
    HIP_TRY(launch_warm_regrets(h->canon_off, rows, h->warm_z, h->warm_mag, scale, h->g.out, s));
    if (add) {
        HIP_TRY(launch_regrets_add_float(h->g, h->g.out, s));
    } else {
        if (h->g.pred) HIP_TRY(hipMemsetAsync(h->g.pred, 0, (size_t)h->g.A * h->es, s));
        HIP_TRY(launch_regrets_from_float(h->g, h->g.out, s));
    }
    HIP_TRY(launch_regret_matching(h->g, s));
    return CFR_OK;
}

void cfr_destroy(cfr_handle *h) {
    if (!h) return;
    (void)hipSetDevice(h->opt.device);
    // work queued on any stream may still read the handle's buffers
    (void)hipDeviceSynchronize();
    free_handle(h);
}

}  // extern "C"
