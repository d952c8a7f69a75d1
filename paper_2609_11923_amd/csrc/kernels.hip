// kernels.hip -- gfx950 kernels of one compiled CFR iteration and of the FP64
// best-response evaluator.
//
// Iteration (paper Algorithm 'alg:iteration', Table 'tab:opsteps'):
//   forward  : per depth level, pi_i(c) = pi_i(parent) * (owner(parent) == i ? sigma(slot) : 1)
//              (eqs. reach, lanes; chance multiplies by 1 because its probabilities
//              live in the values template, eq. template)
//   backward : per depth level, v(h) = sum_children m(c) v(c), m = sigma(slot) below decisions,
//              1 below chance (eqs. cfv, opbwd); terminal entries of v hold the template and
//              are never overwritten, so no per-iteration template copy is needed
//   update   : per information set I of player i with members h,
//              r(I,a) = sum_h s_i pi_{-i}(h) (v(h.a) - v(h))         (eqs. regret, instregret)
//              R <- R + r, CFR+ clamps at 0; sbar += w_t pi_i(I) sigma^t (FP64, Prop. 4);
//              then sigma^{t+1} = regret matching of R (eq. rm) for the next iteration.
// The state type T (reach, values, regrets, strategy) is float -- the paper's
// configured dtype -- or double; strategy sums are double in both.  Every
// reduction runs in a fixed order inside one thread, so results are bitwise
// reproducible run to run (no float atomics).
#include <type_traits>

#include "compiler.hpp"
#include "device.hpp"

namespace cfrx {

constexpr int BLOCK = 256;
// one thread per set of an update group; uint8 member-to-set indices
static_assert(GROUP_SETS_MAX <= BLOCK && GROUP_SETS_MAX <= 256, "update group sets");

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float max_t(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double max_t(double a, double b) { return fmax(a, b); }

// child a of node n: explicit layouts list children, the breadth-first layout numbers them
template <bool EXPLICIT>
__device__ __forceinline__ int32_t child_of(const int32_t *__restrict__ kid, int32_t edge) {
    if constexpr (EXPLICIT) return kid[edge];
    else return edge;
}

// Forward reach of one node c (eqs. reach, lanes): both lanes copy the parent's reach; the lane of
// the parent's owner multiplies by sigma(slot).  Terminals carry no reach.
template <typename T>
__device__ __forceinline__ void forward_node(int32_t c, const int2 *__restrict__ up, const T *__restrict__ sigma,
                                             T *__restrict__ r1, T *__restrict__ r2) {
    const int2 u = up[c];
    if (!(u.y & CODE_INTERNAL)) return;
    const int owner = u.y & CODE_OWNER_MASK;
    const T s = owner ? sigma[u.y >> CODE_SLOT_SHIFT] : T(1);
    const T a = r1[u.x], b = r2[u.x];
    r1[c] = owner == 1 ? a * s : a;
    r2[c] = owner == 2 ? b * s : b;
}

// nodes per thread of k_forward
constexpr int FWD_NPT = 4;

// XCD-aware tile order.  The dispatcher hands the workgroups of a launch to the 8 XCDs in turn
// (workgroup b to XCD b mod 8) and each XCD has its own L2, so neighbouring tiles -- which share
// cache lines: the child values of interleaved information sets, the strategy rows of one set --
// would be fetched once per XCD.  Tiles are dealt out instead in runs of XCD_RUN consecutive tiles
// per XCD: workgroup b = 8 i + x runs tile (i / R) 8R + x R + (i mod R), R = XCD_RUN, a bijection
// of [0, M) with M the largest multiple of 8R not above n; tiles from M on keep their index.  Runs
// (rather than one contiguous eighth of the level per XCD) keep the XCDs' shares of a level
// alike where the work per tile drifts along it.  Measured: on the 256-subgame batch the update
// levels took 13 % less time than with the plain order, the large game was 1 % faster; one
// contiguous eighth per XCD was as fast on the batch but 3-7 % slower on the large game.
constexpr int32_t XCD_RUN = 16;
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t n) {
    const int32_t M = n / (8 * XCD_RUN) * (8 * XCD_RUN);
    if (b >= M) return b;
    const int32_t x = b & 7, i = b >> 3;
    return i / XCD_RUN * (8 * XCD_RUN) + x * XCD_RUN + i % XCD_RUN;
}

// One forward level, FWD_NPT nodes per thread (strided by the block size, so each wave's accesses
// stay contiguous): all edge codes are loaded first, then all parent reaches and strategies, with
// the strategy load unconditional (chance parents carry slot 0, a valid address) and only the
// stores masked, so a thread keeps every load of its nodes in flight together.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_forward(int32_t lo, int32_t hi, const int2 *__restrict__ up,
                                                   const T *__restrict__ sigma, T *__restrict__ r1,
                                                   T *__restrict__ r2, int32_t *tick,
                                                   const int32_t *__restrict__ tiles) {
    if (tick && blockIdx.x == 0 && threadIdx.x == 0) tick[0] += 1;
    if (hi <= lo) return;
    // with retired games only the listed tiles run (a tile shared with a retired game rewrites that
    // game's reach with the same values: its strategy no longer changes)
    const int32_t x = xcd_tile((int32_t)blockIdx.x, (int32_t)gridDim.x);
    const int32_t tile = tiles ? tiles[x] : x;
    const int32_t base = lo + tile * (BLOCK * FWD_NPT) + (int32_t)threadIdx.x;
    int2 u[FWD_NPT];
#pragma unroll
    for (int i = 0; i < FWD_NPT; i++) u[i] = up[min(base + i * BLOCK, hi - 1)];
    T sv[FWD_NPT], a[FWD_NPT], b[FWD_NPT];
#pragma unroll
    for (int i = 0; i < FWD_NPT; i++) {
        sv[i] = sigma[u[i].y >> CODE_SLOT_SHIFT];
        a[i] = r1[u[i].x];
        b[i] = r2[u[i].x];
    }
#pragma unroll
    for (int i = 0; i < FWD_NPT; i++) {
        const int32_t c = base + i * BLOCK;
        if (c >= hi || !(u[i].y & CODE_INTERNAL)) continue;
        const int owner = u[i].y & CODE_OWNER_MASK;
        r1[c] = owner == 1 ? a[i] * sv[i] : a[i];
        r2[c] = owner == 2 ? b[i] * sv[i] : b[i];
    }
}

// Arrays read and written by the backward/update level.
template <typename T>
struct LevelArgs {
    const int32_t *grp_iset_off, *slot_off, *mem_off;
    const int2 *mem;
    const int8_t *iset_player;
    const int32_t *kid_off, *kid, *chance_node, *bigc_node;
    const int32_t *grp_list, *chance_list, *bigc_list;   // batches with retired games (nullptr: all)
    const int32_t *koff, *mnode;   // affine layouts: per-slot child offset, compact member list
    const uint16_t *mpos;          // affine layouts: set-major position of each member of a node-order group
    const int8_t *grp_perm;        // affine layouts: 1 where a group's member list is in node order
    T *v;
    T *r1, *r2;   // reach lanes (the level only reads them; the persistent form's forward levels write)
    T *R;
    double *sbar;
    T *sigma;
    T *pred;      // PCFR+ prediction buffer, nullptr for the other rules
};

// What the update of iteration t does (paper Sec. 6, update rules; see cfr.h).
struct RuleArgs {
    int rule;          // CFR_RULE_*
    int upd;           // players whose sets are updated: bit 0 player 1, bit 1 player 2
    double w;          // average weight (t or 1 for CFR and CFR+, t^2 for PCFR+, 1 for DCFR)
    double pos, neg;   // DCFR: discounts of positive and of other regrets
    double sdisc;      // DCFR: strategy-sum discount
};

__device__ __forceinline__ RuleArgs rule_args(int rule, int linear, int upd, int32_t t) {
    RuleArgs r;
    r.rule = rule;
    r.upd = upd;
    const double td = (double)t;
    r.w = rule == CFR_RULE_DCFR ? 1.0 : rule == CFR_RULE_PCFR_PLUS ? td * td : linear ? td : 1.0;
    r.pos = r.neg = r.sdisc = 1.0;
    if (rule == CFR_RULE_DCFR) {
        const double ta = pow(td, DCFR_ALPHA), tb = pow(td, DCFR_BETA);
        r.pos = ta / (ta + 1.0);
        r.neg = tb / (tb + 1.0);
        r.sdisc = pow(td / (td + 1.0), DCFR_GAMMA);
    }
    return r;
}

// Value of an internal chance node: the sum of its children (chance folded into the template).
template <typename T, bool EXPLICIT>
__device__ __forceinline__ void chance_value(int32_t h, const LevelArgs<T> &a) {
    const int32_t b = a.kid_off[h], e = a.kid_off[h + 1];
    T acc = T(0);
    // eight children per step, loads unconditional (past the last child they repeat it) so they
    // are in flight together; the sum keeps child order
    constexpr int U = 8;
    for (int32_t c0 = b; c0 < e; c0 += U) {
        int32_t ch[U];
        T x[U];
#pragma unroll
        for (int i = 0; i < U; i++) ch[i] = child_of<EXPLICIT>(a.kid, min(c0 + i, e - 1));
#pragma unroll
        for (int i = 0; i < U; i++) x[i] = a.v[ch[i]];
#pragma unroll
        for (int i = 0; i < U; i++) acc = c0 + i < e ? acc + x[i] : acc;
    }
    a.v[h] = acc;
}

// Value of a chance node with large fan-out, by a whole block: each thread sums a strided slice
// of the children in order, then a fixed-shape tree reduction over the block (deterministic).
// Must be called by every thread of the block.
template <typename T, bool EXPLICIT>
__device__ void big_chance_value(int32_t h, const LevelArgs<T> &a, T *red) {
    const int tid = threadIdx.x;
    const int32_t b = a.kid_off[h], e = a.kid_off[h + 1];
    T acc = T(0);
    // this thread's children b + tid, b + tid + BLOCK, ... summed in that order, eight loads in
    // flight at a time (past the last child the index is clamped and the value not added)
    constexpr int U = 8;
    for (int32_t c0 = b + tid; c0 < e; c0 += U * BLOCK) {
        int32_t ch[U];
        T x[U];
#pragma unroll
        for (int i = 0; i < U; i++) ch[i] = child_of<EXPLICIT>(a.kid, min(c0 + i * BLOCK, e - 1));
#pragma unroll
        for (int i = 0; i < U; i++) x[i] = a.v[ch[i]];
#pragma unroll
        for (int i = 0; i < U; i++) acc = c0 + i * BLOCK < e ? acc + x[i] : acc;
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) a.v[h] = red[0];
    __syncthreads();
}

// The update of one information set from its instantaneous regrets r (already summed over the
// members, player 1's sign) and its state as loaded (R, sigma^t, sbar): R <- R + sign r with the
// rule's clamp or discount, sbar += w pi_i(I) sigma^t (FP64; DCFR discounts it), then
// sigma^{t+1} = regret matching of R (PCFR+: of R plus the prediction, which becomes this
// iteration's instantaneous regret and is stored here).  Rk and sb are updated in place and the
// new strategy is returned in sn.
template <typename T, int MAXA, bool EXT>
__device__ __forceinline__ void set_update_compute(const RuleArgs &ru, const LevelArgs<T> &a, int32_t s0, int32_t nA,
                                                   int pl, double pown, const T (&r)[MAXA], T (&Rk)[MAXA],
                                                   const T (&sk)[MAXA], double (&sb)[MAXA], T (&sn)[MAXA]) {
    const T sign = pl == 1 ? T(1) : T(-1);
    T tot = T(0);
    T Rn[MAXA];
    if constexpr (!EXT) {
        const bool clamp = ru.rule != CFR_RULE_CFR;
#pragma unroll
        for (int k = 0; k < MAXA; k++)
            if (k < nA) {
                sb[k] += ru.w * pown * (double)sk[k];
                T y = fma_t(sign, r[k], Rk[k]);
                if (clamp) y = max_t(y, T(0));
                Rk[k] = y;
                Rn[k] = max_t(y, T(0));
                tot += Rn[k];
            }
    } else {
        if (ru.rule == CFR_RULE_DCFR) {
            const T pos = (T)ru.pos, neg = (T)ru.neg;
#pragma unroll
            for (int k = 0; k < MAXA; k++)
                if (k < nA) {
                    sb[k] = (sb[k] + pown * (double)sk[k]) * ru.sdisc;
                    T y = fma_t(sign, r[k], Rk[k]);
                    y = y > T(0) ? y * pos : y * neg;
                    Rk[k] = y;
                    Rn[k] = max_t(y, T(0));
                    tot += Rn[k];
                }
        } else if (ru.rule == CFR_RULE_PCFR_PLUS) {
#pragma unroll
            for (int k = 0; k < MAXA; k++)
                if (k < nA) {
                    sb[k] += ru.w * pown * (double)sk[k];
                    const T y = max_t(fma_t(sign, r[k], Rk[k]), T(0));
                    const T m = sign * r[k];
                    Rk[k] = y;
                    a.pred[s0 + k] = m;
                    Rn[k] = max_t(y + m, T(0));
                    tot += Rn[k];
                }
        } else {
            const bool clamp = ru.rule != CFR_RULE_CFR;
#pragma unroll
            for (int k = 0; k < MAXA; k++)
                if (k < nA) {
                    sb[k] += ru.w * pown * (double)sk[k];
                    T y = fma_t(sign, r[k], Rk[k]);
                    if (clamp) y = max_t(y, T(0));
                    Rk[k] = y;
                    Rn[k] = max_t(y, T(0));
                    tot += Rn[k];
                }
        }
    }
    const T inv = tot > T(0) ? T(1) / tot : T(0);
    const T uni = T(1) / (T)nA;
#pragma unroll
    for (int k = 0; k < MAXA; k++) sn[k] = tot > T(0) ? Rn[k] * inv : uni;
}

// set_update_compute, then the set's new regrets, strategy sums and strategy stored in place.
template <typename T, int MAXA, bool EXT>
__device__ __forceinline__ void set_update_from(const RuleArgs &ru, const LevelArgs<T> &a, int32_t s0, int32_t nA,
                                                int pl, double pown, const T (&r)[MAXA], T (&Rk)[MAXA],
                                                const T (&sk)[MAXA], double (&sb)[MAXA]) {
    T sn[MAXA];
    set_update_compute<T, MAXA, EXT>(ru, a, s0, nA, pl, pown, r, Rk, sk, sb, sn);
#pragma unroll
    for (int k = 0; k < MAXA; k++)
        if (k < nA) {
            a.R[s0 + k] = Rk[k];
            a.sbar[s0 + k] = sb[k];
            a.sigma[s0 + k] = sn[k];
        }
}

// Load the set's state, then set_update_from.
template <typename T, int MAXA>
__device__ __forceinline__ void load_set_state(const LevelArgs<T> &a, int32_t s0, int32_t nA, T (&Rk)[MAXA],
                                               T (&sk)[MAXA], double (&sb)[MAXA]) {
    // unconditional loads (past the last action they repeat it): all in flight at once
#pragma unroll
    for (int k = 0; k < MAXA; k++) {
        const int32_t q = s0 + min(k, nA - 1);
        Rk[k] = a.R[q];
        sk[k] = a.sigma[q];
        sb[k] = a.sbar[q];
    }
}

template <typename T, int MAXA, bool EXT>
__device__ __forceinline__ void set_update(const RuleArgs &ru, const LevelArgs<T> &a, int32_t s0, int32_t nA, int pl,
                                           double pown, const T (&r)[MAXA]) {
    T Rk[MAXA], sk[MAXA];
    double sb[MAXA];
    load_set_state<T, MAXA>(a, s0, nA, Rk, sk, sb);
    set_update_from<T, MAXA, EXT>(ru, a, s0, nA, pl, pown, r, Rk, sk, sb);
}

// Phase 2 of a group: a set's instantaneous regrets r(I, a) += po(h) * diff(h, a) over its staged
// members [k0, k1) in ascending order, one fused multiply-add chain per action.  The LDS reads of
// U members are issued before their multiply-adds (the order of the chain is unchanged), so a set
// with many members does not wait one LDS round trip per member.  The first NA columns are
// accumulated (NA bounds the group's action counts): past a set's actions the columns hold repeats
// that are never read afterwards.
template <typename T, int MAXA, int NA = MAXA>
__device__ __forceinline__ void reduce_members(const T *po, const T *diff, int32_t k0, int32_t k1, T (&r)[MAXA]) {
    constexpr int U = NA <= 4 ? (sizeof(T) == 4 ? 8 : 4) : 2;
    int32_t k = k0;
    for (; k + U <= k1; k += U) {
        T p[U], d[U][NA];
#pragma unroll
        for (int i = 0; i < U; i++) {
            p[i] = po[k + i];
#pragma unroll
            for (int q = 0; q < NA; q++) d[i][q] = diff[(k + i) * MAXA + q];
        }
#pragma unroll
        for (int i = 0; i < U; i++)
#pragma unroll
            for (int q = 0; q < NA; q++) r[q] = fma_t(p[i], d[i][q], r[q]);
    }
    for (; k < k1; k++) {
        const T p = po[k];
#pragma unroll
        for (int q = 0; q < NA; q++) r[q] = fma_t(p, diff[k * MAXA + q], r[q]);
    }
}

// LDS staging of one update group (members of a chunk, the group's set offsets)
template <typename T, int MAXA, int MPT>
struct GroupLds {
    T po[MPT * BLOCK];
    alignas(16) T diff[MPT * BLOCK * MAXA];
    int32_t moff[BLOCK + 1];
    int32_t slot[BLOCK + 1];
};

// One update group: consecutive information sets of one depth with at most MPT * BLOCK members
// and GROUP_SETS sets.  Phase 1 (one thread per member h, coalesced over the member list):
//   v(h) = sum_a sigma^t(I, a) v(h.a)   -- written to v: the backward value pass at h
//   stage pi_{-i}(h) and v(h.a) - v(h) in LDS.
// Phase 2 (one thread per set I): reduce the set's members from LDS in ascending member order,
//   r(I,a) = sum_h s_i pi_{-i}(h) (v(h.a) - v(h)), then R <- R + r (CFR+: max(R, 0)),
//   sbar += w_t pi_i(I) sigma^t (FP64), sigma^{t+1} = regret matching of R.
// Only this group reads sigma(I) during the backward pass (all members of I are here), and the
// forward pass has already consumed it, so overwriting sigma(I) with sigma^{t+1} is safe.
// Sets with more members than a chunk are streamed through LDS chunk by chunk.  Must be called by
// every thread of the block (it synchronises the block).
template <typename T, int MAXA, int MPT, bool EXPLICIT, bool EXT>
__device__ void group_update(int32_t g, const RuleArgs &ru, const LevelArgs<T> &a, GroupLds<T, MAXA, MPT> &L) {
    // EXT: the discounted and predictive rules (DCFR, PCFR+); otherwise CFR or CFR+ (lean tail)
    constexpr int CHUNK = MPT * BLOCK;
    const int tid = threadIdx.x;
    const int32_t i0 = a.grp_iset_off[g], i1 = a.grp_iset_off[g + 1];
    const int32_t nsets = i1 - i0;
    if (tid < nsets) {
        L.moff[tid] = a.mem_off[i0 + tid];
        L.slot[tid] = a.slot_off[i0 + tid];
    }
    if (tid == 0) {
        L.moff[nsets] = a.mem_off[i1];
        L.slot[nsets] = a.slot_off[i1];
    }
    __syncthreads();
    const int32_t mbeg = L.moff[0], mend = L.moff[nsets];
    const bool has_set = tid < nsets;
    int32_t s0 = 0, nA = 0, m0 = 0, m1 = 0, pl = 1;
    if (has_set) {
        s0 = L.slot[tid];
        nA = L.slot[tid + 1] - s0;
        m0 = L.moff[tid];
        m1 = L.moff[tid + 1];
        pl = a.iset_player[i0 + tid];
    }
    T r[MAXA];
#pragma unroll
    for (int k = 0; k < MAXA; k++) r[k] = T(0);
    for (int32_t cb = mbeg; cb < mend; cb += CHUNK) {
        const int32_t ce = min(cb + CHUNK, mend);
        // loads first and unconditional (past the chunk's end a lane repeats its first member, past
        // a set's last action the last child and slot), then the arithmetic and the masked stores
        bool in[MPT];
        int32_t sb[MPT], na[MPT], hh[MPT];
        T po[MPT], sg[MPT][MAXA], cv[MPT][MAXA];
#pragma unroll
        for (int u = 0; u < MPT; u++) {
            const int32_t j = u * BLOCK + tid;
            in[u] = cb + j < ce;
            const int32_t m = cb + (in[u] ? j : 0);
            // the set of member m: the last k with moff[k] <= m
            int32_t lo = 0, hi = nsets - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (L.moff[mid] <= m) lo = mid; else hi = mid - 1;
            }
            sb[u] = L.slot[lo];
            na[u] = L.slot[lo + 1] - sb[u];
            const int2 x = a.mem[m];
            hh[u] = x.x & MEMBER_NODE_MASK;
            po[u] = ((x.x & MEMBER_P2) ? a.r1 : a.r2)[hh[u]];
#pragma unroll
            for (int k = 0; k < MAXA; k++) {
                const int32_t kk = min(k, na[u] - 1);
                cv[u][k] = a.v[child_of<EXPLICIT>(a.kid, x.y + kk)];
                sg[u][k] = a.sigma[sb[u] + kk];
            }
        }
#pragma unroll
        for (int u = 0; u < MPT; u++) {
            T vh = T(0);
#pragma unroll
            for (int k = 0; k < MAXA; k++) vh = k < na[u] ? fma_t(sg[u][k], cv[u][k], vh) : vh;
            if (!in[u]) continue;
            const int32_t j = u * BLOCK + tid;
            a.v[hh[u]] = vh;
            L.po[j] = po[u];
#pragma unroll
            for (int k = 0; k < MAXA; k++) L.diff[j * MAXA + k] = cv[u][k] - vh;
        }
        __syncthreads();
        if (has_set) reduce_members<T, MAXA>(L.po, L.diff, max(m0, cb) - cb, min(m1, ce) - cb, r);
        __syncthreads();
    }
    if (!has_set) return;
    // alternating order: the other player's half leaves this set's state alone (values only)
    if (!((ru.upd >> (pl - 1)) & 1)) return;
    const T *own = pl == 1 ? a.r1 : a.r2;
    set_update<T, MAXA, EXT>(ru, a, s0, nA, pl, (double)own[a.mem[m0].x & MEMBER_NODE_MASK], r);
}

// LDS staging of one update group in an affine layout: the slot offsets of its sets, the set of each
// member of the chunk and (FP32 state, up to 16 actions) each set's child offsets and strategy row,
// besides the member values of group_update.  The rows hold GS sets, the game's group bound (128 or
// 256): with 128 an FP32 block's LDS fits six per compute unit instead of five.  For FP64 the rows
// would cost a resident block per compute unit (measured slower), so members read them through the
// cache instead.
template <typename T, int MAXA, int MPT, int GS>
struct GroupLdsA {
    static constexpr bool ROWS = MAXA <= 16 && sizeof(T) == 4;
    static constexpr int RA = ROWS ? MAXA : 1;
    T po[MPT * BLOCK];
    alignas(16) T diff[MPT * BLOCK * MAXA];
    alignas(16) int32_t ko[GS * RA];
    alignas(16) T sg[GS * RA];
    int32_t slot[GS + 1];
    int32_t wmax[BLOCK / 64];
    uint8_t mset[MPT * BLOCK];
};

// Calls f with the smallest action bound of {2, 3, MAXA} (MAXA = 4) or {4, MAXA} (wider
// instantiations) that is at least n, as a compile-time constant, so a pass over sets or members
// that need fewer actions issues fewer loads (large game: FP64 state 5 % faster, FP32 unchanged; a
// 16-action instantiation would otherwise load 16 children per member of a 2-action set).  n must
// be uniform over the wave (or the block).
template <int MAXA, typename F>
__device__ __forceinline__ void with_action_bound(int32_t n, F &&f) {
    if constexpr (MAXA <= 4) {
        if (n <= 2) f(std::integral_constant<int, 2>{});
        else if (n <= 3) f(std::integral_constant<int, 3>{});
        else f(std::integral_constant<int, MAXA>{});
    } else {
        if (n <= 4) f(std::integral_constant<int, 4>{});
        else f(std::integral_constant<int, MAXA>{});
    }
}

// group_update for affine layouts (child a of member h is h + koff[slot a]): the same arithmetic
// in the same order, so the results are bitwise those of group_update.  What changes is how the
// loads are issued.  The vector-memory pipeline (address and data units at ~90 % busy) bounds
// this pass, so the per-slot child offsets and strategy, the same for every member of a set, are
// loaded once per set (by its thread, into an LDS row) instead of once per member; a member then
// loads only its record, its opponent reach and its child values.  Loads are unconditional: past
// a set's last action they repeat its last child (an address already read), lanes past the
// chunk's end repeat its first member, so a chunk's loads are in flight together; only stores
// and arithmetic are masked.  (A guard that skips a load no lane needs compiles to a branch with
// a full wait at its join, which costs more than the load.)  The number of child loads per member
// is the group's widest set, bucketed (with_action_bound; the public-state layout orders states by
// action count, so most groups are uniform): a block-uniform choice made once per group, outside
// the loops.  Where a group's sets interleave -- a player-2 set's members are strided by the
// opponent's hand count -- the host lists the group's members in node order instead (grp_perm) with
// each one's set-major position: consecutive lanes then touch consecutive nodes, children and values
// instead of one cache line each, and the staging stays set-major, so the reduction, and every
// result, is unchanged.  The two orders are separate instantiations of the member pass, chosen per
// group.  Each set thread fetches its own reach through its first member.
template <typename T, int MAXA, int MPT, bool EXT, int GS>
__device__ void group_update_affine(int32_t g, const RuleArgs &ru, const LevelArgs<T> &a,
                                    GroupLdsA<T, MAXA, MPT, GS> &L) {
    constexpr int CHUNK = MPT * BLOCK;
    constexpr bool ROWS = GroupLdsA<T, MAXA, MPT, GS>::ROWS;
    const int tid = threadIdx.x;
    const int32_t i0 = a.grp_iset_off[g], i1 = a.grp_iset_off[g + 1];
    const int32_t nsets = i1 - i0;
    const int32_t mbeg = a.mem_off[i0], mend = a.mem_off[i1];
    const bool has_set = tid < nsets;
    const int32_t ti = i0 + (has_set ? tid : nsets - 1);
    const int32_t m0 = a.mem_off[ti], m1 = a.mem_off[ti + 1];
    const int32_t s0 = a.slot_off[ti], nA = a.slot_off[ti + 1] - s0;
    const int pl = a.iset_player[ti];
    const bool perm = a.grp_perm[g] != 0;
    // the set's first member: in a set-major list at m0 (lines the member pass reads anyway; the
    // 8-byte member records would cost one extra line per set); in a node-order list, from them
    int32_t h0;
    if (perm) h0 = a.mem[m0].x & MEMBER_NODE_MASK;
    else h0 = a.mnode[m0] & MEMBER_NODE_MASK;
    const T *__restrict__ r1 = a.r1;
    const T *__restrict__ r2 = a.r2;
    const T *__restrict__ sig = a.sigma;
    const int32_t *__restrict__ koff = a.koff;
    // the widest set of this wave, then (after the barrier) of the group
    int32_t wa = has_set ? nA : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) wa = max(wa, __shfl_xor(wa, off));
    wa = __builtin_amdgcn_readfirstlane(wa);
    if constexpr (ROWS) {
        // row k of a set holds slot min(k, nA - 1): every column a member may read is filled
        with_action_bound<MAXA>(wa, [&](auto nb) {
            constexpr int NB = decltype(nb)::value;
            int32_t kr[NB];
            T sr[NB];
#pragma unroll
            for (int k = 0; k < NB; k++) {
                const int32_t q = s0 + min(k, nA - 1);
                kr[k] = koff[q];
                sr[k] = sig[q];
            }
            if (has_set) {
#pragma unroll
                for (int k = 0; k < MAXA; k++) {
                    L.ko[tid * MAXA + k] = kr[min(k, NB - 1)];
                    L.sg[tid * MAXA + k] = sr[min(k, NB - 1)];
                }
            }
        });
    }
    if ((tid & 63) == 0) L.wmax[tid >> 6] = wa;
    if (has_set) {
        L.slot[tid] = s0;
        if (tid == nsets - 1) L.slot[nsets] = s0 + nA;
        // member -> set map of the first chunk: a group of several sets fits one chunk, and a group
        // that needs more chunks holds a single set (index 0 throughout)
        const int32_t e = min(m1, mbeg + CHUNK);
        for (int32_t m = m0; m < e; m++) L.mset[m - mbeg] = (uint8_t)tid;
    }
    __syncthreads();
    int32_t ga = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; w++) ga = max(ga, L.wmax[w]);
    const T pown = (pl == 1 ? r1 : r2)[h0];
    T r[MAXA];
#pragma unroll
    for (int k = 0; k < MAXA; k++) r[k] = T(0);
    auto member_pass = [&](auto nag, auto permc) {
        constexpr int NA = decltype(nag)::value;
        constexpr bool PERM = decltype(permc)::value;
        for (int32_t cb = mbeg; cb < mend; cb += CHUNK) {
            const int32_t ce = min(cb + CHUNK, mend);
            bool in[MPT];
            int32_t hn[MPT], pj[MPT], st[MPT], sb[MPT], na[MPT];
#pragma unroll
            for (int u = 0; u < MPT; u++) {
                const int32_t j = u * BLOCK + tid;
                in[u] = cb + j < ce;
                const int32_t jj = in[u] ? j : 0;
                // thread j takes the group's j-th listed member; in a node-order group pj is its
                // slot in the set-major staging
                hn[u] = a.mnode[cb + jj];
                if constexpr (PERM) pj[u] = a.mpos[cb + jj];
                else pj[u] = jj;
                st[u] = L.mset[pj[u]];
                sb[u] = L.slot[st[u]];
                na[u] = L.slot[st[u] + 1] - sb[u];
            }
            T po[MPT], cv[MPT][NA], sg[MPT][ROWS ? 1 : NA];
#pragma unroll
            for (int u = 0; u < MPT; u++) {
                const int32_t h = hn[u] & MEMBER_NODE_MASK;
                po[u] = ((hn[u] & MEMBER_P2) ? r1 : r2)[h];
                int32_t ko[NA];
#pragma unroll
                for (int k = 0; k < NA; k++) {
                    if constexpr (ROWS) {
                        ko[k] = L.ko[st[u] * MAXA + k];
                    } else {
                        const int32_t q = sb[u] + min(k, na[u] - 1);
                        ko[k] = koff[q];
                        sg[u][k] = sig[q];
                    }
                }
#pragma unroll
                for (int k = 0; k < NA; k++) cv[u][k] = a.v[h + ko[k]];
            }
#pragma unroll
            for (int u = 0; u < MPT; u++) {
                T vh = T(0);
#pragma unroll
                for (int k = 0; k < NA; k++) {
                    T sk;
                    if constexpr (ROWS) sk = L.sg[st[u] * MAXA + k];
                    else sk = sg[u][k];
                    vh = k < na[u] ? fma_t(sk, cv[u][k], vh) : vh;
                }
                if (!in[u]) continue;
                const int32_t j = pj[u];
                a.v[hn[u] & MEMBER_NODE_MASK] = vh;
                L.po[j] = po[u];
#pragma unroll
                for (int k = 0; k < NA; k++) L.diff[j * MAXA + k] = cv[u][k] - vh;
            }
            __syncthreads();
            if (has_set) reduce_members<T, MAXA, NA>(L.po, L.diff, max(m0, cb) - cb, min(m1, ce) - cb, r);
            __syncthreads();
        }
    };
    with_action_bound<MAXA>(ga, [&](auto nag) {
        if (perm) member_pass(nag, std::true_type{});
        else member_pass(nag, std::false_type{});
    });
    if constexpr (ROWS && MAXA <= 4) {
        // The group's slots [S0, S1) are contiguous: move their regrets, strategy sums and strategy
        // through LDS (the member staging is free now) with coalesced passes of the whole block,
        // instead of each set thread loading and storing its few slots.  Slots of sets this half
        // leaves alone are written back unchanged.
        const int32_t S0 = L.slot[0], S1 = L.slot[nsets];
        double *sbs = reinterpret_cast<double *>(L.diff);            // [<= CHUNK]
        T *Rs = reinterpret_cast<T *>(sbs + CHUNK), *Ss = Rs + CHUNK; // [<= CHUNK] each
        for (int32_t q = tid; q < S1 - S0; q += BLOCK) {
            sbs[q] = a.sbar[S0 + q];
            Rs[q] = a.R[S0 + q];
            Ss[q] = sig[S0 + q];
        }
        __syncthreads();
        if (has_set && ((ru.upd >> (pl - 1)) & 1)) {
            const int32_t b = s0 - S0;
            T Rk[MAXA], sk[MAXA], sn[MAXA];
            double sb[MAXA];
#pragma unroll
            for (int k = 0; k < MAXA; k++) {
                const int32_t q = b + min(k, nA - 1);
                Rk[k] = Rs[q];
                sk[k] = Ss[q];
                sb[k] = sbs[q];
            }
            set_update_compute<T, MAXA, EXT>(ru, a, s0, nA, pl, (double)pown, r, Rk, sk, sb, sn);
#pragma unroll
            for (int k = 0; k < MAXA; k++)
                if (k < nA) {
                    Rs[b + k] = Rk[k];
                    sbs[b + k] = sb[k];
                    Ss[b + k] = sn[k];
                }
        }
        __syncthreads();
        for (int32_t q = tid; q < S1 - S0; q += BLOCK) {
            a.sbar[S0 + q] = sbs[q];
            a.R[S0 + q] = Rs[q];
            a.sigma[S0 + q] = Ss[q];
        }
    } else {
        if (!has_set) return;
        if (!((ru.upd >> (pl - 1)) & 1)) return;
        set_update<T, MAXA, EXT>(ru, a, s0, nA, pl, (double)pown, r);
    }
}

// AF: 0 the child-list update, 1 the affine update with rows for 256 sets per group, 2 the affine
// update with rows for 128 (FP32 state, at most 4 actions)
constexpr int aff_sets(int AF) { return AF == 2 ? 128 : GROUP_SETS_MAX; }

template <typename T, int MAXA, int MPT, bool EXPLICIT, int AF>
using LevelLds = std::conditional_t<AF != 0, GroupLdsA<T, MAXA, MPT, aff_sets(AF)>, GroupLds<T, MAXA, MPT>>;

template <typename T, int MAXA, int MPT, bool EXPLICIT, bool EXT, int AF>
__device__ __forceinline__ void update_group(int32_t g, const RuleArgs &ru, const LevelArgs<T> &a,
                                             LevelLds<T, MAXA, MPT, EXPLICIT, AF> &L) {
    if constexpr (AF != 0) group_update_affine<T, MAXA, MPT, EXT, aff_sets(AF)>(g, ru, a, L);
    else group_update<T, MAXA, MPT, EXPLICIT, EXT>(g, ru, a, L);
}

// FP64 state with at most 4 actions and the lean rule tail: ask for 6 waves per SIMD (78 registers, no
// spills; the LDS of 6 workgroups fits) instead of the 5 that 86 registers allow.  The discounted and
// predictive tails would spill under that bound.  FP32 needs no bound: its registers allow 6 and its
// LDS too with 128-set groups (5 with 256).
template <typename T, int MAXA, bool EXT>
constexpr int level_min_waves() { return (sizeof(T) == 8 && MAXA <= 4 && !EXT) ? 6 : 1; }
template <typename T, int MAXA, int MPT, bool EXPLICIT, bool EXT, int AF>
__global__ void __launch_bounds__(BLOCK, (level_min_waves<T, MAXA, EXT>())) k_level(int32_t gbeg, int32_t ngroups, int32_t bbeg, int32_t nbig,
                                                 int32_t cbeg, int32_t nchance, LevelArgs<T> a,
                                                 const int32_t *__restrict__ tcount, int rule, int linear, int upd) {
    __shared__ LevelLds<T, MAXA, MPT, EXPLICIT, AF> L;
    const int32_t blk = (int32_t)blockIdx.x;
    // with retired games in a batch the ranges index lists of the work that still runs (a retired
    // game's values feed only its own parents)
    if (blk >= ngroups + nbig) {
        const int32_t j = (blk - ngroups - nbig) * BLOCK + (int32_t)threadIdx.x;
        if (j < nchance) chance_value<T, EXPLICIT>(a.chance_node[a.chance_list ? a.chance_list[cbeg + j] : cbeg + j], a);
        return;
    }
    if (blk >= ngroups) {
        const int32_t b = bbeg + blk - ngroups;
        big_chance_value<T, EXPLICIT>(a.bigc_node[a.bigc_list ? a.bigc_list[b] : b], a, L.po);
        return;
    }
    const int32_t x = gbeg + xcd_tile(blk, ngroups);
    const int32_t grp = a.grp_list ? a.grp_list[x] : x;
    const RuleArgs ru = rule_args(rule, linear, upd, tcount[0]);
    update_group<T, MAXA, MPT, EXPLICIT, EXT, AF>(grp, ru, a, L);
}

// Per-game barrier among the W blocks of one game.  Thread 0 publishes the block's writes
// (device-scope release), arrives on the game's counter and waits, with a bounded spin, until all
// W blocks of this epoch arrived; on time-out it raises the error flag and stops waiting, so every
// wave still exits.  Returns false once the error flag is up.
__device__ __forceinline__ bool game_barrier(int32_t *ctr, int32_t W, int32_t &epoch, int32_t *err,
                                             int64_t timeout_ticks) {
    __shared__ int32_t s_ok;
    if (W == 1) {
        __syncthreads();
        return true;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        epoch += 1;
        __threadfence();
        atomicAdd(ctr, 1);
        // Arrivals are counted modulo 2^32 and compared by signed difference, so the count may wrap
        // over a long launch.  The poll is a relaxed load: an acquiring load per poll would
        // invalidate this compute unit's caches on every spin.  One fence after the count is
        // reached makes the other blocks' writes visible.
        const uint32_t target = (uint32_t)epoch * (uint32_t)W;
        const int64_t t_start = (int64_t)wall_clock64();
        int32_t ok = 1;
        while ((int32_t)((uint32_t)__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                (int64_t)wall_clock64() - t_start > timeout_ticks) {
                atomicExch(err, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// The work of one (game, rank): n_iter whole iterations of game gm as rank `rank` of its W workgroups,
// which stride over each forward level's nodes and each backward level's update groups and chance
// nodes and meet at the game's barrier between levels.  Iteration t0 + k (k = 1..n_iter) uses the
// same arithmetic, in the same order per set, as the level-synchronous kernels.  Returns false once
// a barrier reported an error.
template <typename T, int MAXA, int MPT, bool EXPLICIT, bool EXT, int AF>
__device__ bool persistent_game(int32_t gm, int32_t rank, int32_t W, const int32_t *__restrict__ game_range,
                                const int32_t *__restrict__ game_depth, int32_t MD, int32_t n_iter,
                                const int2 *__restrict__ up, const LevelArgs<T> &a, int32_t t0, int32_t *barrier,
                                int32_t *err, int64_t timeout_ticks, int rule, int linear, int alternating,
                                LevelLds<T, MAXA, MPT, EXPLICIT, AF> &L) {
    const int32_t *gr = game_range + (size_t)gm * (MD + 1) * GR_FIELDS_DEV;
    const int32_t Ds = game_depth[gm];
    const int tid = threadIdx.x;
    int32_t epoch = 0;
    const int halves = alternating ? 2 : 1;
    for (int32_t it = 1; it <= n_iter; it++) {
        for (int half = 0; half < halves; half++) {
            const RuleArgs ru = rule_args(rule, linear, alternating ? 1 << half : 3, t0 + it);
            for (int32_t d = 1; d <= Ds; d++) {
                const int32_t lo = gr[d * GR_FIELDS_DEV], hi = gr[d * GR_FIELDS_DEV + 1];
                for (int32_t c = lo + rank * BLOCK + tid; c < hi; c += W * BLOCK)
                    forward_node<T>(c, up, a.sigma, a.r1, a.r2);
                if (!game_barrier(barrier + gm, W, epoch, err, timeout_ticks)) return false;
            }
            for (int32_t d = Ds - 1; d >= 0; d--) {
                const int32_t *r = gr + d * GR_FIELDS_DEV;
                for (int32_t g = r[2] + rank; g < r[3]; g += W) update_group<T, MAXA, MPT, EXPLICIT, EXT, AF>(g, ru, a, L);
                for (int32_t b = r[6] + rank; b < r[7]; b += W) big_chance_value<T, EXPLICIT>(a.bigc_node[b], a, L.po);
                for (int32_t j = r[4] + rank * BLOCK + tid; j < r[5]; j += W * BLOCK) chance_value<T, EXPLICIT>(a.chance_node[j], a);
                if (!game_barrier(barrier + gm, W, epoch, err, timeout_ticks)) return false;
            }
        }
    }
    return true;
}

// The batched persistent form: one launch runs n_iter whole iterations of every game of a forest.
// The work is a list of tickets (game, rank, W), one queue per XCD: a game's W ranks are consecutive
// tickets of one queue.  A workgroup claims tickets of the queue of the XCD it runs on (the hardware
// XCC id), in order, runs each claimed rank to the end, then takes the other queues' remaining
// tickets.  A game's barrier therefore waits only for ranks claimed by workgroups already running,
// and the others are claimed next by whichever workgroup frees up: the launch needs one game's
// workgroups resident at once, not the whole grid, and any grid size is correct.
template <typename T, int MAXA, int MPT, bool EXPLICIT, bool EXT, int AF>
__global__ void __launch_bounds__(BLOCK) k_persistent(const int4 *__restrict__ tickets, const int32_t *__restrict__ q_off,
                                                      int32_t *claim, const int32_t *__restrict__ game_range,
                                                      const int32_t *__restrict__ game_depth, int32_t MD, int32_t n_iter,
                                                      const int2 *__restrict__ up, LevelArgs<T> a,
                                                      const int32_t *__restrict__ tcount, int32_t *barrier,
                                                      int32_t *err, int64_t timeout_ticks, int rule, int linear,
                                                      int alternating) {
    __shared__ LevelLds<T, MAXA, MPT, EXPLICIT, AF> L;
    __shared__ int32_t s_ticket;
    const int32_t t0 = tcount[0];
    // XCC_ID hardware register (bits 3:0): the XCD this workgroup runs on
    const int home = (int)(__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (PERSISTENT_QUEUES - 1));
    for (int k = 0; k < PERSISTENT_QUEUES; k++) {
        const int q = (home + k) & (PERSISTENT_QUEUES - 1);
        const int32_t qlo = q_off[q], qn = q_off[q + 1] - qlo;
        for (;;) {
            if (threadIdx.x == 0) s_ticket = atomicAdd(claim + q, 1);
            __syncthreads();
            const int32_t t = s_ticket;
            __syncthreads();
            if (t >= qn) break;
            const int4 wt = tickets[qlo + t];
            if (!persistent_game<T, MAXA, MPT, EXPLICIT, EXT, AF>(wt.x, wt.y, wt.z, game_range, game_depth, MD, n_iter, up,
                                                                a, t0, barrier, err, timeout_ticks, rule, linear,
                                                                alternating, L))
                return;
        }
    }
}

// ---- the LDS-resident schedule for tiny standalone games --------------------------------------
//
// One workgroup runs n_iter whole iterations of a game whose state fits in LDS: the values (with
// the terminal template), both reach lanes, strategy, regrets, strategy sums and (PCFR+) the
// prediction are staged in, every level of every iteration runs between block barriers, and the
// state is written back at the end.  No launch per level and no trip to HBM inside the loop.  The
// structure arrays stay in global memory (read-only and small, so cache-resident).  One thread
// per information set walks its members in ascending order with the level kernels' arithmetic,
// so the iterates are bitwise those of the level launches.

// The update of one set by one thread: member values v(h) = sum_a sigma v(h.a), the set's
// instantaneous regrets summed over its members in ascending order, then set_update.
template <typename T, int MAXA, bool EXPLICIT, bool EXT>
__device__ void set_serial(int32_t i, const RuleArgs &ru, const LevelArgs<T> &a) {
    const int32_t s0 = a.slot_off[i], nA = a.slot_off[i + 1] - s0;
    const int32_t m0 = a.mem_off[i], m1 = a.mem_off[i + 1];
    const int pl = a.iset_player[i];
    T sg[MAXA], r[MAXA];
#pragma unroll
    for (int k = 0; k < MAXA; k++) {
        sg[k] = a.sigma[s0 + min(k, nA - 1)];
        r[k] = T(0);
    }
    for (int32_t m = m0; m < m1; m++) {
        const int2 x = a.mem[m];
        const int32_t h = x.x & MEMBER_NODE_MASK;
        const T po = ((x.x & MEMBER_P2) ? a.r1 : a.r2)[h];
        T cv[MAXA];
#pragma unroll
        for (int k = 0; k < MAXA; k++) cv[k] = a.v[child_of<EXPLICIT>(a.kid, x.y + min(k, nA - 1))];
        T vh = T(0);
#pragma unroll
        for (int k = 0; k < MAXA; k++) vh = k < nA ? fma_t(sg[k], cv[k], vh) : vh;
        a.v[h] = vh;
#pragma unroll
        for (int q = 0; q < MAXA; q++) r[q] = fma_t(po, cv[q] - vh, r[q]);
    }
    if (!((ru.upd >> (pl - 1)) & 1)) return;
    const T *own = pl == 1 ? a.r1 : a.r2;
    set_update<T, MAXA, EXT>(ru, a, s0, nA, pl, (double)own[a.mem[m0].x & MEMBER_NODE_MASK], r);
}

// Dynamic LDS of k_lds: strategy sums (double) first, then v, r1, r2 [N] and sigma, R (and the
// PCFR+ prediction) [A] in the state type, then BLOCK reduction slots for big chance nodes.
size_t lds_schedule_bytes(int32_t N, int32_t A, int fp64, int pred) {
    const size_t es = fp64 ? 8 : 4;
    return 8 * (size_t)A + es * (3 * (size_t)N + (pred ? 3 : 2) * (size_t)A + BLOCK);
}

template <typename T, int MAXA, bool EXPLICIT, bool EXT>
__global__ void __launch_bounds__(BLOCK) k_lds(const int32_t *__restrict__ gr, int32_t D, int32_t N, int32_t A,
                                               int32_t n_iter, const int2 *__restrict__ up, LevelArgs<T> g,
                                               const int32_t *__restrict__ tcount, int rule, int linear,
                                               int alternating) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *sb = reinterpret_cast<double *>(smem);
    T *v = reinterpret_cast<T *>(sb + A);
    T *r1 = v + N, *r2 = r1 + N, *sig = r2 + N, *R = sig + A;
    T *pred = g.pred ? R + A : nullptr;
    T *red = R + A + (g.pred ? A : 0);
    const int tid = threadIdx.x;
    for (int32_t i = tid; i < N; i += BLOCK) {
        v[i] = g.v[i];
        r1[i] = g.r1[i];
        r2[i] = g.r2[i];
    }
    for (int32_t q = tid; q < A; q += BLOCK) {
        sb[q] = g.sbar[q];
        sig[q] = g.sigma[q];
        R[q] = g.R[q];
        if (pred) pred[q] = g.pred[q];
    }
    __syncthreads();
    LevelArgs<T> a = g;
    a.v = v; a.r1 = r1; a.r2 = r2; a.sigma = sig; a.R = R; a.sbar = sb; a.pred = pred;
    const int32_t t0 = tcount[0];
    const int halves = alternating ? 2 : 1;
    for (int32_t it = 1; it <= n_iter; it++) {
        for (int half = 0; half < halves; half++) {
            const RuleArgs ru = rule_args(rule, linear, alternating ? 1 << half : 3, t0 + it);
            for (int32_t d = 1; d <= D; d++) {
                const int32_t lo = gr[d * GR_FIELDS_DEV], hi = gr[d * GR_FIELDS_DEV + 1];
                for (int32_t c = lo + tid; c < hi; c += BLOCK) forward_node<T>(c, up, sig, r1, r2);
                __syncthreads();
            }
            for (int32_t d = D - 1; d >= 0; d--) {
                const int32_t *r = gr + d * GR_FIELDS_DEV;
                const int32_t ib = a.grp_iset_off[r[2]], ie = a.grp_iset_off[r[3]];
                for (int32_t i = ib + tid; i < ie; i += BLOCK) set_serial<T, MAXA, EXPLICIT, EXT>(i, ru, a);
                for (int32_t j = r[4] + tid; j < r[5]; j += BLOCK) chance_value<T, EXPLICIT>(a.chance_node[j], a);
                for (int32_t b = r[6]; b < r[7]; b++) big_chance_value<T, EXPLICIT>(a.bigc_node[b], a, red);
                __syncthreads();
            }
        }
    }
    for (int32_t i = tid; i < N; i += BLOCK) {
        g.v[i] = v[i];
        g.r1[i] = r1[i];
        g.r2[i] = r2[i];
    }
    for (int32_t q = tid; q < A; q += BLOCK) {
        g.sbar[q] = sb[q];
        g.sigma[q] = sig[q];
        g.R[q] = R[q];
        if (pred) g.pred[q] = pred[q];
    }
}

__global__ void k_fill_int(int32_t n, int32_t *p, int32_t value) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = value;
}

__global__ void k_add_counter(int32_t *t, int32_t n) {
    if (threadIdx.x == 0) t[0] += n;
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_regret_matching(int32_t I, const int32_t *__restrict__ slot_off,
                                                           const T *__restrict__ R, const T *__restrict__ pred,
                                                           T *__restrict__ sigma) {
    int32_t i = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i >= I) return;
    int32_t s0 = slot_off[i], s1 = slot_off[i + 1];
    // PCFR+: regret matching of R + prediction
    auto x = [&](int32_t q) { return pred ? R[q] + pred[q] : R[q]; };
    T tot = T(0);
    for (int32_t q = s0; q < s1; q++) tot += max_t(x(q), T(0));
    const T inv = tot > T(0) ? T(1) / tot : T(0);
    const T uni = T(1) / (T)(s1 - s0);
    for (int32_t q = s0; q < s1; q++) sigma[q] = tot > T(0) ? max_t(x(q), T(0)) * inv : uni;
}

__global__ void k_tick(int32_t *t) {
    if (threadIdx.x == 0) t[0] += 1;
}

__global__ void __launch_bounds__(BLOCK) k_average(int32_t I, const int32_t *__restrict__ slot_off,
                                                   const double *__restrict__ sbar, double *__restrict__ sigbar,
                                                   float *__restrict__ out) {
    int32_t i = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i >= I) return;
    int32_t s0 = slot_off[i], s1 = slot_off[i + 1];
    double tot = 0.0;
    for (int32_t q = s0; q < s1; q++) tot += sbar[q];
    const double uni = 1.0 / (double)(s1 - s0);
    for (int32_t q = s0; q < s1; q++) {
        double x = tot > 0.0 ? sbar[q] / tot : uni;
        sigbar[q] = x;
        out[q] = (float)x;
    }
}

// dst[i] = src[map i] (map == nullptr: identity)
template <typename S, typename D>
__global__ void __launch_bounds__(BLOCK) k_gather(int32_t n, const int32_t *__restrict__ map,
                                                  const S *__restrict__ src, D *__restrict__ dst) {
    int32_t i = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i < n) dst[i] = (D)src[map ? map[i] : i];
}

// dst[map i] = src[i] (map == nullptr: identity)
template <typename S, typename D>
__global__ void __launch_bounds__(BLOCK) k_scatter(int32_t n, const int32_t *__restrict__ map,
                                                   const S *__restrict__ src, D *__restrict__ dst) {
    int32_t i = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i < n) dst[map ? map[i] : i] = (D)src[i];
}

// dst[map i] += src[i]
template <typename S, typename D>
__global__ void __launch_bounds__(BLOCK) k_scatter_add(int32_t n, const int32_t *__restrict__ map,
                                                       const S *__restrict__ src, D *__restrict__ dst) {
    int32_t i = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i < n) {
        const int32_t j = map ? map[i] : i;
        dst[j] = dst[j] + (D)src[i];
    }
}

// ---- in-place re-solve: the chance-folded template of a game's terminals ---------------------
__global__ void __launch_bounds__(BLOCK) k_gather_payoffs(int64_t lo, int64_t hi, const int32_t *__restrict__ in,
                                                          const double *__restrict__ pay, double *__restrict__ u) {
    const int64_t j = lo + (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (j < hi) u[j] = pay[in[j]];
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_template(int64_t lo, int64_t hi, const int32_t *__restrict__ node,
                                                    const int32_t *__restrict__ branch, const double *__restrict__ u,
                                                    const double *__restrict__ pic, const double *__restrict__ root,
                                                    T *__restrict__ v, double *__restrict__ vbr) {
    const int64_t j = lo + (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (j >= hi) return;
    const double c = root ? root[branch[j]] * pic[j] : pic[j];
    const double t = c * u[j];
    v[node[j]] = (T)t;
    vbr[node[j]] = t;
}

// ---- best response (FP64) -------------------------------------------------

__global__ void __launch_bounds__(BLOCK) k_br_forward(int32_t lo, int32_t hi, const int2 *__restrict__ up,
                                                      const double *__restrict__ sigbar, double *__restrict__ q,
                                                      int br) {
    int32_t c = lo + (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (c >= hi) return;
    int2 u = up[c];
    if (!(u.y & CODE_INTERNAL)) return;
    int owner = u.y & CODE_OWNER_MASK;
    double m = (owner != 0 && owner != br) ? sigbar[u.y >> CODE_SLOT_SHIFT] : 1.0;
    q[c] = q[u.x] * m;
}

template <bool EXPLICIT>
__global__ void __launch_bounds__(BLOCK) k_br_argmax(int32_t ilo, int32_t ihi, const int32_t *__restrict__ slot_off,
                                                     const int32_t *__restrict__ mem_off,
                                                     const int2 *__restrict__ mem,
                                                     const int8_t *__restrict__ iset_player,
                                                     const int32_t *__restrict__ kid_off,
                                                     const int32_t *__restrict__ kid,
                                                     const double *__restrict__ vbr, const double *__restrict__ q,
                                                     int32_t *__restrict__ astar, int br) {
    int32_t i = ilo + (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i >= ihi) return;
    if (iset_player[i] != br) return;
    int32_t nA = slot_off[i + 1] - slot_off[i];
    int32_t m0 = mem_off[i], m1 = mem_off[i + 1];
    const double sign = br == 1 ? 1.0 : -1.0;
    int best = 0;
    double bq = 0.0;
    for (int a = 0; a < nA; a++) {
        double Q = 0.0;
        for (int32_t m = m0; m < m1; m++) {
            const int2 x = mem[m];
            Q += q[x.x & MEMBER_NODE_MASK] * (sign * vbr[child_of<EXPLICIT>(kid, x.y + a)]);
        }
        if (a == 0 || Q > bq) { bq = Q; best = a; }
    }
    astar[i] = best;
}

template <bool EXPLICIT>
__global__ void __launch_bounds__(BLOCK) k_br_backward(int32_t lo, int32_t hi, const int32_t *__restrict__ kid_off,
                                                       const int32_t *__restrict__ kid,
                                                       const int32_t *__restrict__ node_slot,
                                                       const int32_t *__restrict__ node_iset,
                                                       const int8_t *__restrict__ iset_player,
                                                       const double *__restrict__ sigbar,
                                                       const int32_t *__restrict__ astar, double *__restrict__ vbr,
                                                       int br) {
    int32_t h = lo + (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (h >= hi) return;
    int32_t b = kid_off[h], e = kid_off[h + 1];
    if (b == e) return;
    int32_t s = node_slot[h];
    double acc = 0.0;
    if (s < 0) {
        for (int32_t c = b; c < e; c++) acc += vbr[child_of<EXPLICIT>(kid, c)];
    } else {
        int32_t i = node_iset[h];
        if (iset_player[i] == br) {
            acc = vbr[child_of<EXPLICIT>(kid, b + astar[i])];
        } else {
            for (int32_t c = b; c < e; c++) acc += sigbar[s + (c - b)] * vbr[child_of<EXPLICIT>(kid, c)];
        }
    }
    vbr[h] = acc;
}

// ---- launchers ------------------------------------------------------------

template <typename T>
static hipError_t forward_t(const DevGame &g, int32_t lo, int32_t hi, int32_t *tick, const int32_t *fwd_tiles,
                           int64_t n_tiles, hipStream_t s) {
    T *r = (T *)g.reach;
    // one block still runs the counter bump
    if (fwd_tiles && n_tiles == 0) hi = lo;
    const unsigned blocks = hi <= lo ? 1u : fwd_tiles ? (unsigned)n_tiles
                                                       : (unsigned)((hi - lo + BLOCK * FWD_NPT - 1) / (BLOCK * FWD_NPT));
    hipLaunchKernelGGL(k_forward<T>, dim3(blocks), dim3(BLOCK), 0, s, lo, hi, g.up, (const T *)g.sigma, r,
                       r + g.N, tick, fwd_tiles);
    return hipGetLastError();
}

hipError_t launch_forward(const DevGame &g, int d, int32_t lo, int32_t hi, int32_t *tick, hipStream_t s) {
    if (hi <= lo && !tick) return hipSuccess;
    const int32_t *tiles = g.use_lists ? g.fwd_list + g.fwd_off[d] : nullptr;
    const int64_t nt = g.use_lists ? g.fwd_off[d + 1] - g.fwd_off[d] : 0;
    if (g.use_lists && nt == 0 && !tick) return hipSuccess;
    return g.fp64 ? forward_t<double>(g, lo, hi, tick, tiles, nt, s) : forward_t<float>(g, lo, hi, tick, tiles, nt, s);
}

template <typename T>
static LevelArgs<T> level_args(const DevGame &g) {
    LevelArgs<T> a;
    a.grp_iset_off = g.grp_iset_off; a.slot_off = g.slot_off; a.mem_off = g.mem_off; a.mem = g.mem;
    a.iset_player = g.iset_player; a.kid_off = g.kid_off; a.kid = g.kid; a.chance_node = g.chance_node;
    a.bigc_node = g.bigc_node;
    a.koff = g.koff; a.mnode = g.mnode; a.mpos = g.mpos; a.grp_perm = g.grp_perm;
    a.grp_list = g.use_lists ? g.grp_list : nullptr;
    a.chance_list = g.use_lists ? g.chance_list : nullptr;
    a.bigc_list = g.use_lists ? g.bigc_list : nullptr;
    a.v = (T *)g.v;
    a.r1 = (T *)g.reach;
    a.r2 = (T *)g.reach + g.N;
    a.R = (T *)g.R; a.sbar = g.sbar; a.sigma = (T *)g.sigma;
    a.pred = (T *)g.pred;
    return a;
}

template <typename T, int MAXA, int MPT, bool EX, bool XT, int AF>
static hipError_t level_t(const DevGame &g, int d, IterFlags f, hipStream_t s) {
    // all work of depth d, or with retired games the listed part of it
    const int32_t gbeg = g.use_lists ? (int32_t)g.grp_off[d] : g.grp_depth_off[d];
    const int32_t ng = g.use_lists ? (int32_t)(g.grp_off[d + 1] - g.grp_off[d]) : g.grp_depth_off[d + 1] - gbeg;
    const int32_t cbeg = g.use_lists ? (int32_t)g.chance_off_l[d] : g.chance_off[d];
    const int32_t nc = g.use_lists ? (int32_t)(g.chance_off_l[d + 1] - g.chance_off_l[d]) : g.chance_off[d + 1] - cbeg;
    const int32_t bbeg = g.use_lists ? (int32_t)g.bigc_off_l[d] : g.bigc_off[d];
    const int32_t nb = g.use_lists ? (int32_t)(g.bigc_off_l[d + 1] - g.bigc_off_l[d]) : g.bigc_off[d + 1] - bbeg;
    const unsigned blocks = (unsigned)ng + (unsigned)nb + grid_for(nc);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_level<T, MAXA, MPT, EX, XT, AF>), dim3(blocks), dim3(BLOCK), 0, s,
                       gbeg, ng, bbeg, nb, cbeg, nc, level_args<T>(g), g.t, f.rule, f.linear, f.upd);
    return hipGetLastError();
}

// the discounted and predictive rules get their own instantiation, so CFR and CFR+ keep a lean update
inline bool ext_rule(int rule) { return rule == CFR_RULE_DCFR || rule == CFR_RULE_PCFR_PLUS; }

// Instantiation selector shared by the level and persistent launches: state type, action bound
// (members per thread must match the group capacity the compiler used, group_members: four for
// FP32 state with at most 4 actions, two for FP64, else one), child addressing (implicit,
// explicit, affine; AF, see aff_sets) and rule class.
template <typename T, bool EX, bool XT, int AF, typename F>
static auto by_actions(const DevGame &g, F &&f) {
    static_assert(AF != 2 || sizeof(T) == 4, "128-set rows are an FP32 instantiation");
    if constexpr (AF == 2) {
        return f.template operator()<T, 4, 4, EX, XT, 2>();
    } else {
        if (g.max_actions <= 4) return f.template operator()<T, 4, sizeof(T) == 4 ? 4 : 2, EX, XT, AF>();
        if (g.max_actions <= 16) return f.template operator()<T, 16, 1, EX, XT, AF>();
        return f.template operator()<T, 64, 1, EX, XT, AF>();
    }
}

template <typename T, typename F>
static auto by_kind(const DevGame &g, int rule, F &&f) {
    const bool x = ext_rule(rule);
    if (g.affine) {
        // FP32 state, at most 4 actions, groups of at most 128 sets: the instantiation with 128-set rows
        if constexpr (sizeof(T) == 4)
            if (g.max_actions <= 4 && g.group_sets == 128)
                return x ? by_actions<T, true, true, 2>(g, f) : by_actions<T, true, false, 2>(g, f);
        return x ? by_actions<T, true, true, 1>(g, f) : by_actions<T, true, false, 1>(g, f);
    }
    if (g.explicit_kids) return x ? by_actions<T, true, true, 0>(g, f) : by_actions<T, true, false, 0>(g, f);
    return x ? by_actions<T, false, true, 0>(g, f) : by_actions<T, false, false, 0>(g, f);
}

struct LevelLaunch {
    const DevGame &g; int d; IterFlags f; hipStream_t s;
    template <typename T, int MAXA, int MPT, bool EX, bool XT, int AF>
    hipError_t operator()() const { return level_t<T, MAXA, MPT, EX, XT, AF>(g, d, f, s); }
};

hipError_t launch_level(const DevGame &g, int d, IterFlags f, hipStream_t s) {
    const LevelLaunch L{g, d, f, s};
    return g.fp64 ? by_kind<double>(g, f.rule, L) : by_kind<float>(g, f.rule, L);
}

struct PersistentLaunch {
    const DevGame &g; const PersistentPlan &p; int32_t T_; IterFlags f; int alt; hipStream_t s;
    template <typename T, int MAXA, int MPT, bool EX, bool XT, int AF>
    hipError_t operator()() const {
        hipLaunchKernelGGL((k_persistent<T, MAXA, MPT, EX, XT, AF>), dim3(p.blocks), dim3(BLOCK), 0, s, p.tickets,
                           p.q_off, p.claim, p.game_range, p.game_depth, p.max_depth, T_, g.up, level_args<T>(g), g.t,
                           p.barrier, p.err, p.timeout_ticks, f.rule, f.linear, alt);
        return hipGetLastError();
    }
};

hipError_t launch_persistent(const DevGame &g, const PersistentPlan &p, int32_t T_, IterFlags f, int alt,
                             hipStream_t s) {
    // the barrier counters and, right after them, the queues' claim counters start at zero
    const int32_t nz = p.n_games + PERSISTENT_QUEUES;
    hipLaunchKernelGGL(k_fill_int, dim3((nz + 255) / 256), dim3(256), 0, s, nz, p.barrier, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const PersistentLaunch L{g, p, T_, f, alt, s};
    e = g.fp64 ? by_kind<double>(g, f.rule, L) : by_kind<float>(g, f.rule, L);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_add_counter, dim3(1), dim3(64), 0, s, g.t, T_);
    return hipGetLastError();
}

struct LdsLaunch {
    const DevGame &g; const int32_t *gr; int32_t T_; IterFlags f; int alt; hipStream_t s; size_t bytes;
    bool prepare;   // true: only raise the kernel's dynamic LDS limit to bytes
    template <typename T, int MAXA, int MPT, bool EX, bool XT, int AF>
    hipError_t operator()() const {
        if constexpr (MAXA > 16) {
            return hipErrorInvalidValue;
        } else {
            auto fn = k_lds<T, MAXA, EX, XT>;
            if (prepare)
                return hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            hipLaunchKernelGGL(fn, dim3(1), dim3(BLOCK), bytes, s, gr, g.max_depth, g.N, g.A, T_, g.up,
                               level_args<T>(g), g.t, f.rule, f.linear, alt);
            return hipGetLastError();
        }
    }
};

// the serial update reads the child list when the layout has one (affine offsets serve only the
// member-parallel form)
template <typename T>
static hipError_t lds_dispatch(const DevGame &g, const LdsLaunch &L) {
    const bool x = ext_rule(L.f.rule);
    if (g.explicit_kids) return x ? by_actions<T, true, true, 0>(g, L) : by_actions<T, true, false, 0>(g, L);
    return x ? by_actions<T, false, true, 0>(g, L) : by_actions<T, false, false, 0>(g, L);
}

hipError_t prepare_lds(const DevGame &g, int rule, size_t *bytes) {
    *bytes = lds_schedule_bytes(g.N, g.A, g.fp64, g.pred != nullptr);
    if (g.max_actions > 16) return hipErrorInvalidValue;
    const LdsLaunch L{g, nullptr, 0, IterFlags{rule, 0, 3}, 0, nullptr, *bytes, true};
    return g.fp64 ? lds_dispatch<double>(g, L) : lds_dispatch<float>(g, L);
}

hipError_t launch_lds(const DevGame &g, const int32_t *game_range, int32_t T_, IterFlags f, int alt, hipStream_t s) {
    const size_t bytes = lds_schedule_bytes(g.N, g.A, g.fp64, g.pred != nullptr);
    const LdsLaunch L{g, game_range, T_, f, alt, s, bytes, false};
    hipError_t e = g.fp64 ? lds_dispatch<double>(g, L) : lds_dispatch<float>(g, L);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_add_counter, dim3(1), dim3(64), 0, s, g.t, T_);
    return hipGetLastError();
}

struct PersistentFn {
    template <typename T, int MAXA, int MPT, bool EX, bool XT, int AF>
    const void *operator()() const { return reinterpret_cast<const void *>(&k_persistent<T, MAXA, MPT, EX, XT, AF>); }
};

// the instantiation launch_persistent uses for this game
hipError_t persistent_occupancy(const DevGame &g, int *blocks_per_cu) {
    const void *fn = g.fp64 ? by_kind<double>(g, g.rule, PersistentFn{}) : by_kind<float>(g, g.rule, PersistentFn{});
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, BLOCK, 0);
}

hipError_t launch_regret_matching(const DevGame &g, hipStream_t s) {
    if (g.I == 0) return hipSuccess;
    if (g.fp64)
        hipLaunchKernelGGL(k_regret_matching<double>, dim3(grid_for(g.I)), dim3(BLOCK), 0, s, g.I, g.slot_off,
                           (const double *)g.R, (const double *)g.pred, (double *)g.sigma);
    else
        hipLaunchKernelGGL(k_regret_matching<float>, dim3(grid_for(g.I)), dim3(BLOCK), 0, s, g.I, g.slot_off,
                           (const float *)g.R, (const float *)g.pred, (float *)g.sigma);
    return hipGetLastError();
}

hipError_t launch_tick(const DevGame &g, hipStream_t s) {
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, g.t);
    return hipGetLastError();
}

hipError_t launch_average(const DevGame &g, hipStream_t s) {
    if (g.I == 0) return hipSuccess;
    hipLaunchKernelGGL(k_average, dim3(grid_for(g.I)), dim3(BLOCK), 0, s, g.I, g.slot_off, g.sbar, g.sigbar, g.out2);
    return hipGetLastError();
}

hipError_t launch_sigma_to_float(const DevGame &g, float *dst, hipStream_t s) {
    if (g.A == 0) return hipSuccess;
    if (g.fp64)
        hipLaunchKernelGGL((k_gather<double, float>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map,
                           (const double *)g.sigma, dst);
    else
        hipLaunchKernelGGL((k_gather<float, float>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map,
                           (const float *)g.sigma, dst);
    return hipGetLastError();
}

hipError_t launch_gather_float(const DevGame &g, const float *src, float *dst, hipStream_t s) {
    if (g.A == 0) return hipSuccess;
    hipLaunchKernelGGL((k_gather<float, float>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map, src, dst);
    return hipGetLastError();
}

hipError_t launch_regrets_from_float(const DevGame &g, const float *src, hipStream_t s) {
    if (g.A == 0) return hipSuccess;
    if (g.fp64)
        hipLaunchKernelGGL((k_scatter<float, double>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map, src,
                           (double *)g.R);
    else
        hipLaunchKernelGGL((k_scatter<float, float>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map, src,
                           (float *)g.R);
    return hipGetLastError();
}

hipError_t launch_regrets_add_float(const DevGame &g, const float *src, hipStream_t s) {
    if (g.A == 0) return hipSuccess;
    if (g.fp64)
        hipLaunchKernelGGL((k_scatter_add<float, double>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map,
                           src, (double *)g.R);
    else
        hipLaunchKernelGGL((k_scatter_add<float, float>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map,
                           src, (float *)g.R);
    return hipGetLastError();
}

// dst[map q] <- src[q] for a canonical FP64 source: into the state type (R, prediction) or into the FP64
// strategy sums
hipError_t launch_scatter_double(const DevGame &g, const double *src, void *dst, bool state_type, hipStream_t s) {
    if (g.A == 0) return hipSuccess;
    if (!state_type)
        hipLaunchKernelGGL((k_scatter<double, double>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map, src,
                           (double *)dst);
    else if (g.fp64)
        hipLaunchKernelGGL((k_scatter<double, double>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map, src,
                           (double *)dst);
    else
        hipLaunchKernelGGL((k_scatter<double, float>), dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, g.slot_map, src,
                           (float *)dst);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_zero(int32_t n, T *__restrict__ p) {
    const int32_t i = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i < n) p[i] = T(0);
}

// A slots of the state type set to zero (a fill kernel, so it may sit in a captured graph)
hipError_t launch_fill_state(const DevGame &g, void *dst, hipStream_t s) {
    if (g.A == 0) return hipSuccess;
    if (g.fp64) hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, (double *)dst);
    else hipLaunchKernelGGL(k_zero<float>, dim3(grid_for(g.A)), dim3(BLOCK), 0, s, g.A, (float *)dst);
    return hipGetLastError();
}

hipError_t launch_gather_payoffs(int64_t lo, int64_t hi, const int32_t *in, const double *payoff_in, double *u,
                                 hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    hipLaunchKernelGGL(k_gather_payoffs, dim3((unsigned)((hi - lo + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, lo, hi,
                       in, payoff_in, u);
    return hipGetLastError();
}

hipError_t launch_template(const DevGame &g, int64_t lo, int64_t hi, const int32_t *node, const int32_t *branch,
                           const double *u, const double *pic, const double *root, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    const dim3 grid((unsigned)((hi - lo + BLOCK - 1) / BLOCK));
    if (g.fp64)
        hipLaunchKernelGGL(k_template<double>, grid, dim3(BLOCK), 0, s, lo, hi, node, branch, u, pic, root,
                           (double *)g.v, g.vbr);
    else
        hipLaunchKernelGGL(k_template<float>, grid, dim3(BLOCK), 0, s, lo, hi, node, branch, u, pic, root,
                           (float *)g.v, g.vbr);
    return hipGetLastError();
}

hipError_t launch_br_forward(const DevGame &g, int32_t lo, int32_t hi, int br, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    hipLaunchKernelGGL(k_br_forward, dim3(grid_for(hi - lo)), dim3(BLOCK), 0, s, lo, hi, g.up, g.sigbar, g.qbr, br);
    return hipGetLastError();
}

hipError_t launch_br_argmax(const DevGame &g, int32_t ilo, int32_t ihi, int br, hipStream_t s) {
    if (ihi <= ilo) return hipSuccess;
    if (g.explicit_kids)
        hipLaunchKernelGGL(k_br_argmax<true>, dim3(grid_for(ihi - ilo)), dim3(BLOCK), 0, s, ilo, ihi, g.slot_off,
                           g.mem_off, g.mem, g.iset_player, g.kid_off, g.kid, g.vbr, g.qbr, g.astar, br);
    else
        hipLaunchKernelGGL(k_br_argmax<false>, dim3(grid_for(ihi - ilo)), dim3(BLOCK), 0, s, ilo, ihi, g.slot_off,
                           g.mem_off, g.mem, g.iset_player, g.kid_off, g.kid, g.vbr, g.qbr, g.astar, br);
    return hipGetLastError();
}

hipError_t launch_br_backward(const DevGame &g, int32_t lo, int32_t hi, int br, hipStream_t s) {
    if (hi <= lo) return hipSuccess;
    if (g.explicit_kids)
        hipLaunchKernelGGL(k_br_backward<true>, dim3(grid_for(hi - lo)), dim3(BLOCK), 0, s, lo, hi, g.kid_off, g.kid,
                           g.node_slot, g.node_iset, g.iset_player, g.sigbar, g.astar, g.vbr, br);
    else
        hipLaunchKernelGGL(k_br_backward<false>, dim3(grid_for(hi - lo)), dim3(BLOCK), 0, s, lo, hi, g.kid_off, g.kid,
                           g.node_slot, g.node_iset, g.iset_player, g.sigbar, g.astar, g.vbr, br);
    return hipGetLastError();
}

}  // namespace cfrx
