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
#include "device.hpp"

namespace cfrx {

constexpr int BLOCK = 256;

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

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_forward(int32_t lo, int32_t hi, const int2 *__restrict__ up,
                                                   const T *__restrict__ sigma, T *__restrict__ r1,
                                                   T *__restrict__ r2, int32_t *tick) {
    if (tick && blockIdx.x == 0 && threadIdx.x == 0) tick[0] += 1;
    int32_t c = lo + (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (c >= hi) return;
    int2 u = up[c];
    if (!(u.y & CODE_INTERNAL)) return;
    int owner = u.y & CODE_OWNER_MASK;
    T s = owner ? sigma[u.y >> CODE_SLOT_SHIFT] : T(1);
    T a = r1[u.x], b = r2[u.x];
    r1[c] = owner == 1 ? a * s : a;
    r2[c] = owner == 2 ? b * s : b;
}

// One backward level fused with the regret / average / regret-matching update of the
// information sets on that level.  Launched once per depth d (deepest first) with
//   blocks [0, ngroups)            one update group each: consecutive information sets of depth d
//                                  with at most BLOCK members and BLOCK sets in total
//   blocks [ngroups, ...)          one thread per internal chance node of depth d
// Group blocks, phase 1 (one thread per member h, coalesced over the member list):
//   v(h) = sum_a sigma^t(I, a) v(h.a)   -- written to v, the backward value pass at h
//   stage pi_{-i}(h) and v(h.a) - v(h) in LDS.
// Phase 2 (one thread per set I): reduce the set's members from LDS in ascending member order,
//   r(I,a) = sum_h s_i pi_{-i}(h) (v(h.a) - v(h)), then R <- R + r (CFR+: max(R, 0)),
//   sbar += w_t pi_i(I) sigma^t (FP64), sigma^{t+1} = regret matching of R.
// Only this block reads sigma(I) during the backward pass (all members of I are here), and the
// forward pass has already consumed it, so overwriting sigma(I) with sigma^{t+1} is safe.
// Sets with more than BLOCK members are streamed through LDS in chunks.
template <typename T, int MAXA, int MPT, bool EXPLICIT>
__global__ void __launch_bounds__(BLOCK) k_level(
    int32_t gbeg, int32_t ngroups, const int32_t *__restrict__ chance_node, int32_t cbeg, int32_t nchance,
    const int32_t *__restrict__ grp_iset_off, const int32_t *__restrict__ slot_off,
    const int32_t *__restrict__ mem_off, const int2 *__restrict__ mem, const int8_t *__restrict__ iset_player,
    const int32_t *__restrict__ kid_off, const int32_t *__restrict__ kid, T *__restrict__ v,
    const T *__restrict__ r1, const T *__restrict__ r2, T *__restrict__ R, double *__restrict__ sbar,
    T *__restrict__ sigma, const int32_t *__restrict__ tcount, int plus, int linear) {
    constexpr int CHUNK = MPT * BLOCK;
    const int tid = threadIdx.x;
    if ((int32_t)blockIdx.x >= ngroups) {
        const int32_t j = ((int32_t)blockIdx.x - ngroups) * BLOCK + tid;
        if (j >= nchance) return;
        const int32_t h = chance_node[cbeg + j];
        const int32_t b = kid_off[h], e = kid_off[h + 1];
        T acc = T(0);
        for (int32_t c = b; c < e; c++) acc += v[child_of<EXPLICIT>(kid, c)];
        v[h] = acc;
        return;
    }
    __shared__ T s_po[CHUNK];
    __shared__ T s_diff[CHUNK * MAXA];
    __shared__ int32_t s_moff[BLOCK + 1];
    __shared__ int32_t s_slot[BLOCK + 1];
    const int32_t g = gbeg + (int32_t)blockIdx.x;
    const int32_t i0 = grp_iset_off[g], i1 = grp_iset_off[g + 1];
    const int32_t nsets = i1 - i0;
    if (tid < nsets) {
        s_moff[tid] = mem_off[i0 + tid];
        s_slot[tid] = slot_off[i0 + tid];
    }
    if (tid == 0) {
        s_moff[nsets] = mem_off[i1];
        s_slot[nsets] = slot_off[i1];
    }
    __syncthreads();
    const int32_t mbeg = s_moff[0], mend = s_moff[nsets];
    const bool has_set = tid < nsets;
    int32_t s0 = 0, nA = 0, m0 = 0, m1 = 0, pl = 1;
    if (has_set) {
        s0 = s_slot[tid];
        nA = s_slot[tid + 1] - s0;
        m0 = s_moff[tid];
        m1 = s_moff[tid + 1];
        pl = iset_player[i0 + tid];
    }
    T r[MAXA];
#pragma unroll
    for (int a = 0; a < MAXA; a++) r[a] = T(0);
    for (int32_t cb = mbeg; cb < mend; cb += CHUNK) {
        const int32_t ce = min(cb + CHUNK, mend);
#pragma unroll
        for (int u = 0; u < MPT; u++) {
            const int32_t j = u * BLOCK + tid;
            const int32_t m = cb + j;
            if (m < ce) {
                // the set of member m: the last k with s_moff[k] <= m
                int32_t lo = 0, hi = nsets - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (s_moff[mid] <= m) lo = mid; else hi = mid - 1;
                }
                const int32_t sb = s_slot[lo], na = s_slot[lo + 1] - sb;
                const int2 x = mem[m];
                const int32_t h = x.x & MEMBER_NODE_MASK;
                const T po = (x.x & MEMBER_P2) ? r1[h] : r2[h];
                T cv[MAXA];
                T vh = T(0);
#pragma unroll
                for (int a = 0; a < MAXA; a++)
                    if (a < na) cv[a] = v[child_of<EXPLICIT>(kid, x.y + a)];
#pragma unroll
                for (int a = 0; a < MAXA; a++)
                    if (a < na) vh = fma_t(sigma[sb + a], cv[a], vh);
                v[h] = vh;
                s_po[j] = po;
#pragma unroll
                for (int a = 0; a < MAXA; a++)
                    if (a < na) s_diff[j * MAXA + a] = cv[a] - vh;
            }
        }
        __syncthreads();
        if (has_set) {
            const int32_t lo = max(m0, cb), hi = min(m1, ce);
            for (int32_t k = lo - cb; k < hi - cb; k++) {
                const T po = s_po[k];
#pragma unroll
                for (int a = 0; a < MAXA; a++)
                    if (a < nA) r[a] = fma_t(po, s_diff[k * MAXA + a], r[a]);
            }
        }
        __syncthreads();
    }
    if (!has_set) return;
    const T *own = pl == 1 ? r1 : r2;
    const T sign = pl == 1 ? T(1) : T(-1);
    const double w = linear ? (double)tcount[0] : 1.0;
    const double pown = (double)own[mem[m0].x & MEMBER_NODE_MASK];
    T tot = T(0);
    T Rn[MAXA];
#pragma unroll
    for (int a = 0; a < MAXA; a++) {
        if (a < nA) {
            const int32_t q = s0 + a;
            sbar[q] += w * pown * (double)sigma[q];
            T y = fma_t(sign, r[a], R[q]);
            if (plus) y = max_t(y, T(0));
            R[q] = y;
            Rn[a] = max_t(y, T(0));
            tot += Rn[a];
        }
    }
    const T inv = tot > T(0) ? T(1) / tot : T(0);
    const T uni = T(1) / (T)nA;
#pragma unroll
    for (int a = 0; a < MAXA; a++)
        if (a < nA) sigma[s0 + a] = tot > T(0) ? Rn[a] * inv : uni;
}

template <typename T>
__global__ void __launch_bounds__(BLOCK) k_regret_matching(int32_t I, const int32_t *__restrict__ slot_off,
                                                           const T *__restrict__ R, T *__restrict__ sigma) {
    int32_t i = (int32_t)(blockIdx.x * BLOCK + threadIdx.x);
    if (i >= I) return;
    int32_t s0 = slot_off[i], s1 = slot_off[i + 1];
    T tot = T(0);
    for (int32_t q = s0; q < s1; q++) tot += max_t(R[q], T(0));
    const T inv = tot > T(0) ? T(1) / tot : T(0);
    const T uni = T(1) / (T)(s1 - s0);
    for (int32_t q = s0; q < s1; q++) sigma[q] = tot > T(0) ? max_t(R[q], T(0)) * inv : uni;
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
static hipError_t forward_t(const DevGame &g, int32_t lo, int32_t hi, int32_t *tick, hipStream_t s) {
    T *r = (T *)g.reach;
    const unsigned blocks = hi > lo ? grid_for(hi - lo) : 1u;   // one block still runs the counter bump
    hipLaunchKernelGGL(k_forward<T>, dim3(blocks), dim3(BLOCK), 0, s, lo, hi, g.up, (const T *)g.sigma, r,
                       r + g.N, tick);
    return hipGetLastError();
}

hipError_t launch_forward(const DevGame &g, int32_t lo, int32_t hi, int32_t *tick, hipStream_t s) {
    if (hi <= lo && !tick) return hipSuccess;
    return g.fp64 ? forward_t<double>(g, lo, hi, tick, s) : forward_t<float>(g, lo, hi, tick, s);
}

template <typename T, int MAXA, int MPT, bool EX>
static hipError_t level_t(const DevGame &g, int d, IterFlags f, hipStream_t s) {
    const int32_t gbeg = g.grp_depth_off[d], ng = g.grp_depth_off[d + 1] - gbeg;
    const int32_t cbeg = g.chance_off[d], nc = g.chance_off[d + 1] - cbeg;
    const unsigned blocks = (unsigned)ng + grid_for(nc);
    if (blocks == 0) return hipSuccess;
    const T *r = (const T *)g.reach;
    hipLaunchKernelGGL((k_level<T, MAXA, MPT, EX>), dim3(blocks), dim3(BLOCK), 0, s, gbeg, ng, g.chance_node, cbeg, nc,
                       g.grp_iset_off, g.slot_off, g.mem_off, g.mem, g.iset_player, g.kid_off, g.kid, (T *)g.v, r,
                       r + g.N, (T *)g.R, g.sbar, (T *)g.sigma, g.t, f.plus, f.linear);
    return hipGetLastError();
}

template <typename T, bool EX>
static hipError_t level_dispatch_ex(const DevGame &g, int d, IterFlags f, hipStream_t s) {
    // members per thread must match the group capacity the compiler used (group_members)
    if (g.max_actions <= 4) return level_t<T, 4, 2, EX>(g, d, f, s);
    if (g.max_actions <= 16) return level_t<T, 16, 1, EX>(g, d, f, s);
    return level_t<T, 64, 1, EX>(g, d, f, s);
}

template <typename T>
static hipError_t level_dispatch(const DevGame &g, int d, IterFlags f, hipStream_t s) {
    return g.explicit_kids ? level_dispatch_ex<T, true>(g, d, f, s) : level_dispatch_ex<T, false>(g, d, f, s);
}

hipError_t launch_level(const DevGame &g, int d, IterFlags f, hipStream_t s) {
    return g.fp64 ? level_dispatch<double>(g, d, f, s) : level_dispatch<float>(g, d, f, s);
}

hipError_t launch_regret_matching(const DevGame &g, hipStream_t s) {
    if (g.I == 0) return hipSuccess;
    if (g.fp64)
        hipLaunchKernelGGL(k_regret_matching<double>, dim3(grid_for(g.I)), dim3(BLOCK), 0, s, g.I, g.slot_off,
                           (const double *)g.R, (double *)g.sigma);
    else
        hipLaunchKernelGGL(k_regret_matching<float>, dim3(grid_for(g.I)), dim3(BLOCK), 0, s, g.I, g.slot_off,
                           (const float *)g.R, (float *)g.sigma);
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
