// mlp.hip -- the warm-start network on the matrix cores, and the kernels that turn a compiled
// game into network rows and network outputs into initial regrets.
//
// The network maps a 128-wide feature row of an information set through ReLU hidden layers to
// four logits z; p = softplus(z) over the set's legal actions is both the predicted strategy
// (after normalisation) and, scaled, the initial regrets R0 that CFR+ starts from.  Training
// minimises the weighted cross entropy between normalise(p) and the average strategy the solver
// produced, with Adam (Kingma and Ba 2015) on FP32 master weights.  The paper has no learned
// part; these definitions are the project's own.
//
// Arithmetic: every hidden-layer product runs on v_mfma_f32_32x32x16_bf16 with bfloat16
// operands and FP32 accumulation.  Stored in bfloat16 (round to nearest even): feature rows,
// the weight copies the matrix cores read, hidden activations, and the gradients of the hidden
// pre-activations.  FP32: biases, logits, the loss, all parameter gradients, Adam state.  The
// four-wide output layer is a per-row dot product on the vector units (64 lanes, 4 hidden units
// each) fused with the loss.  Every reduction has a fixed order (block partials, then one
// sequential pass), so a step is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cfr.h"
#include "mlp.hpp"

namespace cfrx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float softplus_f(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoid_f(float z) { return 1.f / (1.f + expf(-z)); }
constexpr float LOG_CUT = -30.f;  // below: log softplus(z) = z, sigmoid(z) / softplus(z) = 1

// ---- tiled GEMM ---------------------------------------------------------------------------
// C[M][N] = sum_k A(m, k) B(k, n) over one K range per block (grid z = split).  A(m, k) is
// A[m * lda + k] (row major) or, with A_T, At[k * lda + m]; B(k, n) is B[k * ldb + n] or, with
// B_T, Bt[n * ldb + k].  Block tile 64 x 64 x 32, four wavefronts of 32 x 32 each; both operand
// tiles are staged in LDS k-contiguous so every MFMA operand is one 16-byte LDS read.
constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;  // LDS row stride 80 bytes

enum { EPI_BIAS_RELU = 0, EPI_GRAD_MASK = 1, EPI_PARTIAL = 2 };

struct GemmArgs {
    const uint16_t *A, *B;
    int M, N, K, lda, ldb, kchunk;
    const float *bias;      // EPI_BIAS_RELU: relu(acc + bias[n]) -> bf16
    const uint16_t *mask;   // EPI_GRAD_MASK: acc where mask[m][n] > 0, else 0 -> bf16
    uint16_t *C16;          // [M][N] bf16
    float *C32;             // EPI_PARTIAL: [split][M][N]
};

template <bool A_T, bool B_T, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[BM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int k_beg = blockIdx.z * g.kchunk;
    const int k_end = min(g.K, k_beg + g.kchunk);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x16 acc;
    for (int i = 0; i < 16; i++) acc[i] = 0.f;
    for (int k0 = k_beg; k0 < k_end; k0 += BK) {
        if (!A_T) {  // 64 rows x 4 chunks of 8 k
            const int m = tid >> 2, kk = (tid & 3) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (m0 + m < g.M && k0 + kk < k_end) v = *(const uint4 *)(g.A + (int64_t)(m0 + m) * g.lda + k0 + kk);
            *(uint4 *)&As[m][kk] = v;
        } else {     // 32 k x 8 chunks of 8 m, transposed into LDS
            const int kk = tid >> 3, m = (tid & 7) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (k0 + kk < k_end && m0 + m < g.M) v = *(const uint4 *)(g.A + (int64_t)(k0 + kk) * g.lda + m0 + m);
            const uint16_t *e = (const uint16_t *)&v;
#pragma unroll
            for (int j = 0; j < 8; j++) As[m + j][kk] = e[j];
        }
        if (B_T) {   // 64 columns x 4 chunks of 8 k
            const int n = tid >> 2, kk = (tid & 3) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (n0 + n < g.N && k0 + kk < k_end) v = *(const uint4 *)(g.B + (int64_t)(n0 + n) * g.ldb + k0 + kk);
            *(uint4 *)&Bs[n][kk] = v;
        } else {     // 32 k x 8 chunks of 8 n, transposed into LDS
            const int kk = tid >> 3, n = (tid & 7) * 8;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (k0 + kk < k_end && n0 + n < g.N) v = *(const uint4 *)(g.B + (int64_t)(k0 + kk) * g.ldb + n0 + n);
            const uint16_t *e = (const uint16_t *)&v;
#pragma unroll
            for (int j = 0; j < 8; j++) Bs[n + j][kk] = e[j];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            // lane l supplies row (col) l % 32 and k = ks + 8 (l / 32) .. + 7 of both operands
            const bf16x8 a = *(const bf16x8 *)&As[wm + (lane & 31)][ks + (lane >> 5) * 8];
            const bf16x8 b = *(const bf16x8 *)&Bs[wn + (lane & 31)][ks + (lane >> 5) * 8];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator i of lane l holds row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32
    const int col = n0 + wn + (lane & 31);
    if (col >= g.N) return;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int row = m0 + wm + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
        if (row >= g.M) continue;
        float x = acc[i];
        const int64_t o = (int64_t)row * g.N + col;
        if (EPI == EPI_BIAS_RELU) {
            g.C16[o] = to_bf16(fmaxf(x + g.bias[col], 0.f));
        } else if (EPI == EPI_GRAD_MASK) {
            g.C16[o] = to_bf16(from_bf16(g.mask[o]) > 0.f ? x : 0.f);
        } else {
            g.C32[(int64_t)blockIdx.z * g.M * g.N + o] = x;
        }
    }
}

// ---- output layer, loss and its gradient ---------------------------------------------------
struct HeadArgs {
    const uint16_t *H;      // [rows][hidden] last hidden activations
    const uint16_t *W;      // [hidden][4] bf16 output weights
    const float *b;         // [4]
    const float *T;         // [rows][4] target distribution (training)
    const float *w;         // [rows] row weights or nullptr (training)
    const uint8_t *nact;    // [rows] legal actions (training; clamped to 1..4)
    const float *inv_wsum;  // device scalar 1 / sum of row weights (training)
    int rows;
    float *z;               // [rows][4] logits (inference)
    uint16_t *dA;           // [rows][hidden] gradient of the last hidden pre-activation (training)
    float *part;            // [gridDim.x][hidden * 4 + 5] block partials (training)
};

template <int HPL, bool TRAIN>
__global__ __launch_bounds__(256) void k_head(HeadArgs a) {
    constexpr int HID = 64 * HPL;
    constexpr int NP = HID * 4 + 5;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float wk[HPL][4];
#pragma unroll
    for (int j = 0; j < HPL; j++)
#pragma unroll
        for (int c = 0; c < 4; c++) wk[j][c] = from_bf16(a.W[(lane * HPL + j) * 4 + c]);
    float gw[HPL][4], gb[4] = {0.f, 0.f, 0.f, 0.f}, gl = 0.f;
#pragma unroll
    for (int j = 0; j < HPL; j++)
#pragma unroll
        for (int c = 0; c < 4; c++) gw[j][c] = 0.f;
    const float invw = TRAIN ? *a.inv_wsum : 0.f;
    for (int r = blockIdx.x * 4 + wave; r < a.rows; r += gridDim.x * 4) {
        float h[HPL];
        const uint16_t *hr = a.H + (int64_t)r * HID + lane * HPL;
#pragma unroll
        for (int j = 0; j < HPL; j++) h[j] = from_bf16(hr[j]);
        float z[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < HPL; j++) s = fmaf(h[j], wk[j][c], s);
            z[c] = s;
        }
        // butterfly: every lane ends with the same sums
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int c = 0; c < 4; c++) z[c] += __shfl_xor(z[c], off, 64);
#pragma unroll
        for (int c = 0; c < 4; c++) z[c] += a.b[c];
        if (!TRAIN) {
            if (lane < 4) a.z[(int64_t)r * 4 + lane] = lane == 0 ? z[0] : lane == 1 ? z[1] : lane == 2 ? z[2] : z[3];
            continue;
        }
        const int n = min(max((int)a.nact[r], 1), 4);
        const float wr = (a.w ? a.w[r] : 1.f) * invw;
        float ls[4], lmax = -INFINITY;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            ls[c] = z[c] < LOG_CUT ? z[c] : logf(softplus_f(z[c]));
            if (c < n) lmax = fmaxf(lmax, ls[c]);
        }
        float se = 0.f;
#pragma unroll
        for (int c = 0; c < 4; c++)
            if (c < n) se += expf(ls[c] - lmax);
        const float lS = lmax + logf(se);
        float tsum = 0.f, ce = 0.f, t[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            t[c] = c < n ? a.T[(int64_t)r * 4 + c] : 0.f;
            tsum += t[c];
            ce -= t[c] * (ls[c] - lS);
        }
        float dz[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            if (c < n) {
                const float ratio = z[c] < LOG_CUT ? 1.f : sigmoid_f(z[c]) / softplus_f(z[c]);
                const float lsig = -softplus_f(-z[c]);
                dz[c] = wr * (-t[c] * ratio + tsum * expf(lsig - lS));
            } else {
                dz[c] = 0.f;
            }
        }
        uint16_t *dr = a.dA + (int64_t)r * HID + lane * HPL;
#pragma unroll
        for (int j = 0; j < HPL; j++) {
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < 4; c++) d = fmaf(dz[c], wk[j][c], d);
            dr[j] = to_bf16(h[j] > 0.f ? d : 0.f);
#pragma unroll
            for (int c = 0; c < 4; c++) gw[j][c] = fmaf(h[j], dz[c], gw[j][c]);
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < 4; c++) gb[c] += dz[c];
            gl += wr * ce;
        }
    }
    if (!TRAIN) return;
    __shared__ float red[4][NP];
#pragma unroll
    for (int j = 0; j < HPL; j++)
#pragma unroll
        for (int c = 0; c < 4; c++) red[wave][(lane * HPL + j) * 4 + c] = gw[j][c];
    if (lane == 0) {
        for (int c = 0; c < 4; c++) red[wave][HID * 4 + c] = gb[c];
        red[wave][HID * 4 + 4] = gl;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NP; i += 256)
        a.part[(int64_t)blockIdx.x * NP + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// 1 / sum of the row weights (rows when there are none); one block, fixed order
__global__ __launch_bounds__(256) void k_inv_wsum(const float *w, int rows, float *out) {
    __shared__ float s[256];
    float acc = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) acc += w ? w[r] : 1.f;
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0] > 0.f ? 1.f / s[0] : 0.f;
}

// part[b][n] = sum of rows [b * chunk, (b + 1) * chunk) of column n (bias gradients)
__global__ __launch_bounds__(256) void k_colsum(const uint16_t *X, int rows, int N, int chunk, float *part) {
    const int r0 = blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
    for (int n = threadIdx.x; n < N; n += 256) {
        float s = 0.f;
#pragma unroll 8
        for (int r = r0; r < r1; r++) s += from_bf16(X[(int64_t)r * N + n]);
        part[(int64_t)blockIdx.x * N + n] = s;
    }
}

// out[j] = sum over b of part[b * stride + j], in order of b
__global__ void k_reduce(const float *part, int nb, int64_t stride, int n, float *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.f;
#pragma unroll 8
    for (int b = 0; b < nb; b++) s += part[(int64_t)b * stride + j];
    out[j] = s;
}

// Adam (Kingma and Ba 2015, Algorithm 1) on the FP32 master copy; refreshes the bf16 copy.
// c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) for step t.
__global__ void k_adam(float *theta, const float *g, float *m, float *v, uint16_t *theta16, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    theta[i] = th;
    theta16[i] = to_bf16(th);
}

__global__ void k_to_bf16(const float *x, uint16_t *y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// ---- fused inference ------------------------------------------------------------------------
// Inference needs no activations outside the kernel, so one launch runs every layer: a block takes
// FB_ROWS rows, keeps their activations in LDS from the input row to the last hidden layer, and
// writes only the four logits.  Each hidden layer is the product of the LDS activations with the
// layer's weights, streamed through LDS in chunks of 32 input units (double-buffered, the next
// chunk's global loads in flight while the matrix cores work on the current one); the four waves
// each own a 64-row x HID/2-column slab (2 x HID/64 accumulators of 32 x 32).  The arithmetic is the
// layer-by-layer path's, in its order: the same MFMA on the same 16-wide k steps from k = 0 up,
// relu(acc + bias) rounded to bf16, and the output layer's per-lane FMA chain, butterfly and bias
// of k_head, so the logits are bitwise those of the layered kernels.
constexpr int FB_ROWS = 128, FB_BK = 32, FB_LDB = FB_BK + 8;

struct FusedArgs {
    const uint16_t *x;        // [rows][K0] bf16
    const uint16_t *wt;       // hidden layers' weights transposed, layer l at wt_off[l]: [HID][fin_l]
    const float *theta;       // FP32 parameters (biases at boff[l])
    const uint16_t *w_out;    // [HID][4] bf16 output weights
    const float *b_out;       // [4]
    int64_t wt_off[4], boff[4];
    int rows, n_hidden;
    float *z;                 // [rows][4]
};

template <int HID, int K0>
__global__ __launch_bounds__(256) void k_mlp_fused(FusedArgs f) {
    constexpr int LDA = (K0 > HID ? K0 : HID) + 8;   // LDS row stride (bf16), rows stay 16-byte aligned
    constexpr int CT = HID / 64;                     // 32-wide column tiles per wave
    __shared__ __attribute__((aligned(16))) uint16_t act[FB_ROWS * LDA];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][HID * FB_LDB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.x * FB_ROWS;
    // the block's input rows (zeros past the last row)
    for (int i = tid; i < FB_ROWS * K0 / 8; i += 256) {
        const int r = i / (K0 / 8), c = (i % (K0 / 8)) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (r0 + r < f.rows) v = *(const uint4 *)(f.x + (int64_t)(r0 + r) * K0 + c);
        *(uint4 *)&act[r * LDA + c] = v;
    }
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * (HID / 2);
    for (int l = 0; l < f.n_hidden; l++) {
        const int K = l == 0 ? K0 : HID;
        const uint16_t *W = f.wt + f.wt_off[l];
        // chunk k0 of W^T: HID rows of 32 units = HID * 4 16-byte pieces, CT per thread
        uint4 pre[CT];
        auto load_chunk = [&](int k0) {
#pragma unroll
            for (int j = 0; j < CT; j++) {
                const int idx = tid + j * 256, n = idx >> 2, q = (idx & 3) * 8;
                pre[j] = *(const uint4 *)(W + (int64_t)n * K + k0 + q);
            }
        };
        auto store_chunk = [&](int buf) {
#pragma unroll
            for (int j = 0; j < CT; j++) {
                const int idx = tid + j * 256, n = idx >> 2, q = (idx & 3) * 8;
                *(uint4 *)&Bs[buf][n * FB_LDB + q] = pre[j];
            }
        };
        f32x16 acc[2][CT];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < CT; b++)
#pragma unroll
                for (int i = 0; i < 16; i++) acc[a][b][i] = 0.f;
        load_chunk(0);
        store_chunk(0);
        __syncthreads();
        const int nk = K / FB_BK;
        for (int kc = 0; kc < nk; kc++) {
            const int buf = kc & 1;
            if (kc + 1 < nk) load_chunk((kc + 1) * FB_BK);
#pragma unroll
            for (int ks = 0; ks < FB_BK; ks += 16) {
                // lane l supplies row (column) l % 32 and k = ks + 8 (l / 32) .. + 7 of both operands
                bf16x8 av[2], bv[CT];
#pragma unroll
                for (int a = 0; a < 2; a++)
                    av[a] = *(const bf16x8 *)&act[(wm + a * 32 + (lane & 31)) * LDA + kc * FB_BK + ks + (lane >> 5) * 8];
#pragma unroll
                for (int b = 0; b < CT; b++)
                    bv[b] = *(const bf16x8 *)&Bs[buf][(wn + b * 32 + (lane & 31)) * FB_LDB + ks + (lane >> 5) * 8];
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < CT; b++)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
            if (kc + 1 < nk) store_chunk(buf ^ 1);
            __syncthreads();
        }
        // every wave has read this layer's input: overwrite it with relu(acc + bias) in bf16
        // (accumulator i of lane l holds row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32)
        const float *bias = f.theta + f.boff[l];
#pragma unroll
        for (int b = 0; b < CT; b++) {
            const int col = wn + b * 32 + (lane & 31);
            const float bc = bias[col];
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int i = 0; i < 16; i++) {
                    const int row = wm + a * 32 + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
                    act[row * LDA + col] = to_bf16(fmaxf(acc[a][b][i] + bc, 0.f));
                }
        }
        __syncthreads();
    }
    // output layer as k_head computes it: lane l holds hidden units l * HPL .. + HPL - 1
    constexpr int HPL = HID / 64;
    float wk[HPL][4];
#pragma unroll
    for (int j = 0; j < HPL; j++)
#pragma unroll
        for (int c = 0; c < 4; c++) wk[j][c] = from_bf16(f.w_out[(lane * HPL + j) * 4 + c]);
    const float bo0 = f.b_out[0], bo1 = f.b_out[1], bo2 = f.b_out[2], bo3 = f.b_out[3];
    for (int rr = wave; rr < FB_ROWS && r0 + rr < f.rows; rr += 4) {
        float h[HPL];
#pragma unroll
        for (int j = 0; j < HPL; j++) h[j] = from_bf16(act[rr * LDA + lane * HPL + j]);
        float z[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            float sum = 0.f;
#pragma unroll
            for (int j = 0; j < HPL; j++) sum = fmaf(h[j], wk[j][c], sum);
            z[c] = sum;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int c = 0; c < 4; c++) z[c] += __shfl_xor(z[c], off, 64);
        z[0] += bo0; z[1] += bo1; z[2] += bo2; z[3] += bo3;
        if (lane < 4) f.z[(int64_t)(r0 + rr) * 4 + lane] = lane == 0 ? z[0] : lane == 1 ? z[1] : lane == 2 ? z[2] : z[3];
    }
}

// wt[n * fin + k] = W[k * HID + n] for one hidden layer (bf16 copies, so the fused kernel's weight
// chunks are contiguous per output unit)
__global__ void k_transpose_bf16(const uint16_t *W, int fin, int hid, uint16_t *wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)fin * hid) return;
    const int n = (int)(i / fin), k = (int)(i % fin);
    wt[i] = W[(int64_t)k * hid + n];
}

// minibatch rows idx[r] (clamped into [0, n_data)) of the training arrays into staging
__global__ void k_gather_rows(const uint16_t *X, const float *T, const float *w, const uint8_t *nact,
                              const int32_t *idx, int rows, int64_t n_data, int feat, uint16_t *Xs, float *Ts,
                              float *ws, uint8_t *ns) {
    const int r = blockIdx.x;
    if (r >= rows) return;
    const int64_t s = min(max((int64_t)idx[r], (int64_t)0), n_data - 1);
    for (int c = threadIdx.x; c < feat; c += blockDim.x) Xs[(int64_t)r * feat + c] = X[s * feat + c];
    if (threadIdx.x < 4) Ts[(int64_t)r * 4 + threadIdx.x] = T[s * 4 + threadIdx.x];
    if (threadIdx.x == 0) {
        ws[r] = w ? w[s] : 1.f;
        ns[r] = nact[s];
    }
}

// ---- compiled game <-> network rows --------------------------------------------------------
// Columns 120-127 after a probe run: the current strategy (regret matching of the latest regrets)
// and the normalised average strategy over the first four actions (uniform where the sum is 0;
// zero for sets of more than four actions).  One thread per set writes the 16-byte chunk.
template <typename T>
__global__ __launch_bounds__(256) void k_features_probe(FeatureArgs f, const T *sigma, const double *sbar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.I) return;
    const int off = f.canon_off[i], n = f.canon_off[i + 1] - off;
    float col[8];
#pragma unroll
    for (int j = 0; j < 8; j++) col[j] = 0.f;
    if (n <= 4) {
        double sb[4] = {0, 0, 0, 0}, tot = 0.0;
        for (int a = 0; a < n; a++) {
            const int q = f.slot_map ? f.slot_map[off + a] : off + a;
            col[a] = (float)sigma[q];
            sb[a] = sbar[q];
            tot += sb[a];
        }
        for (int a = 0; a < n; a++) col[4 + a] = tot > 0.0 ? (float)(sb[a] / tot) : (float)(1.0 / n);
    }
    uint16_t o[8];
#pragma unroll
    for (int j = 0; j < 8; j++) o[j] = to_bf16(col[j]);
    *(uint4 *)(f.X + i * 128 + 120) = *(const uint4 *)o;
}

// Feature row of information set i (16 threads per row, 8 columns each), and mag[i], the sum of
// the magnitudes of those regrets (the unit of the warm-start regrets):
//   0-63 one-hot hand bucket, 64-95 one-hot public-history code, 96-103 caller scalars,
//   104-107 legal-action mask, 108-111 the first four instantaneous regrets of the uniform
//   strategy over the sum of their magnitudes, 112-115 regret matching (plus) of those regrets,
//   116 acting player (0 / 1), 117-119 zero, 120-127 the strategies of a probe run (uniform here;
//   k_features_probe overwrites them after one).
template <typename T>
__global__ __launch_bounds__(256) void k_features(FeatureArgs f, const T *R) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t >> 4;
    const int chunk = (int)(t & 15);
    if (i >= f.I) return;
    float col[8];
#pragma unroll
    for (int j = 0; j < 8; j++) col[j] = 0.f;
    const int c0 = chunk * 8;
    if (c0 < 64) {
        const int b = f.bucket[i];
        if (b >= c0 && b < c0 + 8) col[b - c0] = 1.f;
    } else if (c0 < 96) {
        const int hcode = f.history[i];
        if (hcode >= c0 - 64 && hcode < c0 - 56) col[hcode - (c0 - 64)] = 1.f;
    } else if (c0 == 96) {
#pragma unroll
        for (int j = 0; j < 8; j++) col[j] = f.scalars[i * 8 + j];
    } else if (c0 == 104 || c0 == 112) {
        const int off = f.canon_off[i], n = f.canon_off[i + 1] - off;
        const int k = min(n, 4);
        double r[4] = {0, 0, 0, 0}, sa = 0.0, sp = 0.0;
        if (n <= 4)
            for (int a = 0; a < k; a++) {
                const int q = f.slot_map ? f.slot_map[off + a] : off + a;
                r[a] = (double)R[q];
                sa += fabs(r[a]);
                sp += r[a] > 0.0 ? r[a] : 0.0;
            }
        if (c0 == 104) {
            f.mag[i] = n <= 4 ? (float)sa : 0.f;
            for (int a = 0; a < k; a++) col[a] = 1.f;
            if (n <= 4 && sa > 0.0)
                for (int a = 0; a < k; a++) col[4 + a] = (float)(r[a] / sa);
        } else {
            if (n <= 4)
                for (int a = 0; a < k; a++) col[a] = sp > 0.0 ? (float)((r[a] > 0.0 ? r[a] : 0.0) / sp) : (float)(1.0 / k);
            col[4] = f.player[i] == 2 ? 1.f : 0.f;
        }
    } else if (c0 == 120) {
        const int n = f.canon_off[i + 1] - f.canon_off[i];
        if (n <= 4)
            for (int a = 0; a < n; a++) col[a] = col[4 + a] = (float)(1.0 / n);
    }
    uint16_t o[8];
#pragma unroll
    for (int j = 0; j < 8; j++) o[j] = to_bf16(col[j]);
    *(uint4 *)(f.X + i * 128 + c0) = *(const uint4 *)o;
}

// R0 over canonical slots: scale * mag(I) * softplus(z) for the legal actions of sets with <= 4
// actions, 0 (the uniform strategy) for larger sets
__global__ void k_warm_regrets(const int32_t *canon_off, int64_t I, const float *z, const float *mag, float scale,
                               float *R0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I) return;
    const int off = canon_off[i], n = canon_off[i + 1] - off;
    const float c = scale * mag[i];
    for (int a = 0; a < n; a++) R0[off + a] = n <= 4 ? c * softplus_f(z[i * 4 + a]) : 0.f;
}

}  // namespace

hipError_t launch_features(const FeatureArgs &f, const void *R, bool fp64, hipStream_t s) {
    if (f.I == 0) return hipSuccess;
    const int64_t threads = f.I * 16;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (fp64) k_features<double><<<blocks, 256, 0, s>>>(f, (const double *)R);
    else k_features<float><<<blocks, 256, 0, s>>>(f, (const float *)R);
    return hipGetLastError();
}

hipError_t launch_features_probe(const FeatureArgs &f, const void *sigma, const double *sbar, bool fp64,
                                 hipStream_t s) {
    if (f.I == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((f.I + 255) / 256);
    if (fp64) k_features_probe<double><<<blocks, 256, 0, s>>>(f, (const double *)sigma, sbar);
    else k_features_probe<float><<<blocks, 256, 0, s>>>(f, (const float *)sigma, sbar);
    return hipGetLastError();
}

hipError_t launch_warm_regrets(const int32_t *canon_off, int64_t I, const float *z, const float *mag, float scale,
                               float *R0, hipStream_t s) {
    if (I == 0) return hipSuccess;
    k_warm_regrets<<<(unsigned)((I + 255) / 256), 256, 0, s>>>(canon_off, I, z, mag, scale, R0);
    return hipGetLastError();
}

}  // namespace cfrx

using namespace cfrx;

// ---- the network handle ---------------------------------------------------------------------
struct cfr_mlp {
    cfr_mlp_desc d{};
    std::vector<int> fin, fout;          // per layer
    std::vector<int64_t> woff, boff;     // offsets into the flat parameter vector
    int64_t P = 0;
    int64_t step = 0;
    int splits_max = 32;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *part = nullptr, *inv_w = nullptr,
          *lossd = nullptr;
    uint16_t *theta16 = nullptr;
    uint16_t *wt = nullptr;              // hidden layers' bf16 weights transposed (fused inference)
    int64_t wt_off[4] = {0, 0, 0, 0};
    std::vector<uint16_t *> H;           // [n_hidden] activations, [max_rows][hidden]
    uint16_t *dA[2] = {nullptr, nullptr};
    uint16_t *xs = nullptr;              // gathered minibatch
    float *ts = nullptr, *ws = nullptr;
    uint8_t *ns = nullptr;
    std::vector<void *> allocs;
};

namespace {
cfr_status mfail(cfr_status s, const std::string &m) {
    set_last_error(m);
    return s;
}

#define MHIP(expr)                                                                                      \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return mfail(CFR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
cfr_status malloc_dev(cfr_mlp *n, T **p, int64_t count) {
    void *q = nullptr;
    const size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return mfail(CFR_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    n->allocs.push_back(q);
    *p = (T *)q;
    return CFR_OK;
}

void free_mlp(cfr_mlp *n) {
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
}

int gemm_splits(int rows, int cap) {
    int s = (rows + 255) / 256;
    return s < 1 ? 1 : (s > cap ? cap : s);
}

template <bool A_T, bool B_T, int EPI>
hipError_t gemm(const GemmArgs &g, int splits, hipStream_t s) {
    dim3 grid((unsigned)((g.M + BM - 1) / BM), (unsigned)((g.N + BN - 1) / BN), (unsigned)splits);
    k_gemm<A_T, B_T, EPI><<<grid, 256, 0, s>>>(g);
    return hipGetLastError();
}

hipError_t head(const cfr_mlp *n, const HeadArgs &a, bool train, int blocks, hipStream_t s) {
    const int hpl = n->d.hidden / 64;
#define HEAD(H_)                                                                                   \
    if (hpl == H_) {                                                                               \
        if (train) k_head<H_, true><<<blocks, 256, 0, s>>>(a);                                     \
        else k_head<H_, false><<<blocks, 256, 0, s>>>(a);                                          \
        return hipGetLastError();                                                                  \
    }
    HEAD(1) HEAD(2) HEAD(4)
#undef HEAD
    return hipErrorInvalidValue;
}

constexpr int HEAD_BLOCKS = 256;

// forward pass of `rows` (<= the buffers' rows) rows; hidden layer l writes its activations to act(l)
template <typename Act>
cfr_status forward_rows_into(cfr_mlp *n, const uint16_t *x, int rows, float *z, bool train, Act act, hipStream_t s) {
    const int L = n->d.n_hidden;
    const uint16_t *in = x;
    for (int l = 0; l < L; l++) {
        GemmArgs g{};
        g.A = in; g.B = n->theta16 + n->woff[l];
        g.M = rows; g.N = n->fout[l]; g.K = n->fin[l]; g.lda = n->fin[l]; g.ldb = n->fout[l]; g.kchunk = g.K;
        g.bias = n->theta + n->boff[l]; g.C16 = act(l);
        MHIP((gemm<false, false, EPI_BIAS_RELU>(g, 1, s)));
        in = act(l);
    }
    if (!train) {
        HeadArgs a{};
        a.H = act(L - 1); a.W = n->theta16 + n->woff[L]; a.b = n->theta + n->boff[L]; a.rows = rows; a.z = z;
        const int blocks = std::min(HEAD_BLOCKS, (rows + 3) / 4);
        MHIP(head(n, a, false, blocks, s));
    }
    return CFR_OK;
}

// forward pass of `rows` (<= max_rows) rows; leaves the hidden activations in n->H (training reads them)
cfr_status forward_rows(cfr_mlp *n, const uint16_t *x, int rows, float *z, bool train, hipStream_t s) {
    return forward_rows_into(n, x, rows, z, train, [n](int l) { return n->H[(size_t)l]; }, s);
}

// ---- the allocation-free inference entry point: its activations live in a file-scope device array ----
// Two ping-pong buffers of NOALLOC_ROWS rows x 256 hidden units (bf16): 8 MiB that every GPU the
// library runs on holds for the life of the process.  In host code `noalloc_scratch` is the symbol's
// host-side stand-in, never a device address: its device address is looked up once per device.
constexpr int NOALLOC_ROWS = 8192;
constexpr int NOALLOC_HIDDEN = 256;
static __device__ __align__(256) uint16_t noalloc_scratch[2 * NOALLOC_ROWS * NOALLOC_HIDDEN];

constexpr int MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
uint16_t *g_noalloc_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch (the device must be current); looked up on first use.
cfr_status noalloc_scratch_ptr(int device, uint16_t **out) {
    if (device < 0 || device >= MAX_DEVICES) return mfail(CFR_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p)
            return mfail(CFR_EDEVICE, std::string("hipGetSymbolAddress of the inference scratch: ") + hipGetErrorString(e));
        g_noalloc_ptr[device] = (uint16_t *)p;
    }
    *out = g_noalloc_ptr[device];
    return CFR_OK;
}

bool valid_desc(const cfr_mlp_desc *d, std::string &why) {
    auto ok_dim = [](int v) { return v == 64 || v == 128 || v == 256; };
    if (!ok_dim(d->in_dim)) { why = "in_dim must be 64, 128 or 256"; return false; }
    if (!ok_dim(d->hidden)) { why = "hidden must be 64, 128 or 256"; return false; }
    if (d->n_hidden < 1 || d->n_hidden > 4) { why = "n_hidden must be in [1, 4]"; return false; }
    if (d->max_rows < 1 || d->max_rows > (1 << 20)) { why = "max_rows must be in [1, 2^20]"; return false; }
    if (!(d->beta1 >= 0.f && d->beta1 < 1.f && d->beta2 >= 0.f && d->beta2 < 1.f && d->eps > 0.f)) {
        why = "Adam constants out of range"; return false;
    }
    return true;
}

}  // namespace

extern "C" {

void cfr_mlp_default_desc(cfr_mlp_desc *d) {
    if (!d) return;
    std::memset(d, 0, sizeof *d);
    d->in_dim = CFR_FEATURES;
    d->hidden = 256;
    d->n_hidden = 3;
    d->max_rows = 4096;
    d->device = 0;
    d->beta1 = 0.9f;
    d->beta2 = 0.999f;
    d->eps = 1e-8f;
}

cfr_status cfr_mlp_create(const cfr_mlp_desc *desc, cfr_mlp **out) {
    if (!out) return mfail(CFR_EINVAL, "out is NULL");
    *out = nullptr;
    cfr_mlp_desc d;
    cfr_mlp_default_desc(&d);
    if (desc) d = *desc;
    std::string why;
    if (!valid_desc(&d, why)) return mfail(CFR_EINVAL, why);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return mfail(CFR_EDEVICE, "no HIP device available");
    if (d.device < 0 || d.device >= ndev) return mfail(CFR_EINVAL, "device ordinal out of range");
    MHIP(hipSetDevice(d.device));
    cfr_mlp *n = new cfr_mlp();
    n->d = d;
    int prev = d.in_dim;
    for (int l = 0; l <= d.n_hidden; l++) {
        const int fo = l < d.n_hidden ? d.hidden : CFR_MLP_OUT;
        n->fin.push_back(prev);
        n->fout.push_back(fo);
        n->woff.push_back(n->P);
        n->P += (int64_t)prev * fo;
        n->boff.push_back(n->P);
        n->P += fo;
        prev = fo;
    }
    const int64_t R = d.max_rows;
    const int64_t hid = d.hidden;
    const int64_t maxw = std::max<int64_t>((int64_t)d.in_dim * hid, hid * hid);
    cfr_status st = CFR_OK;
#define MA(p, c) do { st = malloc_dev(n, &(p), (c)); if (st != CFR_OK) { free_mlp(n); return st; } } while (0)
    MA(n->theta, n->P); MA(n->grad, n->P); MA(n->m, n->P); MA(n->v, n->P); MA(n->theta16, n->P);
    MA(n->part, std::max<int64_t>(std::max<int64_t>((int64_t)n->splits_max * maxw, (int64_t)HEAD_BLOCKS * (hid * 4 + 5)),
                                  (R + 15) / 16 * hid));
    {
        int64_t off = 0;
        for (int l = 0; l < d.n_hidden; l++) { n->wt_off[l] = off; off += (int64_t)n->fin[(size_t)l] * hid; }
        MA(n->wt, off);
    }
    MA(n->inv_w, 1);
    MA(n->lossd, 1);
    n->H.resize((size_t)d.n_hidden);
    for (int l = 0; l < d.n_hidden; l++) MA(n->H[(size_t)l], R * hid);
    MA(n->dA[0], R * hid); MA(n->dA[1], R * hid);
    MA(n->xs, R * d.in_dim); MA(n->ts, R * 4); MA(n->ws, R); MA(n->ns, R);
#undef MA
    // zero parameters until the caller sets them
    hipError_t e = hipMemset(n->theta, 0, (size_t)n->P * 4);
    if (e == hipSuccess) e = hipMemset(n->theta16, 0, (size_t)n->P * 2);
    if (e == hipSuccess) e = hipMemset(n->m, 0, (size_t)n->P * 4);
    if (e == hipSuccess) e = hipMemset(n->v, 0, (size_t)n->P * 4);
    if (e == hipSuccess) e = hipMemset(n->grad, 0, (size_t)n->P * 4);
    if (e != hipSuccess) { free_mlp(n); return mfail(CFR_EDEVICE, std::string("hipMemset: ") + hipGetErrorString(e)); }
    *out = n;
    return CFR_OK;
}

cfr_status cfr_mlp_num_params(cfr_mlp *n, int64_t *count) {
    if (!n || !count) return mfail(CFR_EINVAL, "NULL argument");
    *count = n->P;
    return CFR_OK;
}

cfr_status cfr_mlp_set_params(cfr_mlp *n, const float *params, int64_t len) {
    if (!n || !params) return mfail(CFR_EINVAL, "NULL argument");
    if (len != n->P) return mfail(CFR_EINVAL, "len must equal the parameter count " + std::to_string(n->P));
    MHIP(hipSetDevice(n->d.device));
    MHIP(hipDeviceSynchronize());
    MHIP(hipMemcpy(n->theta, params, (size_t)len * 4, hipMemcpyHostToDevice));
    MHIP(hipMemset(n->m, 0, (size_t)len * 4));
    MHIP(hipMemset(n->v, 0, (size_t)len * 4));
    k_to_bf16<<<(unsigned)((len + 255) / 256), 256>>>(n->theta, n->theta16, len);
    MHIP(hipGetLastError());
    MHIP(hipDeviceSynchronize());
    n->step = 0;
    return CFR_OK;
}

cfr_status cfr_mlp_get(cfr_mlp *n, int which, float *dst, int64_t len) {
    if (!n || !dst) return mfail(CFR_EINVAL, "NULL argument");
    if (len != n->P) return mfail(CFR_EINVAL, "len must equal the parameter count " + std::to_string(n->P));
    const float *src = which == CFR_MLP_PARAMS ? n->theta : which == CFR_MLP_GRADS ? n->grad
                     : which == CFR_MLP_ADAM_M ? n->m : which == CFR_MLP_ADAM_V ? n->v : nullptr;
    if (!src) return mfail(CFR_EINVAL, "unknown buffer");
    MHIP(hipSetDevice(n->d.device));
    MHIP(hipDeviceSynchronize());
    MHIP(hipMemcpy(dst, src, (size_t)len * 4, hipMemcpyDeviceToHost));
    return CFR_OK;
}

cfr_status cfr_mlp_forward(cfr_mlp *n, const void *x, int64_t rows, float *z, void *stream) {
    if (!n || ((!x || !z) && rows > 0) || rows < 0) return mfail(CFR_EINVAL, "bad argument");
    MHIP(hipSetDevice(n->d.device));
    hipStream_t s = (hipStream_t)stream;
    if (rows == 0) return CFR_OK;
    // the weights as they are now (set_params and every Adam step change them), transposed
    for (int l = 0; l < n->d.n_hidden; l++) {
        const int64_t cnt = (int64_t)n->fin[(size_t)l] * n->d.hidden;
        k_transpose_bf16<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(n->theta16 + n->woff[(size_t)l], n->fin[(size_t)l],
                                                                      n->d.hidden, n->wt + n->wt_off[l]);
        MHIP(hipGetLastError());
    }
    FusedArgs f{};
    f.wt = n->wt; f.theta = n->theta;
    f.w_out = n->theta16 + n->woff[(size_t)n->d.n_hidden];
    f.b_out = n->theta + n->boff[(size_t)n->d.n_hidden];
    for (int l = 0; l < n->d.n_hidden; l++) { f.wt_off[l] = n->wt_off[l]; f.boff[l] = n->boff[(size_t)l]; }
    f.n_hidden = n->d.n_hidden;
    // launches of at most 2^20 blocks (2^27 rows) each keep every row index in int
    const int64_t step = (int64_t)FB_ROWS << 20;
    for (int64_t r0 = 0; r0 < rows; r0 += step) {
        f.rows = (int)std::min(step, rows - r0);
        f.x = (const uint16_t *)x + r0 * n->d.in_dim;
        f.z = z + r0 * 4;
        const unsigned blocks = (unsigned)((f.rows + FB_ROWS - 1) / FB_ROWS);
#define FUSED(H_, K_)                                                                              \
        if (n->d.hidden == H_ && n->d.in_dim == K_) k_mlp_fused<H_, K_><<<blocks, 256, 0, s>>>(f); else
        FUSED(64, 64) FUSED(64, 128) FUSED(64, 256) FUSED(128, 64) FUSED(128, 128) FUSED(128, 256)
        FUSED(256, 64) FUSED(256, 128) FUSED(256, 256)
        return mfail(CFR_EINVAL, "unsupported network shape");
#undef FUSED
        MHIP(hipGetLastError());
    }
    return CFR_OK;
}

cfr_status cfr_mlp_forward_noalloc(cfr_mlp *n, const void *x, int64_t rows, float *z, void *stream) {
    if (!n || ((!x || !z) && rows > 0) || rows < 0) return mfail(CFR_EINVAL, "bad argument");
    if (rows > NOALLOC_ROWS)
        return mfail(CFR_EINVAL, "cfr_mlp_forward_noalloc takes at most " + std::to_string(NOALLOC_ROWS) +
                                 " rows per call (" + std::to_string(rows) + " given)");
    if (n->d.hidden > NOALLOC_HIDDEN) return mfail(CFR_EINVAL, "hidden width above the scratch's 256 units");
    MHIP(hipSetDevice(n->d.device));
    uint16_t *buf = nullptr;
    cfr_status st = noalloc_scratch_ptr(n->d.device, &buf);
    if (st != CFR_OK || rows == 0) return st;
    // hidden layer l writes buffer l % 2 and reads the other one (the rows come in x for layer 0)
    const size_t half = (size_t)NOALLOC_ROWS * NOALLOC_HIDDEN;
    return forward_rows_into(n, (const uint16_t *)x, (int)rows, z, false,
                             [buf, half](int l) { return buf + (size_t)(l & 1) * half; }, (hipStream_t)stream);
}

cfr_status cfr_mlp_backward(cfr_mlp *n, const void *x, const float *target, const float *weight,
                            const uint8_t *nact, const int32_t *idx, int64_t n_data, int64_t rows, double *loss,
                            void *stream) {
    if (!n || !x || !target || !nact || rows <= 0) return mfail(CFR_EINVAL, "bad argument");
    if (rows > n->d.max_rows) return mfail(CFR_EINVAL, "rows exceeds max_rows " + std::to_string(n->d.max_rows));
    if (idx && n_data <= 0) return mfail(CFR_EINVAL, "n_data must be positive with an index list");
    MHIP(hipSetDevice(n->d.device));
    hipStream_t s = (hipStream_t)stream;
    const int R = (int)rows, L = n->d.n_hidden, F = n->d.in_dim, HID = n->d.hidden;
    const uint16_t *X = (const uint16_t *)x;
    const float *T = target, *W = weight;
    const uint8_t *NA = nact;
    if (idx) {
        k_gather_rows<<<R, 128, 0, s>>>(X, T, W, NA, idx, R, n_data, F, n->xs, n->ts, n->ws, n->ns);
        MHIP(hipGetLastError());
        X = n->xs; T = n->ts; W = n->ws; NA = n->ns;
    }
    k_inv_wsum<<<1, 256, 0, s>>>(W, R, n->inv_w);
    MHIP(hipGetLastError());
    cfr_status st = forward_rows(n, X, R, nullptr, true, s);
    if (st != CFR_OK) return st;
    // output layer: loss, gradient of the last hidden pre-activation, block partials
    HeadArgs a{};
    a.H = n->H[L - 1]; a.W = n->theta16 + n->woff[L]; a.b = n->theta + n->boff[L];
    a.T = T; a.w = W; a.nact = NA; a.inv_wsum = n->inv_w; a.rows = R;
    a.dA = n->dA[0]; a.part = n->part;
    const int hb = std::min(HEAD_BLOCKS, (R + 3) / 4);
    MHIP(head(n, a, true, hb, s));
    const int NP = HID * 4 + 5;
    // grad of W_out (HID*4), b_out (4) and the loss (1) are contiguous in the partial rows; the
    // flat layout puts b_out right after W_out, so one reduction writes both, the loss goes to inv_w[0]
    k_reduce<<<(unsigned)((HID * 4 + 4 + 255) / 256), 256, 0, s>>>(n->part, hb, NP, HID * 4 + 4, n->grad + n->woff[L]);
    MHIP(hipGetLastError());
    k_reduce<<<1, 64, 0, s>>>(n->part + HID * 4 + 4, hb, NP, 1, n->lossd);
    MHIP(hipGetLastError());
    // hidden layers, last to first
    int cur = 0;
    for (int l = L - 1; l >= 0; l--) {
        const uint16_t *hin = l > 0 ? n->H[(size_t)l - 1] : X;
        const int fi = n->fin[(size_t)l], fo = n->fout[(size_t)l];
        // weight gradient: sum over rows of hin[r][m] dA[r][n] (split over rows)
        const int splits = gemm_splits(R, n->splits_max);
        int kchunk = (R + splits - 1) / splits;
        kchunk = (kchunk + BK - 1) / BK * BK;
        const int used = (R + kchunk - 1) / kchunk;
        GemmArgs g{};
        g.A = hin; g.B = n->dA[cur]; g.M = fi; g.N = fo; g.K = R; g.lda = fi; g.ldb = fo; g.kchunk = kchunk;
        g.C32 = n->part;
        MHIP((gemm<true, false, EPI_PARTIAL>(g, used, s)));
        k_reduce<<<(unsigned)(((int64_t)fi * fo + 255) / 256), 256, 0, s>>>(n->part, used, (int64_t)fi * fo, fi * fo,
                                                                        n->grad + n->woff[(size_t)l]);
        MHIP(hipGetLastError());
        // bias gradient
        const int cchunk = 16;   // R / 16 blocks: enough to fill the device
        const int cb = (R + cchunk - 1) / cchunk;
        k_colsum<<<cb, 256, 0, s>>>(n->dA[cur], R, fo, cchunk, n->part);
        MHIP(hipGetLastError());
        k_reduce<<<(unsigned)((fo + 255) / 256), 256, 0, s>>>(n->part, cb, fo, fo, n->grad + n->boff[(size_t)l]);
        MHIP(hipGetLastError());
        if (l > 0) {
            // gradient of the previous pre-activation: (dA W_l^T) masked by hin > 0
            GemmArgs q{};
            q.A = n->dA[cur]; q.B = n->theta16 + n->woff[(size_t)l];
            q.M = R; q.N = fi; q.K = fo; q.lda = fo; q.ldb = fo; q.kchunk = fo;
            q.mask = hin; q.C16 = n->dA[cur ^ 1];
            MHIP((gemm<false, true, EPI_GRAD_MASK>(q, 1, s)));
            cur ^= 1;
        }
    }
    if (loss) {
        float lh = 0.f;
        MHIP(hipMemcpyAsync(&lh, n->lossd, 4, hipMemcpyDeviceToHost, s));
        MHIP(hipStreamSynchronize(s));
        *loss = lh;
    }
    return CFR_OK;
}

cfr_status cfr_mlp_adam(cfr_mlp *n, float lr, void *stream) {
    if (!n) return mfail(CFR_EINVAL, "NULL argument");
    if (!(lr >= 0.f)) return mfail(CFR_EINVAL, "lr must be >= 0");
    MHIP(hipSetDevice(n->d.device));
    n->step++;
    const double t = (double)n->step;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)n->d.beta1, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)n->d.beta2, t)));
    k_adam<<<(unsigned)((n->P + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        n->theta, n->grad, n->m, n->v, n->theta16, n->P, lr, n->d.beta1, n->d.beta2, n->d.eps, c1, c2);
    MHIP(hipGetLastError());
    return CFR_OK;
}

cfr_status cfr_mlp_train_step(cfr_mlp *n, const void *x, const float *target, const float *weight,
                              const uint8_t *nact, const int32_t *idx, int64_t n_data, int64_t rows, float lr,
                              double *loss, void *stream) {
    cfr_status st = cfr_mlp_backward(n, x, target, weight, nact, idx, n_data, rows, loss, stream);
    if (st != CFR_OK) return st;
    return cfr_mlp_adam(n, lr, stream);
}

void cfr_mlp_destroy(cfr_mlp *n) {
    if (!n) return;
    (void)hipSetDevice(n->d.device);
    (void)hipDeviceSynchronize();
    free_mlp(n);
}

}  // extern "C"

namespace cfrx {
cfr_status mlp_forward_internal(cfr_mlp *n, const void *x, int64_t rows, float *z, hipStream_t s) {
    return cfr_mlp_forward(n, x, rows, z, s);
}
int mlp_in_dim(const cfr_mlp *n) { return n->d.in_dim; }
int mlp_device(const cfr_mlp *n) { return n->d.device; }
}  // namespace cfrx
