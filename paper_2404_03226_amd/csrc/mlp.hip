// Learned cost model: a 32 -> 256 -> 256 -> 2 ReLU network predicting the
// natural log of a task's duration on each worker kind, trained with MSE and
// Adam.  The paper drives inspiring efficiency with per-kind execution-time
// estimates gathered by a cost model (Sections 4.3 and 5); this model replaces
// the per-type average table when task features are available.
//
// Precision: weights, activations and activation gradients are stored as
// bfloat16 (round to nearest even); products accumulate in fp32 on the MFMA
// units (v_mfma_f32_16x16x32_bf16); biases, outputs, weight gradients, Adam
// moments and master weights are fp32.
//
// Packed parameter order: W1 [32,256], b1 [256], W2 [256,256], b2 [256],
// W3 [256,2], b3 [2].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

constexpr int kIn = 32, kHid = 256, kOut = 2;
constexpr int64_t kMaxTrainSteps = 1 << 28;  // steps of one insp_mlp_train call
constexpr int32_t kTrainChunk = 32;          // steps per captured graph
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kIn * kHid, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
                  kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kOut, kParams = kOffB3 + kOut;
static_assert(kParams == 74754, "parameter count");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950); f2bf2
// converts two values with one instruction, a in the low half
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ GEMM
// C[m,n] = sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak], B(k,n) =
// B[k*sbk + n*sbn] (bf16), accumulated in fp32, then: + bias[n], ReLU,
// * (mask(m,n) > 0), stored to C32 (fp32) and/or C16 (bf16); colpart gets
// each 64-row tile's column sums of the final fp32 values (summed later in a
// fixed order, so training is bit-reproducible).  64 x 64 tile per 256-thread block; each wave owns a
// 32 x 32 quarter as 2 x 2 MFMA 16x16x32 tiles; K advances 32 at a time
// through LDS (A row-major, B transposed so both fragments are 16-byte reads).
// Staging reads 8 consecutive bf16 per thread (16 bytes) along whichever
// index of an operand is contiguous in memory (amode/bmode 1: k, 2: m or n;
// 0: element by element).  With ksplit > 1, block z of the grid's third
// dimension sums K range [z kchunk, (z + 1) kchunk) into C32 + z pstride
// (partials, reduced in z order by k_ksum); no epilogue then.
struct GemmArgs {
    int M, N, K;
    const uint16_t *A;
    int64_t sam, sak;
    const uint16_t *B;
    int64_t sbk, sbn;
    const float *bias;
    int relu;
    const uint16_t *mask;
    int64_t smm, smn;
    float *C32;
    int64_t ldc;
    uint16_t *C16;
    int64_t ldc16;
    float *colpart;  // [ceil(M/64)][N] per-tile column sums of the final values
    int amode, bmode;
    int ksplit, kchunk;
    int64_t pstride;
};

constexpr int kTM = 64, kTN = 64, kTK = 32, kLdsRow = kTK + 8;

// K sub-tiles staged per global round trip.  Deeper panels (8, all of a
// 256-deep K in one trip) measured no faster on the training shapes, whose
// kernels sit near the per-launch floor, and cost 4x the LDS.
constexpr int kSub = 1;

// One operand tile, T[r][kk] = X(r0 + r, k0 + kk) with X(r, k) =
// X[r sr + k sk], zero outside rows < R and k < kend, as 8 bf16 per thread:
// mode 2 (sr == 1) thread = (k, 8 consecutive rows), one 16-byte read (the
// host guarantees R % 8 == 0 and alignment); otherwise thread = (row, 8
// consecutive k), one 16-byte read in mode 1 (sk == 1), 8 single reads in
// mode 0.  Loading and storing are split so that a whole panel's reads are
// in flight together.
__device__ __forceinline__ uint4 load_tile(const uint16_t *X, int64_t sr, int64_t sk, int mode, int R, int r0, int k0,
                                           int kend, int tid) {
    uint4 v = {0u, 0u, 0u, 0u};
    if (mode == 2) {
        const int kk = tid >> 3, r = (tid & 7) * 8;
        if (r0 + r < R && k0 + kk < kend)
            v = *reinterpret_cast<const uint4 *>(X + (int64_t)(k0 + kk) * sk + (r0 + r));
    } else if (mode == 1) {
        const int r = tid >> 2, kk = (tid & 3) * 8;
        if (r0 + r < R && k0 + kk < kend)
            v = *reinterpret_cast<const uint4 *>(X + (int64_t)(r0 + r) * sr + (k0 + kk));
    } else {
        const int r = tid >> 2, kk = (tid & 3) * 8;
        uint32_t h[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int rr = r0 + r, k = k0 + kk + i;
            h[i] = (rr < R && k < kend) ? X[(int64_t)rr * sr + (int64_t)k * sk] : 0u;
        }
        v = uint4{h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16, h[6] | h[7] << 16};
    }
    return v;
}

__device__ __forceinline__ void store_tile(uint4 v, int mode, int tid, uint16_t *T) {
    if (mode == 2) {
        const int kk = tid >> 3, r = (tid & 7) * 8;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            T[(r + 2 * j) * kLdsRow + kk] = (uint16_t)(w[j] & 0xFFFFu);
            T[(r + 2 * j + 1) * kLdsRow + kk] = (uint16_t)(w[j] >> 16);
        }
    } else {
        const int r = tid >> 2, kk = (tid & 3) * 8;
        *reinterpret_cast<uint4 *>(&T[r * kLdsRow + kk]) = v;
    }
}

// One 64x64 output tile (bx, by) of g, K split bz when g.ksplit > 1.
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int bx, int by, int bz) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kSub][kTM * kLdsRow];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kSub][kTN * kLdsRow];
    __shared__ float cpart[2 * kTN];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m0 = by * kTM, n0 = bx * kTN;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kbeg = g.ksplit > 1 ? bz * g.kchunk : 0;
    const int kend = g.ksplit > 1 ? min(g.K, kbeg + g.kchunk) : g.K;
    for (int k0 = kbeg; k0 < kend; k0 += kSub * kTK) {
        // stage kSub tiles of A [64 x 32] and B^T [64 x 32]: all reads first
        const int ns = min(kSub, (kend - k0 + kTK - 1) / kTK);
        uint4 ra[kSub], rb[kSub];
#pragma unroll
        for (int j = 0; j < kSub; j++) {
            if (j >= ns) break;
            ra[j] = load_tile(g.A, g.sam, g.sak, g.amode, g.M, m0, k0 + j * kTK, kend, tid);
            rb[j] = load_tile(g.B, g.sbn, g.sbk, g.bmode, g.N, n0, k0 + j * kTK, kend, tid);
        }
#pragma unroll
        for (int j = 0; j < kSub; j++) {
            if (j >= ns) break;
            store_tile(ra[j], g.amode, tid, As[j]);
            store_tile(rb[j], g.bmode, tid, Bs[j]);
        }
        __syncthreads();
        const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
        for (int j = 0; j < kSub; j++) {
            if (j >= ns) break;
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int a = 0; a < 2; a++)
                af[a] = *reinterpret_cast<const bf16x8 *>(&As[j][(wm + a * 16 + fr) * kLdsRow + fk]);
#pragma unroll
            for (int b = 0; b < 2; b++)
                bfr[b] = *reinterpret_cast<const bf16x8 *>(&Bs[j][(wn + b * 16 + fr) * kLdsRow + fk]);
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator layout: value i of a lane is row 4*(lane/16)+i, column lane%16
    if (g.ksplit > 1) {
        float *P = g.C32 + (int64_t)bz * g.pstride;
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int n = n0 + wn + b * 16 + (lane & 15);
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int m = m0 + wm + a * 16 + (lane >> 4) * 4 + i;
                    if (m < g.M && n < g.N) P[(int64_t)m * g.ldc + n] = acc[a][b][i];
                }
        }
        return;
    }
#pragma unroll
    for (int b = 0; b < 2; b++) {
        const int n = n0 + wn + b * 16 + (lane & 15);
        float csum = 0.f;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int m = m0 + wm + a * 16 + (lane >> 4) * 4 + i;
                if (m < g.M && n < g.N) {
                    float v = acc[a][b][i];
                    if (g.bias) v += g.bias[n];
                    if (g.relu) v = fmaxf(v, 0.f);
                    if (g.mask && !(bf2f(g.mask[(int64_t)m * g.smm + (int64_t)n * g.smn]) > 0.f)) v = 0.f;
                    if (g.C32) g.C32[(int64_t)m * g.ldc + n] = v;
                    if (g.C16) g.C16[(int64_t)m * g.ldc16 + n] = f2bf(v);
                    csum += v;
                }
            }
        if (g.colpart) {
            // rows of this lane group, then the four lane groups in order
            const float c0 = __shfl(csum, (lane & 15), 64), c1 = __shfl(csum, (lane & 15) + 16, 64);
            const float c2 = __shfl(csum, (lane & 15) + 32, 64), c3 = __shfl(csum, (lane & 15) + 48, 64);
            if (lane < 16) cpart[(wv >> 1) * kTN + wn + b * 16 + lane] = ((c0 + c1) + c2) + c3;
        }
    }
    if (g.colpart) {
        __syncthreads();
        // the two row halves of the tile, in order; one partial per M-tile
        if (tid < kTN && n0 + tid < g.N)
            g.colpart[(int64_t)by * g.N + n0 + tid] = cpart[tid] + cpart[kTN + tid];
    }
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) { gemm_tile(g, blockIdx.x, blockIdx.y, blockIdx.z); }

// Two independent products in one launch: blocks [0, n0) take g0's tiles
// (x fastest, then y, then the K split), the rest g1's.
__global__ __launch_bounds__(256) void k_gemm2(GemmArgs g0, int gx0, int gy0, int n0, GemmArgs g1, int gx1,
                                                int gy1) {
    int b = blockIdx.x;
    if (b < n0) {
        gemm_tile(g0, b % gx0, b / gx0 % gy0, b / (gx0 * gy0));
    } else {
        b -= n0;
        gemm_tile(g1, b % gx1, b / gx1 % gy1, b / (gx1 * gy1));
    }
}

// Column c of a [rows][cols] array of partial sums, summed by a 1024-thread
// block that owns 64 columns: wave w adds its contiguous share of the rows in
// row order, then the 16 wave sums are added in wave order (a fixed order,
// so the result is reproducible).  Every thread of the block must call it.
__device__ __forceinline__ float col_sum(const float *part, int rows, int cols, int c) {
    __shared__ float red[16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int per = (rows + 15) / 16, r0 = min(rows, w * per), r1 = min(rows, r0 + per);
    float s = 0.f;
    if (c < cols) {
#pragma unroll 8
        for (int r = r0; r < r1; r++) s += part[(int64_t)r * cols + c];
    }
    red[w][lane] = s;
    __syncthreads();
    float t = red[0][lane];
#pragma unroll
    for (int i = 1; i < 16; i++) t += red[i][lane];
    return t;
}

__global__ __launch_bounds__(1024) void k_colreduce(const float *part, int rows, int cols, float *out) {
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const float t = col_sum(part, rows, cols, c);
    if (threadIdx.x < 64 && c < cols) out[c] = t;
}

// k_colreduce over its first `cb` work-groups and, in the others, the sum of
// S split-K partials (k_ksum's order), one output per thread: two
// independent reductions in one launch.
__global__ __launch_bounds__(1024) void k_colreduce_ksum(const float *part, int rows, int cols, float *out, int cb,
                                                          const float *kpart, int S, int64_t pstride, int64_t n,
                                                          float *kout) {
    if ((int)blockIdx.x < cb) {
        const int c = blockIdx.x * 64 + (threadIdx.x & 63);
        const float t = col_sum(part, rows, cols, c);
        if (threadIdx.x < 64 && c < cols) out[c] = t;
        return;
    }
    const int64_t i = (int64_t)(blockIdx.x - cb) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = kpart[i];
#pragma unroll 8
    for (int z = 1; z < S; z++) s += kpart[z * pstride + i];
    kout[i] = s;
}

// -------------------------------------------------------------- helpers
__global__ void k_to_bf16(const float *x, uint16_t *y, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_fill(float *x, int64_t n, float v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Output layer and loss gradient, one wave per row (4 rows per block):
// Y = H2 W3 + b3; with a target T: dY = 2 (Y - T) / (2B), dH2 = (dY W3^T) *
// (H2 > 0) stored as bf16, and per-block partials (in row order) of db2,
// db3 and the loss into `part` [blocks][kHid + 3].
__global__ __launch_bounds__(256) void k_out(const uint16_t *H2, const uint16_t *W3, const float *b3, int64_t rows,
                                             float *Y, const float *T, float *part, uint16_t *dH2,
                                             int32_t *est) {
    __shared__ float rowg[4][kHid];
    __shared__ float rowx[4][3];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t r = blockIdx.x * 4LL + wv;
    float w30[4], w31[4], h[4];
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int i = lane * 4 + j;
        w30[j] = bf2f(W3[i * 2]);
        w31[j] = bf2f(W3[i * 2 + 1]);
        h[j] = r < rows ? bf2f(H2[r * kHid + i]) : 0.f;
        s0 += h[j] * w30[j];
        s1 += h[j] * w31[j];
    }
    for (int off = 32; off >= 1; off >>= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
    }
    const float y0 = s0 + b3[0], y1 = s1 + b3[1];
    if (r < rows && lane == 0) {
        if (Y) {
            Y[2 * r] = y0;
            Y[2 * r + 1] = y1;
        }
        if (est) {
            // integer estimate: clamp(rint(exp(y)), 1, 2^20)
            est[2 * r] = (int32_t)fminf(fmaxf(rintf(expf(y0)), 1.f), (float)(1 << 20));
            est[2 * r + 1] = (int32_t)fminf(fmaxf(rintf(expf(y1)), 1.f), (float)(1 << 20));
        }
    }
    if (!T) return;
    const float scale = 1.0f / (float)rows;  // 2 / (2 rows)
    float d0 = 0.f, d1 = 0.f, l2 = 0.f;
    if (r < rows) {
        const float e0 = y0 - T[2 * r], e1 = y1 - T[2 * r + 1];
        d0 = e0 * scale;
        d1 = e1 * scale;
        l2 = (e0 * e0 + e1 * e1) * 0.5f * scale;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int i = lane * 4 + j;
        float gv = d0 * w30[j] + d1 * w31[j];
        if (!(h[j] > 0.f) || r >= rows) gv = 0.f;
        if (r < rows) dH2[r * kHid + i] = f2bf(gv);
        rowg[wv][i] = gv;
    }
    if (lane == 0) {
        rowx[wv][0] = d0;
        rowx[wv][1] = d1;
        rowx[wv][2] = l2;
    }
    __syncthreads();
    float *pp = part + (int64_t)blockIdx.x * (kHid + 3);
    pp[tid] = ((rowg[0][tid] + rowg[1][tid]) + rowg[2][tid]) + rowg[3][tid];
    if (tid < 3) pp[kHid + tid] = ((rowx[0][tid] + rowx[1][tid]) + rowx[2][tid]) + rowx[3][tid];
}

// db2, db3 and the loss from k_out's per-block partials [rows][kHid + 3].
// Under graph-captured training (tab) this also advances the step index
// tab[0]: the step's minibatch is staged by then and Adam reads tab[0] - 1.
__global__ __launch_bounds__(1024) void k_reduce_out(const float *part, int rows, float *grads, float *loss,
                                                      int32_t *tab) {
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const float t = col_sum(part, rows, kHid + 3, c);
    if (threadIdx.x < 64) {
        if (c < kHid) grads[kOffB2 + c] = t;
        else if (c < kHid + 2) grads[kOffB3 + (c - kHid)] = t;
        else if (c == kHid + 2) loss[0] = t;
    }
    if (tab && blockIdx.x == 0 && threadIdx.x == 0) tab[0] += 1;
}

// dW3[i, c] = sum_r H2[r, i] dY[r, c]; dY recomputed from Y and T.
__global__ __launch_bounds__(256) void k_dw3(const uint16_t *H2, const float *Y, const float *T, int64_t rows,
                                             float *grads) {
    const int i = blockIdx.x;  // hidden unit
    const float scale = 1.0f / (float)rows;
    float a0 = 0.f, a1 = 0.f;
    for (int64_t r = threadIdx.x; r < rows; r += 256) {
        const float h = bf2f(H2[r * kHid + i]);
        a0 += h * (Y[2 * r] - T[2 * r]) * scale;
        a1 += h * (Y[2 * r + 1] - T[2 * r + 1]) * scale;
    }
    __shared__ float s0[256], s1[256];
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s0[threadIdx.x] += s0[threadIdx.x + off];
            s1[threadIdx.x] += s1[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        grads[kOffW3 + 2 * i] = s0[0];
        grads[kOffW3 + 2 * i + 1] = s1[0];
    }
}

// Adam (Kingma and Ba) with bias correction, then the bf16 weight shadows.
// With a table `tab` (graph-captured training) the corrections of the
// current step are read from it instead: tab[0] - 1 is the step index i
// within the call (advanced by k_reduce_out), tab[1 + 2i] and tab[2 + 2i]
// hold 1 - 0.9^step and 1 - 0.999^step as computed by the host for the eager
// step, so both routes round alike.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float bc1, float bc2,
                       uint16_t *w1, uint16_t *w2, uint16_t *w3, const int32_t *tab, int32_t tabn) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (tab) {
        const int32_t s = min(max(tab[0] - 1, 0), tabn - 1);
        bc1 = __int_as_float(tab[1 + 2 * s]);
        bc2 = __int_as_float(tab[2 + 2 * s]);
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (i < kOffB1) w1[i - kOffW1] = f2bf(pi);
    else if (i >= kOffW2 && i < kOffB2) w2[i - kOffW2] = f2bf(pi);
    else if (i >= kOffW3 && i < kOffB3) w3[i - kOffW3] = f2bf(pi);
}

// Minibatch of graph-captured training: rows [o, o + rows) of x (to bf16)
// and of t (copied), o = rows * (tab[0] mod steps), so one captured step
// serves every minibatch of an epoch.
__global__ void k_stage(const float *x, const float *t, const int32_t *tab, int32_t steps, int64_t rows,
                        uint16_t *xb, float *ts) {
    const int64_t o = rows * (int64_t)((uint32_t)tab[0] % (uint32_t)steps);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < rows * kIn) xb[i] = f2bf(x[o * kIn + i]);
    if (i < rows * kOut) ts[i] = t[o * kOut + i];
}

__global__ void k_shadow(const float *p, uint16_t *w1, uint16_t *w2, uint16_t *w3) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < kOffB1) w1[i] = f2bf(p[i]);
    else if (i >= kOffW2 && i < kOffB2) w2[i - kOffW2] = f2bf(p[i]);
    else if (i >= kOffW3 && i < kOffB3) w3[i - kOffW3] = f2bf(p[i]);
}

// Fused inference: y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3 and the
// integer estimates, for many rows.  A block of NW waves is persistent over
// 64-row tiles; wave w owns hidden columns [w C, w C + C), C = 256 / NW, of
// both layers and keeps their W1 and W2 MFMA B-fragments in registers for the
// whole run.  Per tile: layer 1 (K = 32) from x straight into MFMA
// fragments, bf16 hidden activations through LDS, layer 2 (K = 256) from LDS
// fragments, then the two outputs as per-wave partial dot products summed in
// a fixed order.  Both layers are computed transposed (weights as the A
// operand), so that a lane's accumulator holds consecutive hidden units of
// one row.  With NW = 8 the fragments take half the registers of
// NW = 4, so two waves share each SIMD and one's MFMA overlaps the other's
// conversions and LDS traffic.
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

// ReLU of two packed bf16 values at once: a bf16 is negative exactly when its
// bit pattern is as a 16-bit integer, and rounding keeps the sign, so this is
// the rounding of max(x, 0) (with -0 turned into +0).
__device__ __forceinline__ uint32_t relu_bf2(uint32_t q) {
    const s16x2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, q), z));
}
constexpr int kRT = 64, kH1Row = kHid + 8;

constexpr int kInferWaves = 8;

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_infer(const float *x, int64_t rows, const uint16_t *W1, const float *b1,
                                                    const uint16_t *W2, const float *b2, const uint16_t *W3,
                                                    const float *b3, float *Y, int32_t *est) {
    constexpr int CT = kHid / NW / 16;  // 16-column MFMA tiles per wave
    __shared__ __attribute__((aligned(16))) uint16_t H1s[kRT * kH1Row];
    __shared__ float yp[NW][kRT][2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wn = wv * (kHid / NW), lc = lane & 15, lk = (lane >> 4) * 8;
    bf16x8 w1f[CT], w2f[8][CT];
    float bias1[CT][4], bias2[CT][4];
    bf16x2_t w30[CT][2], w31[CT][2];  // output weights of hidden units (i, i + 1), as packed bf16 pairs
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
        const int n = wn + ct * 16 + lc;
        u16x8 t;
#pragma unroll
        for (int i = 0; i < 8; i++) t[i] = W1[(lk + i) * kHid + n];
        w1f[ct] = __builtin_bit_cast(bf16x8, t);
#pragma unroll
        for (int ks = 0; ks < 8; ks++) {
#pragma unroll
            for (int i = 0; i < 8; i++) t[i] = W2[(ks * 32 + lk + i) * kHid + n];
            w2f[ks][ct] = __builtin_bit_cast(bf16x8, t);
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            // the hidden unit this lane's accumulator value i holds in either layer
            const int h = wn + ct * 16 + (lane >> 4) * 4 + i;
            bias1[ct][i] = b1[h];
            bias2[ct][i] = b2[h];
        }
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
            const int h = wn + ct * 16 + (lane >> 4) * 4 + i;
            w30[ct][i / 2] = __builtin_bit_cast(bf16x2_t, (uint32_t)W3[h * 2] | (uint32_t)W3[h * 2 + 2] << 16);
            w31[ct][i / 2] = __builtin_bit_cast(bf16x2_t, (uint32_t)W3[h * 2 + 1] | (uint32_t)W3[h * 2 + 3] << 16);
        }
    }
    const float b30 = b3[0], b31 = b3[1];
    const int64_t tiles = (rows + kRT - 1) / kRT;
    // features of the next tile are read while the current one is in layer 2
    float4 xa[4], xb[4];
    auto load_x = [&](int64_t t0) {
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            const int64_t r = t0 * kRT + rt * 16 + lc;
            if (r < rows) {
                xa[rt] = *reinterpret_cast<const float4 *>(x + r * kIn + lk);
                xb[rt] = *reinterpret_cast<const float4 *>(x + r * kIn + lk + 4);
            } else {
                xa[rt] = float4{0.f, 0.f, 0.f, 0.f};
                xb[rt] = float4{0.f, 0.f, 0.f, 0.f};
            }
        }
    };
    if ((int64_t)blockIdx.x < tiles) load_x(blockIdx.x);
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t r0 = tile * kRT;
        // layer 1: A-fragment row lc of each 16-row tile, K = lk .. lk+7
        bf16x8 af1[4];
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            const uint4 t = {f2bf2(xa[rt].x, xa[rt].y), f2bf2(xa[rt].z, xa[rt].w), f2bf2(xb[rt].x, xb[rt].y),
                             f2bf2(xb[rt].z, xb[rt].w)};
            af1[rt] = __builtin_bit_cast(bf16x8, t);
        }
        if (tile + gridDim.x < tiles) load_x(tile + gridDim.x);
        // computed transposed (W1^T as the A operand), so that a lane holds 4
        // consecutive hidden units of one row and stores them as one 8-byte write
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
                f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f[ct], af1[rt], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0,
                                                                    0);
                uint2 h;
                h.x = relu_bf2(f2bf2(acc[0] + bias1[ct][0], acc[1] + bias1[ct][1]));
                h.y = relu_bf2(f2bf2(acc[2] + bias1[ct][2], acc[3] + bias1[ct][3]));
                *reinterpret_cast<uint2 *>(&H1s[(rt * 16 + lc) * kH1Row + wn + ct * 16 + (lane >> 4) * 4]) = h;
            }
        }
        __syncthreads();
        // layer 2, transposed as well: per 16-column tile a lane holds 4
        // consecutive hidden units of row rt * 16 + lc, so its output partials
        // cover 4 CT units and only the 4 lane groups of a row remain to be added
        float p0[4], p1[4];
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            f32x4 acc[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ct++) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 8; ks++) {
                const bf16x8 hf = *reinterpret_cast<const bf16x8 *>(&H1s[(rt * 16 + lc) * kH1Row + ks * 32 + lk]);
#pragma unroll
                for (int ct = 0; ct < CT; ct++)
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2f[ks][ct], hf, acc[ct], 0, 0, 0);
            }
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int ct = 0; ct < CT; ct++)
#pragma unroll
                for (int i = 0; i < 4; i += 2) {
                    // the bf16 rounding of H2, two units per conversion, and
                    // their products with the output weights as one bf16 dot
                    // product per output
                    const bf16x2_t q = __builtin_bit_cast(
                        bf16x2_t, relu_bf2(f2bf2(acc[ct][i] + bias2[ct][i], acc[ct][i + 1] + bias2[ct][i + 1])));
                    s0 = __builtin_amdgcn_fdot2_f32_bf16(q, w30[ct][i / 2], s0, false);
                    s1 = __builtin_amdgcn_fdot2_f32_bf16(q, w31[ct][i / 2], s1, false);
                }
            p0[rt] = s0;
            p1[rt] = s1;
        }
        // lanes lc, lc + 16, lc + 32, lc + 48 hold the same row
#pragma unroll
        for (int rt = 0; rt < 4; rt++) {
            float s0 = p0[rt], s1 = p1[rt];
            s0 += __shfl_xor(s0, 16, 64);
            s1 += __shfl_xor(s1, 16, 64);
            s0 += __shfl_xor(s0, 32, 64);
            s1 += __shfl_xor(s1, 32, 64);
            if (lane < 16) {
                yp[wv][rt * 16 + lc][0] = s0;
                yp[wv][rt * 16 + lc][1] = s1;
            }
        }
        __syncthreads();
        if (tid < kRT * 2) {
            const int row = tid >> 1, c = tid & 1;
            const int64_t r = r0 + row;
            if (r < rows) {
                float y = yp[0][row][c];
#pragma unroll
                for (int w = 1; w < NW; w++) y += yp[w][row][c];
                y += c ? b31 : b30;
                if (Y) Y[2 * r + c] = y;
                if (est) est[2 * r + c] = (int32_t)fminf(fmaxf(rintf(expf(y)), 1.f), (float)(1 << 20));
            }
        }
        __syncthreads();
    }
}

static unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// out[i] = sum over z = 0 .. S-1, in order, of part[z pstride + i].
__global__ void k_ksum(const float *part, int S, int64_t pstride, int64_t n, float *out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = part[i];
#pragma unroll 8
    for (int z = 1; z < S; z++) s += part[z * pstride + i];
    out[i] = s;
}

constexpr int64_t kKSplitFloats = 16 * kHid * kHid;  // split-K partial buffer

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Launch C = A B.  A plain fp32 product with a contiguous C (ldc == N) and
// few output tiles splits K over the partial buffer `kpart`
// (kKSplitFloats floats) so that the grid fills the chip.
// A product's launch shape: operand read modes, the output tiles (gx, gy)
// and, for a plain fp32 output when kpart is given, a split of K over S
// work-groups whose partials go to kpart (out: where their sum belongs).
struct GemmPlan {
    int gx, gy, S;
    float *out;
};
static GemmPlan gemm_plan(GemmArgs &g, float *kpart) {
    g.amode = (g.sak == 1 && g.sam % 8 == 0 && g.K % 8 == 0 && aligned16(g.A)) ? 1
              : (g.sam == 1 && g.sak % 8 == 0 && g.M % 8 == 0 && aligned16(g.A)) ? 2 : 0;
    g.bmode = (g.sbk == 1 && g.sbn % 8 == 0 && g.K % 8 == 0 && aligned16(g.B)) ? 1
              : (g.sbn == 1 && g.sbk % 8 == 0 && g.N % 8 == 0 && aligned16(g.B)) ? 2 : 0;
    GemmPlan pl;
    pl.gx = (g.N + kTN - 1) / kTN;
    pl.gy = (g.M + kTM - 1) / kTM;
    pl.out = g.C32;
    const int kt = (g.K + kTK - 1) / kTK;
    int S = 1;
    if (kpart && g.C32 && !g.C16 && !g.bias && !g.relu && !g.mask && !g.colpart && g.ldc == g.N) {
        const int64_t mn = (int64_t)g.M * g.N;
        S = std::min<int64_t>({(int64_t)kt, std::max(1, 256 / (pl.gx * pl.gy)),
                               kKSplitFloats / std::max<int64_t>(mn, 1)});
        if (S > 1) {
            g.kchunk = ((kt + S - 1) / S) * kTK;
            S = (g.K + g.kchunk - 1) / g.kchunk;
        }
    }
    pl.S = std::max(S, 1);
    g.ksplit = pl.S;
    if (pl.S > 1) {
        g.pstride = (int64_t)g.M * g.N;
        g.C32 = kpart;
    }
    return pl;
}

static void gemm(hipStream_t st, GemmArgs g, float *kpart = nullptr) {
    const GemmPlan pl = gemm_plan(g, kpart);
    hipLaunchKernelGGL(k_gemm, dim3(pl.gx, pl.gy, pl.S), dim3(256), 0, st, g);
    if (pl.S > 1)
        hipLaunchKernelGGL(k_ksum, dim3(blocks(g.pstride, 256)), dim3(256), 0, st, kpart, pl.S, g.pstride, g.pstride,
                           pl.out);
}

}  // namespace insp

using namespace insp;

struct insp_mlp {
    int device = 0;
    int64_t step = 0;
    DevBuf p, g, m, v;            // fp32 [kParams]
    DevBuf w1, w2, w3;            // bf16 shadows
    DevBuf loss;                  // fp32 [1]
    int64_t cap = 0;              // rows the activation buffers hold
    DevBuf xb, h1, h2, dh2, dh1;  // bf16 activations and gradients
    DevBuf y;                     // fp32 [cap, 2]
    DevBuf part;                  // fp32 partial sums for the fixed-order reductions
    DevBuf kpart;                 // fp32 [kKSplitFloats] split-K partial products
    int64_t gen = 0;              // bumped whenever a buffer above moves
    // graph-captured training
    DevBuf ts;                    // fp32 [cap, 2] staged targets
    DevBuf tab;                   // int32 step index, then the bias-correction table
    hipStream_t cs = nullptr;     // capture stream
    hipGraphExec_t exec = nullptr;
    struct Key {
        const float *x, *t;
        int32_t steps, batch, chunk;
        float lr;
        int64_t gen;
        bool operator==(const Key &o) const {
            return x == o.x && t == o.t && steps == o.steps && batch == o.batch && chunk == o.chunk && lr == o.lr &&
                   gen == o.gen;
        }
    } key{};
    ~insp_mlp() {
        // work queued on the caller's streams may still use the graph and buffers
        (void)hipDeviceSynchronize();
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

// Grow the per-row buffers to `rows`.  All-or-nothing: the new buffers are
// allocated beside the old ones and swapped in only when every allocation
// succeeded, so a failure (INSP_E_NOMEM) leaves the model as it was.
static int mlp_reserve(insp_mlp *m, int64_t rows) {
    if (rows <= m->cap) return INSP_OK;
    DevBuf *cur[8] = {&m->xb, &m->h1, &m->h2, &m->dh2, &m->dh1, &m->y, &m->part, &m->ts};
    const size_t bytes[8] = {(size_t)(2 * kIn * rows),  (size_t)(2 * kHid * rows), (size_t)(2 * kHid * rows),
                             (size_t)(2 * kHid * rows), (size_t)(2 * kHid * rows), (size_t)(4 * kOut * rows),
                             (size_t)(4 * ((rows + 3) / 4 + 1) * (kHid + 3)), (size_t)(4 * kOut * rows)};
    DevBuf fresh[8];
    for (int i = 0; i < 8; i++)
        if (int rc = fresh[i].alloc(bytes[i])) return rc;
    for (int i = 0; i < 8; i++) cur[i]->swap(fresh[i]);  // the old buffers are released on return
    m->cap = rows;
    m->gen++;
    return INSP_OK;
}

// Forward over `rows` rows of fp32 features into the bf16 activation buffers
// (x == nullptr: the bf16 features are already staged in m->xb).
static void mlp_forward(insp_mlp *m, const float *x, int64_t rows, hipStream_t st) {
    const float *P = m->p.as<float>();
    if (x)
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks(rows * kIn, 256)), dim3(256), 0, st, x, m->xb.as<uint16_t>(),
                           rows * kIn);
    GemmArgs g;
    memset(&g, 0, sizeof g);
    g.M = (int)rows; g.N = kHid; g.K = kIn;
    g.A = m->xb.as<uint16_t>(); g.sam = kIn; g.sak = 1;
    g.B = m->w1.as<uint16_t>(); g.sbk = kHid; g.sbn = 1;
    g.bias = P + kOffB1; g.relu = 1;
    g.C16 = m->h1.as<uint16_t>(); g.ldc16 = kHid;
    gemm(st, g);
    g.K = kHid;
    g.A = m->h1.as<uint16_t>(); g.sam = kHid;
    g.B = m->w2.as<uint16_t>();
    g.bias = P + kOffB2;
    g.C16 = m->h2.as<uint16_t>();
    gemm(st, g);
}

// Loss and gradients of one batch into m->g; y out optional.  Every sum is
// taken in a fixed order, so a step is bit-reproducible.  With `tab` the
// batch is minibatch tab[0] mod `steps` of x and t (graph-captured training).
static int mlp_backward(insp_mlp *m, const float *x, const float *t, int64_t B, hipStream_t st,
                        int32_t *tab = nullptr, int32_t steps = 0) {
    float *G = m->g.as<float>();
    float *part = m->part.as<float>();
    if (tab) {
        hipLaunchKernelGGL(k_stage, dim3(blocks(B * kIn, 256)), dim3(256), 0, st, x, t, tab, steps, B,
                           m->xb.as<uint16_t>(), m->ts.as<float>());
        x = nullptr;
        t = m->ts.as<float>();
    }
    mlp_forward(m, x, B, st);
    const int ob = (int)((B + 3) / 4);
    hipLaunchKernelGGL(k_out, dim3(ob), dim3(256), 0, st, m->h2.as<uint16_t>(), m->w3.as<uint16_t>(),
                       m->p.as<float>() + kOffB3, B, m->y.as<float>(), t, part, m->dh2.as<uint16_t>(),
                       (int32_t *)nullptr);
    // db2 (256 columns), db3 (2) and the loss (1) from the block partials;
    // with tab the step index advances here
    hipLaunchKernelGGL(k_reduce_out, dim3(blocks(kHid + 3, 64)), dim3(1024), 0, st, part, ob, G,
                       m->loss.as<float>(), tab);
    hipLaunchKernelGGL(k_dw3, dim3(kHid), dim3(256), 0, st, m->h2.as<uint16_t>(), m->y.as<float>(), t, B, G);
    // dW2 = H1^T dH2 (K split over work-groups) and dH1 = (dH2 W2^T) * (H1 > 0)
    // with its per-tile column sums, both from dH2: one launch; then the sum
    // of dW2's partials and db1 (the column sums in order): one more
    GemmArgs g, gh;
    memset(&g, 0, sizeof g);
    g.M = kHid; g.N = kHid; g.K = (int)B;
    g.A = m->h1.as<uint16_t>(); g.sam = 1; g.sak = kHid;
    g.B = m->dh2.as<uint16_t>(); g.sbk = kHid; g.sbn = 1;
    g.C32 = G + kOffW2; g.ldc = kHid;
    const GemmPlan pw = gemm_plan(g, m->kpart.as<float>());
    memset(&gh, 0, sizeof gh);
    gh.M = (int)B; gh.N = kHid; gh.K = kHid;
    gh.A = m->dh2.as<uint16_t>(); gh.sam = kHid; gh.sak = 1;
    gh.B = m->w2.as<uint16_t>(); gh.sbk = 1; gh.sbn = kHid;
    gh.mask = m->h1.as<uint16_t>(); gh.smm = kHid; gh.smn = 1;
    gh.C16 = m->dh1.as<uint16_t>(); gh.ldc16 = kHid;
    gh.colpart = part;
    const GemmPlan ph = gemm_plan(gh, nullptr);
    const int nw = pw.gx * pw.gy * pw.S, nh = ph.gx * ph.gy;
    hipLaunchKernelGGL(k_gemm2, dim3(nw + nh), dim3(256), 0, st, g, pw.gx, pw.gy, nw, gh, ph.gx, ph.gy);
    const int cb = (int)blocks(kHid, 64);
    if (pw.S > 1)
        hipLaunchKernelGGL(k_colreduce_ksum, dim3(cb + (int)blocks(g.pstride, 1024)), dim3(1024), 0, st, part,
                           (int)((B + kTM - 1) / kTM), kHid, G + kOffB1, cb, m->kpart.as<float>(), pw.S, g.pstride,
                           g.pstride, pw.out);
    else
        hipLaunchKernelGGL(k_colreduce, dim3(cb), dim3(1024), 0, st, part, (int)((B + kTM - 1) / kTM), kHid,
                           G + kOffB1);
    // dW1 = X^T dH1
    memset(&g, 0, sizeof g);
    g.M = kIn; g.N = kHid; g.K = (int)B;
    g.A = m->xb.as<uint16_t>(); g.sam = 1; g.sak = kIn;
    g.B = m->dh1.as<uint16_t>(); g.sbk = kHid; g.sbn = 1;
    g.C32 = G + kOffW1; g.ldc = kHid;
    gemm(st, g, m->kpart.as<float>());
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

extern "C" int insp_mlp_create(const float *params, insp_mlp **out) {
    if (!params || !out) return set_error(INSP_E_INVAL, "null argument");
    std::unique_ptr<insp_mlp> m(new insp_mlp());
    INSP_HIP(hipGetDevice(&m->device));
    int rc;
    if ((rc = m->p.alloc(4 * kParams)) || (rc = m->g.alloc(4 * kParams)) || (rc = m->m.alloc(4 * kParams)) ||
        (rc = m->v.alloc(4 * kParams)) || (rc = m->w1.alloc(2 * kIn * kHid)) || (rc = m->w2.alloc(2 * kHid * kHid)) ||
        (rc = m->w3.alloc(2 * kHid * kOut)) || (rc = m->loss.alloc(4)) || (rc = m->kpart.alloc(4 * kKSplitFloats)))
        return rc;
    INSP_HIP(hipMemcpy(m->p.p, params, 4 * kParams, hipMemcpyHostToDevice));
    INSP_HIP(hipMemset(m->m.p, 0, 4 * kParams));
    INSP_HIP(hipMemset(m->v.p, 0, 4 * kParams));
    hipLaunchKernelGGL(k_shadow, dim3(blocks(kParams, 256)), dim3(256), 0, 0, m->p.as<float>(), m->w1.as<uint16_t>(),
                       m->w2.as<uint16_t>(), m->w3.as<uint16_t>());
    INSP_HIP(hipGetLastError());
    INSP_HIP(hipDeviceSynchronize());
    *out = m.release();
    return INSP_OK;
}

extern "C" void insp_mlp_free(insp_mlp *m) { delete m; }

// The model's buffers live on the device that was current at create: work
// for it must be launched there.
static int check_device(const insp_mlp *m) {
    int dev = -1;
    INSP_HIP(hipGetDevice(&dev));
    if (dev != m->device) return set_error(INSP_E_INVAL, "the current device is not the model's device");
    return INSP_OK;
}

extern "C" int insp_mlp_grads(insp_mlp *m, const float *x, const float *t, int32_t batch, float *grads, float *y,
                              float *loss, void *stream) {
    if (!m || !x || !t || batch < 1 || batch % 32) return set_error(INSP_E_INVAL, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = check_device(m))) return rc;
    if ((rc = mlp_reserve(m, batch)) || (rc = mlp_backward(m, x, t, batch, st))) return rc;
    if (grads) INSP_HIP(hipMemcpyAsync(grads, m->g.p, 4 * kParams, hipMemcpyDeviceToDevice, st));
    if (y) INSP_HIP(hipMemcpyAsync(y, m->y.p, 4 * kOut * (size_t)batch, hipMemcpyDeviceToDevice, st));
    if (loss) INSP_HIP(hipMemcpyAsync(loss, m->loss.p, 4, hipMemcpyDeviceToDevice, st));
    return INSP_OK;
}

extern "C" int insp_mlp_train_step(insp_mlp *m, const float *x, const float *t, int32_t batch, float lr, float *loss,
                                   void *stream) {
    if (!m || !x || !t || batch < 1 || batch % 32 || !(lr > 0.f)) return set_error(INSP_E_INVAL, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = check_device(m))) return rc;
    if ((rc = mlp_reserve(m, batch)) || (rc = mlp_backward(m, x, t, batch, st))) return rc;
    m->step++;
    const float bc1 = 1.f - powf(0.9f, (float)m->step), bc2 = 1.f - powf(0.999f, (float)m->step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(kParams, 256)), dim3(256), 0, st, m->p.as<float>(), m->g.as<float>(),
                       m->m.as<float>(), m->v.as<float>(), kParams, lr, bc1, bc2, m->w1.as<uint16_t>(),
                       m->w2.as<uint16_t>(), m->w3.as<uint16_t>(), (const int32_t *)nullptr, 0);
    if (loss) INSP_HIP(hipMemcpyAsync(loss, m->loss.p, 4, hipMemcpyDeviceToDevice, st));
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

// One step of graph-captured training: minibatch tab[0] mod steps, the step
// index advances once the minibatch is staged, Adam with the tabled
// corrections of step tab[0] - 1.
static int train_enqueue(insp_mlp *m, const float *x, const float *t, int32_t steps, int32_t batch, float lr,
                         int32_t tabn, hipStream_t st) {
    int32_t *tab = m->tab.as<int32_t>();
    int rc;
    if ((rc = mlp_backward(m, x, t, batch, st, tab, steps))) return rc;
    hipLaunchKernelGGL(k_adam, dim3(blocks(kParams, 256)), dim3(256), 0, st, m->p.as<float>(), m->g.as<float>(),
                       m->m.as<float>(), m->v.as<float>(), kParams, lr, 1.f, 1.f, m->w1.as<uint16_t>(),
                       m->w2.as<uint16_t>(), m->w3.as<uint16_t>(), (const int32_t *)tab, tabn);
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

// Captures `chunk` consecutive steps into m->exec (on the model's own
// stream: capture leaves the caller's stream alone).
static int train_capture(insp_mlp *m, const float *x, const float *t, int32_t steps, int32_t batch, float lr,
                         int32_t chunk, int32_t tabn) {
    if (m->exec) {
        (void)hipGraphExecDestroy(m->exec);
        m->exec = nullptr;
    }
    if (!m->cs) INSP_HIP(hipStreamCreateWithFlags(&m->cs, hipStreamNonBlocking));
    INSP_HIP(hipStreamBeginCapture(m->cs, hipStreamCaptureModeThreadLocal));
    int rc = INSP_OK;
    for (int32_t s = 0; s < chunk && rc == INSP_OK; s++) rc = train_enqueue(m, x, t, steps, batch, lr, tabn, m->cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(m->cs, &g);
    if (rc == INSP_OK && e != hipSuccess) rc = set_error(INSP_E_DEVICE, hipGetErrorString(e));
    if (rc == INSP_OK) {
        const hipError_t ei = hipGraphInstantiate(&m->exec, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            m->exec = nullptr;
            rc = set_error(INSP_E_DEVICE, hipGetErrorString(ei));
        }
    }
    if (g) (void)hipGraphDestroy(g);
    return rc;
}

extern "C" int insp_mlp_train(insp_mlp *m, const float *x, const float *t, int64_t n, int32_t batch, int32_t epochs,
                              float lr, float *loss, void *stream) {
    if (!m || n < 0 || epochs < 0 || batch < 1 || batch % 32 || !(lr > 0.f) || (n > 0 && (!x || !t)))
        return set_error(INSP_E_INVAL, "bad argument");
    const int64_t steps = n / batch, total = steps * epochs;
    if (total == 0) return INSP_OK;
    if (total > kMaxTrainSteps) return set_error(INSP_E_RANGE, "more than 2^28 training steps in one call");
    hipStream_t st = (hipStream_t)stream;
    const int64_t words = 1 + 2 * total;
    int rc;
    if ((rc = check_device(m))) return rc;
    if (m->cap < batch || m->tab.bytes < (size_t)(4 * words)) {
        INSP_HIP(hipStreamSynchronize(st));  // earlier work on the stream may still read the old buffers
        if ((rc = mlp_reserve(m, batch))) return rc;
        if (m->tab.bytes < (size_t)(4 * words)) {
            DevBuf fresh;
            if ((rc = fresh.alloc(4 * words))) return rc;
            m->tab.swap(fresh);
            m->gen++;
        }
    }
    // step index 0, then the corrections of steps step+1 .. step+total, as
    // the eager step computes them
    std::vector<int32_t> h((size_t)words);
    h[0] = 0;
    for (int64_t s = 1; s <= total; s++) {
        const float bc1 = 1.f - powf(0.9f, (float)(m->step + s)), bc2 = 1.f - powf(0.999f, (float)(m->step + s));
        memcpy(&h[2 * s - 1], &bc1, 4);
        memcpy(&h[2 * s], &bc2, 4);
    }
    INSP_HIP(hipMemcpyAsync(m->tab.p, h.data(), 4 * words, hipMemcpyHostToDevice, st));
    INSP_HIP(hipStreamSynchronize(st));  // h is released on return
    const int32_t chunk = (int32_t)std::min<int64_t>(total, kTrainChunk);
    const int32_t tabn = (int32_t)((m->tab.bytes / 4 - 1) / 2);  // entries the table holds
    const insp_mlp::Key k{x, t, (int32_t)steps, batch, chunk, lr, m->gen};
    if (!m->exec || !(k == m->key)) {
        m->key = insp_mlp::Key{};
        if ((rc = train_capture(m, x, t, (int32_t)steps, batch, lr, chunk, tabn))) return rc;
        m->key = k;
    }
    for (int64_t s = 0; s + chunk <= total; s += chunk) INSP_HIP(hipGraphLaunch(m->exec, st));
    for (int64_t s = total - total % chunk; s < total; s++)
        if ((rc = train_enqueue(m, x, t, (int32_t)steps, batch, lr, tabn, st))) return rc;
    m->step += total;
    if (loss) INSP_HIP(hipMemcpyAsync(loss, m->loss.p, 4, hipMemcpyDeviceToDevice, st));
    return INSP_OK;
}

extern "C" int insp_mlp_predict(insp_mlp *m, const float *x, int64_t n, float *y, int32_t *est, void *stream) {
    if (!m || (n > 0 && (!x || (!y && !est))) || n < 0) return set_error(INSP_E_INVAL, "bad argument");
    if (n == 0) return INSP_OK;
    // the features are read 16 bytes at a time
    if ((uintptr_t)x & 15) return set_error(INSP_E_INVAL, "x must be 16-byte aligned");
    if (int rc = check_device(m)) return rc;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    const int64_t tiles = (n + kRT - 1) / kRT;
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, (int64_t)cus * 2);
    ProfScope ps(st, "mlp_infer");
    hipLaunchKernelGGL(k_infer<kInferWaves>, dim3(grid), dim3(64 * kInferWaves), 0, st, x, n, m->w1.as<uint16_t>(), m->p.as<float>() + kOffB1,
                       m->w2.as<uint16_t>(), m->p.as<float>() + kOffB2, m->w3.as<uint16_t>(),
                       m->p.as<float>() + kOffB3, y, est);
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

extern "C" int insp_mlp_state(insp_mlp *m, float *params, float *adam_m, float *adam_v, int64_t *step, int to_host) {
    if (!m) return set_error(INSP_E_INVAL, "null model");
    INSP_HIP(hipDeviceSynchronize());
    const hipMemcpyKind k = to_host ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice;
    struct { float *h; DevBuf *d; } parts[3] = {{params, &m->p}, {adam_m, &m->m}, {adam_v, &m->v}};
    for (auto &pp : parts)
        if (pp.h) {
            if (to_host) INSP_HIP(hipMemcpy(pp.h, pp.d->p, 4 * kParams, k));
            else INSP_HIP(hipMemcpy(pp.d->p, pp.h, 4 * kParams, k));
        }
    if (step) {
        if (to_host) *step = m->step;
        else m->step = *step;
    }
    if (!to_host && params) {
        hipLaunchKernelGGL(k_shadow, dim3(blocks(kParams, 256)), dim3(256), 0, 0, m->p.as<float>(),
                           m->w1.as<uint16_t>(), m->w2.as<uint16_t>(), m->w3.as<uint16_t>());
        INSP_HIP(hipGetLastError());
        INSP_HIP(hipDeviceSynchronize());
    }
    return INSP_OK;
}
