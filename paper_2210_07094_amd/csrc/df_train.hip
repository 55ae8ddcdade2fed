// Training the DNN chemistry integrator on the device: the MLP's backward pass and Adam.
//
// The network of the DNN form (Sec. "Chemistry Integration": z-scored (T, p, Box-Cox(Y)) in,
// hidden GELU layers, z-scored Box-Cox increments out) is fitted to pairs the integrator
// produces: df_dnn_make_batch turns states before and after an integrator step into
// (input, target) rows; df_dnn_train_step takes one Adam step on the mean squared error
//   L = 1/(B O) sum_b sum_o (u_bo - t_bo)^2 .
// Forward in bf16 on the matrix cores with fp32 accumulation, as inference, keeping each hidden
// layer's pre-activation a_l; backward:
//   du = 2 (u - t) / (B O);   dh_last = du W_out;   da_l = dh_l * GELU'(a_l)
//   dh_{l-1} = da_l W_l  (bf16 GEMM with the transposed weights, GELU' in the epilogue)
//   dW_l = da_l^T in_l,  db_l = sum_b da_l      (fp32, reductions over the batch; dW on MFMA)
// Adam (Kingma and Ba, ICLR 2015) on fp32 master weights; each update rewrites the handle's
// bf16 weights (so df_dnn_step runs the trained network) and the transposed bf16 copies.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "df_internal.h"

namespace df {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16_t tbf(float x) {
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16_t((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16_t(u >> 16);
}
__device__ __forceinline__ float fbf(bf16_t h) { return __uint_as_float(unsigned(h) << 16); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

constexpr int kT = 256;

// batch rows: x fp32 [B][n_in] -> bf16 [Bp][in_pad], zero beyond n_in and beyond B
__global__ __launch_bounds__(kT) void load_x_kernel(const float *__restrict__ x, int64_t B, int64_t Bp, int n_in,
                                                    int in_pad, bf16_t *__restrict__ xb) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (e >= Bp * in_pad) return;
    const int64_t b = e / in_pad;
    const int c = int(e % in_pad);
    xb[e] = (b < B && c < n_in) ? tbf(x[b * n_in + c]) : bf16_t(0);
}

// output layer and loss, one wavefront per batch row (the 64 lanes split the hidden units,
// lane i taking units i, i + 64, ...): u = W h + b (bf16 operands, fp32 partial sums per lane,
// combined by a fixed butterfly, so every lane holds u), du = 2 (u - t)/(B O), the row loss, and
// da of the last hidden layer, each lane writing its own units
template <int O>
__global__ __launch_bounds__(kT) void out_loss_kernel(const bf16_t *__restrict__ h, const bf16_t *__restrict__ a,
                                                      int hid, const bf16_t *__restrict__ W,
                                                      const float *__restrict__ bias, const float *__restrict__ t,
                                                      int64_t B, int64_t Bp, float *__restrict__ du,
                                                      float *__restrict__ row_loss, bf16_t *__restrict__ da) {
    static_assert(O <= 64, "one lane per output writes du");
    const int lane = int(threadIdx.x) & 63;
    const int64_t b = int64_t(blockIdx.x) * (kT / 64) + (threadIdx.x >> 6);
    if (b >= Bp) return;
    bf16_t *dar = da + b * hid;
    if (b >= B) {
        for (int i = lane; i < hid; i += 64) dar[i] = 0;
        if (lane < O) du[b * O + lane] = 0.0f;
        if (lane == 0) row_loss[b] = 0.0f;
        return;
    }
    const bf16_t *hr = h + b * hid;
    float u[O];
#pragma unroll
    for (int o = 0; o < O; ++o) u[o] = 0.0f;
    for (int i = lane; i < hid; i += 64) {
        const float hv = fbf(hr[i]);
#pragma unroll
        for (int o = 0; o < O; ++o) u[o] = fmaf(fbf(W[o * hid + i]), hv, u[o]);
    }
#pragma unroll
    for (int o = 0; o < O; ++o)
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) u[o] += __shfl_xor(u[o], m);
    const float sc = 2.0f / float(B * O);
    float g[O], l = 0.0f;
#pragma unroll
    for (int o = 0; o < O; ++o) {
        const float e = u[o] + bias[o] - t[b * O + o];
        l = fmaf(e, e, l);
        g[o] = sc * e;
        if (lane == o) du[b * O + o] = g[o];
    }
    if (lane == 0) row_loss[b] = l;
    const bf16_t *ar = a + b * hid;
    for (int i = lane; i < hid; i += 64) {
        float s = 0.0f;
#pragma unroll
        for (int o = 0; o < O; ++o) s = fmaf(g[o], fbf(W[o * hid + i]), s);
        dar[i] = tbf(s * gelu_d(fbf(ar[i])));
    }
}

// loss = sum of row losses / (B O), fixed-order tree in one block
__global__ __launch_bounds__(kT) void loss_sum_kernel(const float *__restrict__ row_loss, int64_t B, int O,
                                                      float *__restrict__ loss) {
    __shared__ double part[kT];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < B; b += kT) s += double(row_loss[b]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = float(part[0] / double(B * O));
}

// dW[M][N] (fp32) = sum_b A[b][M] X[b][N] over the batch rows (bf16 operands, MFMA 16x16x32 with
// fp32 accumulation): one wave per 32 x 32 tile of dW and slice of the batch (S slices of whole
// 32-row steps; block (tile, s) takes steps s, s + S, ...), four MFMA tiles, 32 batch rows per
// step.  The batch is the reduction dimension, so each step's 32 x 32 slices of A and X are read
// as 16-byte row pieces and written to LDS transposed ([m][b]); a lane then reads operand row
// (lane % 16) with the 8 batch rows 8 (lane / 16) .. + 7 as one 16-byte fragment.  The blocks of
// the first column of tiles also sum A over their batch rows (the bias gradient db).  With S = 1
// the sums go to dW and db, else to the slice's partial arrays P[s][M][N] and Pb[s][M], which
// wgrad_reduce_kernel adds in slice order: the result does not depend on the launch.
constexpr int kWgT = 32 + 8;  // LDS row stride of the transposed slices (bf16)

// orders the LDS writes and reads of the lanes of one wavefront (the workgroup is one wave, so a
// workgroup barrier would not order them)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__global__ __launch_bounds__(64) void wgrad_kernel(const bf16_t *__restrict__ A, int lda, const bf16_t *__restrict__ X,
                                                   int ldx, int64_t Bp, int S, float *__restrict__ dW, int ldw,
                                                   int tiles_n, float *__restrict__ db) {
    __shared__ __attribute__((aligned(16))) bf16_t At[32 * kWgT], Xt[32 * kWgT];
    const int lane = threadIdx.x;
    const int tile = int(blockIdx.x) / S, sl = int(blockIdx.x) % S;
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int m0 = tm * 32, n0 = tn * 32;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    float cs[2] = {0.0f, 0.0f};
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // this lane's two 16-byte pieces of each slice: batch row c / 4, columns 8 (c % 4) .. + 7
    const int c0 = lane, c1 = lane + 64;
    for (int64_t b0 = int64_t(sl) * 32; b0 < Bp; b0 += int64_t(S) * 32) {
        const u32x4 a0 = *reinterpret_cast<const u32x4 *>(A + (b0 + c0 / 4) * lda + m0 + 8 * (c0 % 4));
        const u32x4 a1 = *reinterpret_cast<const u32x4 *>(A + (b0 + c1 / 4) * lda + m0 + 8 * (c1 % 4));
        const u32x4 x0 = *reinterpret_cast<const u32x4 *>(X + (b0 + c0 / 4) * ldx + n0 + 8 * (c0 % 4));
        const u32x4 x1 = *reinterpret_cast<const u32x4 *>(X + (b0 + c1 / 4) * ldx + n0 + 8 * (c1 % 4));
        wave_lds_sync();  // the previous step's fragment reads are done
        // value q of a 16-byte piece is the low (q even) or high (q odd) half of word q / 2
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int sh = 16 * (q & 1);
            At[(8 * (c0 % 4) + q) * kWgT + c0 / 4] = bf16_t(a0[q / 2] >> sh);
            At[(8 * (c1 % 4) + q) * kWgT + c1 / 4] = bf16_t(a1[q / 2] >> sh);
            Xt[(8 * (c0 % 4) + q) * kWgT + c0 / 4] = bf16_t(x0[q / 2] >> sh);
            Xt[(8 * (c1 % 4) + q) * kWgT + c1 / 4] = bf16_t(x1[q / 2] >> sh);
        }
        wave_lds_sync();
        bf16x8 af[2], xf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            af[i] = *reinterpret_cast<const bf16x8 *>(At + (i * 16 + fr) * kWgT + fk);
            xf[i] = *reinterpret_cast<const bf16x8 *>(Xt + (i * 16 + fr) * kWgT + fk);
#pragma unroll
            for (int q = 0; q < 8; ++q) cs[i] += float(af[i][q]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], xf[j], acc[i][j], 0, 0, 0);
    }
    float *out = (S == 1) ? dW : dW + size_t(sl) * size_t(gridDim.x / S / tiles_n * 32) * ldw;
    // lane holds column (lane % 16) and rows 4 (lane / 16) + r of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[int64_t(m0 + i * 16 + (lane >> 4) * 4 + r) * ldw + n0 + j * 16 + fr] = acc[i][j][r];
    if (tn == 0) {
        // lanes l, l + 16, l + 32, l + 48 hold the four batch quarters of row m0 + i 16 + l
        float *outb = (S == 1) ? db : db + size_t(sl) * size_t(gridDim.x / S / tiles_n * 32);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float v = cs[i];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 16) outb[m0 + i * 16 + lane] = v;
        }
    }
}

// Weight gradient of a layer whose padded widths are multiples of 160, dW[m][n] = sum over the
// batch slice of A[b][m] X[b][n] (A: the gradient at the layer's output [Bp][lda], X: its input
// [Bp][ldx]), and with tn == 0 the bias gradient sum_b A[b][m]: one 160 x 160 tile and one batch
// slice per block of five waves.  Per 64-row step of the slice, each of the 320 threads loads one
// 8 x 8 piece (eight batch rows of 16 bytes) of A (threads 0..159) or X (160..319), transposes it
// in registers and writes it as eight 16-byte rows of the transposed tile in LDS, so that the
// MFMA fragments (eight consecutive batch rows of one m or n) are single 16-byte reads.  Wave w
// owns rows 32 w .. 32 w + 31 of the tile and its 160 columns (2 x 10 MFMA tiles).  The slice's
// steps are 64-row steps sl, sl + S, ...; the partial sums of slice sl go to dW + sl rows_total ldw
// (and db + sl rows_total) when S > 1.
constexpr int kWbT = 160, kWbK = 64, kWbLd = kWbK + 8;  // tile side, batch rows per step, LDS row stride
constexpr int kWbThreads = 320;
__global__ __launch_bounds__(kWbThreads) void wgrad_big_kernel(const bf16_t *__restrict__ A, int lda,
                                                               const bf16_t *__restrict__ X, int ldx, int64_t Bp,
                                                               int S, float *__restrict__ dW, int ldw, int tiles_n,
                                                               int rows_total, float *__restrict__ db) {
    __shared__ __attribute__((aligned(16))) bf16_t At[kWbT * kWbLd], Xt[kWbT * kWbLd];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int tile = int(blockIdx.x) / S, sl = int(blockIdx.x) % S;
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int m0 = tm * kWbT, n0 = tn * kWbT;
    // this thread's piece: batch group bg (rows 8 bg .. 8 bg + 7 of the step), column group cg
    const bool isA = t < kWbT;
    const int u = isA ? t : t - kWbT;
    const int bg = u & 7, cg = u >> 3;
    const bf16_t *src = isA ? A + (m0 + 8 * cg) : X + (n0 + 8 * cg);
    const int64_t ld = isA ? lda : ldx;
    bf16_t *dst = (isA ? At : Xt) + (8 * cg) * kWbLd + 8 * bg;
    u32x4 r[8];
    auto load = [&](int64_t b0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = *reinterpret_cast<const u32x4 *>(src + (b0 + 8 * bg + j) * ld);
    };
    auto store = [&]() {
        // column c of the piece holds the values of batch rows 0..7, two to a word (row 2p low)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            u32x4 v;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const unsigned lo = r[2 * p][c >> 1], hi = r[2 * p + 1][c >> 1];
                v[p] = (c & 1) ? ((lo >> 16) | (hi & 0xffff0000u)) : ((lo & 0xffffu) | (hi << 16));
            }
            *reinterpret_cast<u32x4 *>(dst + c * kWbLd) = v;
        }
    };
    floatx4 acc[2][10];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 10; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    float cs[2] = {0.0f, 0.0f};
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    const int64_t step = int64_t(S) * kWbK;
    int64_t b0 = int64_t(sl) * kWbK;
    if (b0 < Bp) load(b0);
    for (; b0 < Bp; b0 += step) {
        __syncthreads();  // the previous step's fragment reads are done
        store();
        __syncthreads();
        if (b0 + step < Bp) load(b0 + step);
#pragma unroll
        for (int kk = 0; kk < kWbK; kk += 32) {
            bf16x8 af[2], xf[10];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                af[i] = *reinterpret_cast<const bf16x8 *>(At + (w * 32 + i * 16 + fr) * kWbLd + kk + fk);
                if (tn == 0) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) cs[i] += float(af[i][q]);
                }
            }
#pragma unroll
            for (int j = 0; j < 10; ++j) xf[j] = *reinterpret_cast<const bf16x8 *>(Xt + (j * 16 + fr) * kWbLd + kk + fk);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 10; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], xf[j], acc[i][j], 0, 0, 0);
        }
    }
    float *out = (S == 1) ? dW : dW + size_t(sl) * size_t(rows_total) * size_t(ldw);
    // lane holds column (lane % 16) and rows 4 (lane / 16) + r of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 10; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                out[int64_t(m0 + w * 32 + i * 16 + (lane >> 4) * 4 + q) * ldw + n0 + j * 16 + fr] = acc[i][j][q];
    if (tn == 0) {
        // lanes l, l + 16, l + 32, l + 48 hold the four batch quarters of row w 32 + i 16 + l
        float *outb = (S == 1) ? db : db + size_t(sl) * size_t(rows_total);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float v = cs[i];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 16) outb[m0 + w * 32 + i * 16 + lane] = v;
        }
    }
}

// dW = sum over the S slices of P[s] (in slice order), db likewise from Pb
__global__ __launch_bounds__(kT) void wgrad_reduce_kernel(const float *__restrict__ P, const float *__restrict__ Pb,
                                                          int S, int64_t nw, int nb, float *__restrict__ dW,
                                                          float *__restrict__ db) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (e < nw) {
        float v = 0.0f;
        for (int k = 0; k < S; ++k) v += P[size_t(k) * nw + e];
        dW[e] = v;
    } else if (e < nw + nb) {
        const int64_t c = e - nw;
        float v = 0.0f;
        for (int k = 0; k < S; ++k) v += Pb[size_t(k) * nb + c];
        db[c] = v;
    }
}

// batch slices of the weight gradient of a layer with `tiles` 32 x 32 tiles: enough blocks to
// fill the chip (about 2048 waves), at most 32 and at most one per 32-row step
int wgrad_slices(int64_t tiles, int64_t Bp) {
    int64_t S = (2048 + tiles - 1) / tiles;
    S = std::min<int64_t>(S, 32);
    S = std::min<int64_t>(S, std::max<int64_t>(1, Bp / 32));
    return int(std::max<int64_t>(S, 1));
}

// How a hidden layer's weight gradient is computed: 160 x 160 tiles (wgrad_big_kernel) where both
// padded widths are multiples of 160 and the padded batch of 64, else 32 x 32 tiles; S batch
// slices, enough for about 400 blocks (2000 waves) of the large tiles.
struct WgradPlan {
    bool big;
    int S;
    int64_t tiles;
    int tiles_n;
};
WgradPlan wgrad_plan(const DnnLayer &Ly, int64_t Bp) {
    WgradPlan p{};
    p.big = Ly.n_pad % kWbT == 0 && Ly.k_pad % kWbT == 0 && Bp % kWbK == 0;
    if (p.big) {
        p.tiles_n = Ly.k_pad / kWbT;
        p.tiles = int64_t(Ly.n_pad / kWbT) * p.tiles_n;
        int64_t S = (400 + p.tiles - 1) / p.tiles;
        S = std::min<int64_t>(S, 32);
        S = std::min<int64_t>(S, std::max<int64_t>(1, Bp / kWbK));
        p.S = int(std::max<int64_t>(S, 1));
    } else {
        p.tiles_n = Ly.k_pad / 32;
        p.tiles = int64_t(Ly.n_pad / 32) * p.tiles_n;
        p.S = wgrad_slices(p.tiles, Bp);
    }
    return p;
}

// output layer gradients: dW[o][i] = sum_b du[b][o] h[b][i], db[o] = sum_b du[b][o]; one
// block per input column i (column hid: the bias), the batch spread over the threads and the
// partial sums added in a fixed-order tree
template <int O>
__global__ __launch_bounds__(kT) void wgrad_out_kernel(const float *__restrict__ du, const bf16_t *__restrict__ h,
                                                       int hid, int64_t B, float *__restrict__ dW,
                                                       float *__restrict__ db) {
    __shared__ float part[O][kT];
    const int i = blockIdx.x, t = threadIdx.x;
    float s[O];
#pragma unroll
    for (int o = 0; o < O; ++o) s[o] = 0.0f;
    for (int64_t b = t; b < B; b += kT) {
        const float hv = (i < hid) ? fbf(h[b * hid + i]) : 1.0f;
#pragma unroll
        for (int o = 0; o < O; ++o) s[o] = fmaf(du[b * O + o], hv, s[o]);
    }
#pragma unroll
    for (int o = 0; o < O; ++o) part[o][t] = s[o];
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int o = 0; o < O; ++o) part[o][t] += part[o][t + w];
        __syncthreads();
    }
    if (t < O) {
        if (i < hid)
            dW[t * hid + i] = part[t][0];
        else
            db[t] = part[t][0];
    }
}

// Adam over every parameter block of the network in one launch.  Segment q is one parameter
// block [rows][cols] (padded storage, real part rows_r x cols_r; padding stays zero), taken by the
// thread blocks first[q] .. first[q + 1] - 1; it writes the fp32 master, the bf16 copy (if Wb), the
// transposed bf16 copy (if WT) and an fp32 copy (if wf).
constexpr int kAdamSegs = 32;
struct AdamSeg {
    float *w, *m, *v;
    const float *g;
    bf16_t *Wb, *WT;
    float *wf;
    int rows, cols, rows_r, cols_r;
};
struct AdamSegs {
    AdamSeg seg[kAdamSegs];
    int64_t first[kAdamSegs + 1];
    int n;
};
__global__ __launch_bounds__(kT) void adam_all_kernel(AdamSegs sg, float lr, float b1, float b2, float eps, float bc1,
                                                      float bc2) {
    const int64_t blk = blockIdx.x;
    int q = 0;
    while (q + 1 < sg.n && blk >= sg.first[q + 1]) ++q;  // block-uniform
    const AdamSeg &a = sg.seg[q];
    const int64_t e = (blk - sg.first[q]) * kT + threadIdx.x;
    if (e >= int64_t(a.rows) * a.cols) return;
    const int r = int(e / a.cols), c = int(e % a.cols);
    if (r >= a.rows_r || c >= a.cols_r) return;
    const float gi = a.g[e];
    const float mi = b1 * a.m[e] + (1.0f - b1) * gi;
    const float vi = b2 * a.v[e] + (1.0f - b2) * gi * gi;
    a.m[e] = mi;
    a.v[e] = vi;
    const float wi = a.w[e] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    a.w[e] = wi;
    if (a.Wb) a.Wb[e] = tbf(wi);
    if (a.WT) a.WT[int64_t(c) * a.rows + r] = tbf(wi);
    if (a.wf) a.wf[e] = wi;
}

// trainer set-up: fp32 master from the handle's bf16 weights, transposed bf16 copies
__global__ __launch_bounds__(kT) void init_master_kernel(const bf16_t *__restrict__ Wb, int rows, int cols,
                                                         float *__restrict__ w, bf16_t *__restrict__ WT) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (e >= int64_t(rows) * cols) return;
    w[e] = fbf(Wb[e]);
    if (WT) WT[int64_t(e % cols) * rows + e / cols] = Wb[e];
}

// the bf16 copies of a layer from its fp32 master: the handle's weights and the transposed copy
__global__ __launch_bounds__(kT) void refresh_bf16_kernel(const float *__restrict__ w, int rows, int cols,
                                                          bf16_t *__restrict__ Wb, bf16_t *__restrict__ WT) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (e >= int64_t(rows) * cols) return;
    const bf16_t v = tbf(w[e]);
    Wb[e] = v;
    if (WT) WT[int64_t(e % cols) * rows + e / cols] = v;
}

// (input, target) rows from states before (T, p, Y0) and after (Y1) an integrator step of the
// network's dt: x = z-score of (T, p, Box-Cox(Y0)), t = z-score of Box-Cox(Y1) - Box-Cox(Y0);
// valid = 1 inside the training box (the rows of invalid cells are still written)
template <int K>
__global__ __launch_bounds__(kT) void make_batch_kernel(DnnDevParams prm, int64_t n, int64_t ld,
                                                        const double *__restrict__ p, const double *__restrict__ T,
                                                        const double *__restrict__ Y0, const double *__restrict__ Y1,
                                                        float *__restrict__ x, float *__restrict__ t,
                                                        int32_t *__restrict__ valid) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    constexpr int NI = K + 2;
    double f[NI];
    f[0] = T[i];
    f[1] = p[i];
    bool ok = isfinite(f[0]) && f[0] > 0.0 && isfinite(f[1]) && f[1] > 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double y0 = Y0[k * ld + i], y1 = Y1[k * ld + i];
        ok = ok && isfinite(y0) && isfinite(y1);
        const double z0 = (pow(fmax(y0, 0.0), prm.lambda) - 1.0) / prm.lambda;
        const double z1 = (pow(fmax(y1, 0.0), prm.lambda) - 1.0) / prm.lambda;
        f[2 + k] = z0;
        t[i * K + k] = float(((z1 - z0) - prm.mu_out[k]) / prm.sig_out[k]);
    }
#pragma unroll
    for (int c = 0; c < NI; ++c) {
        ok = ok && f[c] >= prm.lo[c] && f[c] <= prm.hi[c];
        x[i * NI + c] = float((f[c] - prm.mu_in[c]) / prm.sig_in[c]);
    }
    if (valid) valid[i] = ok ? 1 : 0;
}

int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

}  // namespace
}  // namespace df

struct df_trainer {
    df_dnn *dnn;
    int64_t max_batch, bp;
    int nh;  // hidden layers
    void *blob;
    std::vector<float *> W, b, mW, vW, mb, vb, gW, gb;  // per layer (hidden then output), padded
    std::vector<df::bf16_t *> WT;                        // per hidden layer: [k_pad][n_pad], or null
    df::bf16_t *x;
    std::vector<df::bf16_t *> h, a, da;  // per hidden layer [bp][n_pad]
    float *du, *row_loss, *loss;
    float *part, *part_b;  // weight-gradient partial sums over batch slices
    int64_t step;
};

using namespace df;

extern "C" {

df_status df_dnn_trainer_create(df_dnn *d, int64_t max_batch, df_trainer **out) {
    clear_error();
    if (!d || !out || max_batch < 1) return fail(DF_E_INVALID, "df_dnn_trainer_create: bad arguments");
    *out = nullptr;
    const int L = int(d->layers.size()), nh = L - 1;
    if (d->K != 9 || d->layers.back().n_out != 9)
        return fail(DF_E_UNSUPPORTED, "df_dnn_trainer_create: the output layer kernels are compiled for 9 outputs");
    // the weight-gradient kernel tiles every hidden layer's padded weights in 32 x 32 blocks, and
    // the output layer reads its input width from the last hidden layer's padding
    for (int l = 0; l < L - 1; ++l)
        if (d->layers[l].n_pad % 32 || d->layers[l].k_pad % 32)
            return fail(DF_E_UNSUPPORTED, "df_dnn_trainer_create: hidden widths must pad to multiples of 32");
    if (L < 2 || d->layers.back().k_pad != d->layers[L - 2].n_pad)
        return fail(DF_E_UNSUPPORTED, "df_dnn_trainer_create: unexpected layer padding");
    auto *t = new df_trainer;
    t->dnn = d;
    t->max_batch = max_batch;
    t->bp = rup(max_batch, kGemmBM);
    t->nh = nh;
    t->step = 0;
    // one allocation: per layer 6 fp32 blocks of W's size (W, mW, vW, gW) and b's (b, mb, vb, gb),
    // transposed bf16 copies, activations
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t o = 0;
    std::vector<size_t> oW(L), ob(L), oT(L, 0), oh(nh), oa(nh), oda(nh);
    for (int l = 0; l < L; ++l) {
        const size_t nw = size_t(d->layers[l].n_pad) * d->layers[l].k_pad, nb = size_t(d->layers[l].n_pad);
        oW[l] = o;
        o = al(o + 4 * nw * 4);
        ob[l] = o;
        o = al(o + 4 * nb * 4);
        if (l >= 1 && l < nh) {
            oT[l] = o;
            o = al(o + nw * 2);
        }
    }
    const size_t ox = o;
    o = al(o + size_t(t->bp) * d->layers[0].k_pad * 2);
    for (int l = 0; l < nh; ++l) {
        const size_t na = size_t(t->bp) * d->layers[l].n_pad * 2;
        oh[l] = o;
        o = al(o + na);
        oa[l] = o;
        o = al(o + na);
        oda[l] = o;
        o = al(o + na);
    }
    const int O = d->layers.back().n_out;
    const size_t odu = o;
    o = al(o + size_t(t->bp) * O * 4);
    const size_t orl = o;
    o = al(o + size_t(t->bp) * 4);
    const size_t ol = o;
    o = al(o + 4);
    // partial weight gradients of the hidden layers, for the largest slice count of any of them
    size_t part = 0, part_b = 0;
    for (int l = 0; l < nh; ++l) {
        const DnnLayer &Ly = d->layers[l];
        const int S = wgrad_plan(Ly, t->bp).S;
        if (S > 1) {
            part = std::max(part, size_t(S) * Ly.n_pad * Ly.k_pad);
            part_b = std::max(part_b, size_t(S) * Ly.n_pad);
        }
    }
    const size_t opart = o;
    o = al(o + part * 4);
    const size_t opb = o;
    o = al(o + part_b * 4);
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(d->device) != hipSuccess) {
        delete t;
        return fail(DF_E_HIP, "df_dnn_trainer_create: cannot select the network's device");
    }
    hipError_t e = hipMalloc(&t->blob, o);
    if (e == hipSuccess) e = hipMemset(t->blob, 0, o);
    if (e != hipSuccess) {
        if (t->blob) (void)hipFree(t->blob);
        (void)hipSetDevice(prev);
        delete t;
        return fail(DF_E_HIP, std::string("df_dnn_trainer_create: ") + hipGetErrorString(e));
    }
    auto *base = static_cast<unsigned char *>(t->blob);
    for (int l = 0; l < L; ++l) {
        const size_t nw = size_t(d->layers[l].n_pad) * d->layers[l].k_pad, nb = size_t(d->layers[l].n_pad);
        auto *w = reinterpret_cast<float *>(base + oW[l]);
        t->W.push_back(w);
        t->mW.push_back(w + nw);
        t->vW.push_back(w + 2 * nw);
        t->gW.push_back(w + 3 * nw);
        auto *bb = reinterpret_cast<float *>(base + ob[l]);
        t->b.push_back(bb);
        t->mb.push_back(bb + nb);
        t->vb.push_back(bb + 2 * nb);
        t->gb.push_back(bb + 3 * nb);
        t->WT.push_back((l >= 1 && l < nh) ? reinterpret_cast<bf16_t *>(base + oT[l]) : nullptr);
        hipLaunchKernelGGL(init_master_kernel, dim3(unsigned((nw + kT - 1) / kT)), dim3(kT), 0, 0, d->layers[l].W,
                           d->layers[l].n_pad, d->layers[l].k_pad, w, t->WT.back());
        (void)hipMemcpy(bb, d->layers[l].b, nb * 4, hipMemcpyDeviceToDevice);
    }
    t->x = reinterpret_cast<bf16_t *>(base + ox);
    for (int l = 0; l < nh; ++l) {
        t->h.push_back(reinterpret_cast<bf16_t *>(base + oh[l]));
        t->a.push_back(reinterpret_cast<bf16_t *>(base + oa[l]));
        t->da.push_back(reinterpret_cast<bf16_t *>(base + oda[l]));
    }
    t->du = reinterpret_cast<float *>(base + odu);
    t->row_loss = reinterpret_cast<float *>(base + orl);
    t->loss = reinterpret_cast<float *>(base + ol);
    t->part = reinterpret_cast<float *>(base + opart);
    t->part_b = reinterpret_cast<float *>(base + opb);
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipFree(t->blob);
        delete t;
        return fail(DF_E_HIP, std::string("df_dnn_trainer_create: ") + hipGetErrorString(e));
    }
    *out = t;
    return DF_OK;
}

void df_dnn_trainer_free(df_trainer *t) {
    if (!t) return;
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(t->dnn->device) == hipSuccess) {
        (void)hipFree(t->blob);
        (void)hipSetDevice(prev);
    }
    delete t;
}

void df_adam_default_opts(df_adam_opts *o) {
    if (!o) return;
    o->lr = 1e-4f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->eps = 1e-8f;
}

df_status df_dnn_train_step(df_trainer *t, int64_t batch, const float *x, const float *target,
                            const df_adam_opts *adam, int32_t update, float *loss, void *hip_stream) {
    clear_error();
    const char *who = "df_dnn_train_step";
    if (!t) return fail(DF_E_INVALID, std::string(who) + ": null trainer");
    if (batch < 1 || batch > t->max_batch) return fail(DF_E_INVALID, std::string(who) + ": need 1 <= batch <= max_batch");
    if (!x || !target) return fail(DF_E_INVALID, std::string(who) + ": null x or target");
    df_adam_opts ao;
    df_adam_default_opts(&ao);
    if (adam) ao = *adam;
    if (!(ao.lr >= 0.0f) || !(ao.beta1 >= 0.0f && ao.beta1 < 1.0f) || !(ao.beta2 >= 0.0f && ao.beta2 < 1.0f) ||
        !(ao.eps > 0.0f))
        return fail(DF_E_INVALID, std::string(who) + ": bad Adam options");
    df_dnn *d = t->dnn;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": hipGetDevice failed");
    if (prev != d->device && hipSetDevice(d->device) != hipSuccess)
        return fail(DF_E_HIP, std::string(who) + ": cannot select the network's device");
    auto s = static_cast<hipStream_t>(hip_stream);
    const int nh = t->nh;
    const int64_t B = batch, Bp = rup(batch, kGemmBM);
    const DnnLayer &L0 = d->layers[0];
    const DnnLayer &Lo = d->layers.back();
    constexpr int O = 9;
    df_status st = DF_OK;
    auto chk = [&](const char *what) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess && st == DF_OK) st = fail(DF_E_HIP, std::string(who) + ": " + what + ": " + hipGetErrorString(e));
    };
    hipLaunchKernelGGL(load_x_kernel, dim3(unsigned((Bp * L0.k_pad + kT - 1) / kT)), dim3(kT), 0, s, x, B, Bp,
                       L0.n_in, L0.k_pad, t->x);
    chk("input");
    // forward, keeping the pre-activations
    const bf16_t *in = t->x;
    int in_ld = L0.k_pad;
    for (int l = 0; l < nh && st == DF_OK; ++l) {
        const DnnLayer &Ly = d->layers[l];
        st = launch_gemm_bf16_epi(in, in_ld, Ly.W, Ly.k_pad, Ly.b, t->h[l], Ly.n_pad, Bp, Ly.n_pad, Ly.k_pad,
                                  GemmEpi::gelu_save, t->a[l], s);
        in = t->h[l];
        in_ld = Ly.n_pad;
    }
    const int hid = Lo.k_pad;
    if (st == DF_OK) {
        hipLaunchKernelGGL(out_loss_kernel<O>, dim3(unsigned((Bp + kT / 64 - 1) / (kT / 64))), dim3(kT), 0, s, t->h[nh - 1],
                           t->a[nh - 1], hid, Lo.W, Lo.b, target, B, Bp, t->du, t->row_loss, t->da[nh - 1]);
        chk("output layer");
        hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(kT), 0, s, t->row_loss, B, O, t->loss);
        chk("loss");
        hipLaunchKernelGGL(wgrad_out_kernel<O>, dim3(unsigned(hid + 1)), dim3(kT), 0, s, t->du, t->h[nh - 1], hid, B,
                           t->gW[nh], t->gb[nh]);
        chk("output layer gradient");
    }
    // backward through the hidden layers
    for (int l = nh - 1; l >= 0 && st == DF_OK; --l) {
        const DnnLayer &Ly = d->layers[l];
        const bf16_t *inl = (l == 0) ? t->x : t->h[l - 1];
        const int inl_ld = Ly.k_pad;
        const WgradPlan wp = wgrad_plan(Ly, Bp);
        const int S = wp.S;
        if (wp.big)
            hipLaunchKernelGGL(wgrad_big_kernel, dim3(unsigned(wp.tiles * S)), dim3(kWbThreads), 0, s, t->da[l],
                               Ly.n_pad, inl, inl_ld, Bp, S, S > 1 ? t->part : t->gW[l], Ly.k_pad, wp.tiles_n,
                               Ly.n_pad, S > 1 ? t->part_b : t->gb[l]);
        else
            hipLaunchKernelGGL(wgrad_kernel, dim3(unsigned(wp.tiles * S)), dim3(64), 0, s, t->da[l], Ly.n_pad, inl,
                               inl_ld, Bp, S, S > 1 ? t->part : t->gW[l], Ly.k_pad, wp.tiles_n,
                               S > 1 ? t->part_b : t->gb[l]);
        chk("weight gradient");
        if (S > 1) {
            const int64_t nw = int64_t(Ly.n_pad) * Ly.k_pad;
            hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(unsigned((nw + Ly.n_pad + kT - 1) / kT)), dim3(kT), 0, s,
                               t->part, t->part_b, S, nw, Ly.n_pad, t->gW[l], t->gb[l]);
            chk("weight gradient sum");
        }
        if (l > 0 && st == DF_OK)
            st = launch_gemm_bf16_epi(t->da[l], Ly.n_pad, t->WT[l], Ly.n_pad, nullptr, t->da[l - 1], Ly.k_pad, Bp,
                                      Ly.k_pad, Ly.n_pad, GemmEpi::gelu_grad, t->a[l - 1], s);
    }
    if (st == DF_OK && loss) {
        if (hipMemcpyAsync(loss, t->loss, 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
            st = fail(DF_E_HIP, std::string(who) + ": copying the loss failed");
    }
    if (st == DF_OK && update) {
        ++t->step;
        const float bc1 = float(1.0 - std::pow(double(ao.beta1), double(t->step)));
        const float bc2 = float(1.0 - std::pow(double(ao.beta2), double(t->step)));
        // every layer's weights and biases in one launch
        AdamSegs sg{};
        int64_t blocks = 0;
        for (int l = 0; l <= nh && sg.n + 2 <= kAdamSegs; ++l) {
            DnnLayer &Ly = d->layers[l];
            sg.seg[sg.n] = AdamSeg{t->W[l], t->mW[l], t->vW[l], t->gW[l], Ly.W, t->WT[l], nullptr,
                                   Ly.n_pad, Ly.k_pad, Ly.n_out, Ly.n_in};
            sg.first[sg.n++] = blocks;
            blocks += (int64_t(Ly.n_pad) * Ly.k_pad + kT - 1) / kT;
            sg.seg[sg.n] = AdamSeg{t->b[l], t->mb[l], t->vb[l], t->gb[l], nullptr, nullptr, Ly.b,
                                   Ly.n_pad, 1, Ly.n_out, 1};
            sg.first[sg.n++] = blocks;
            blocks += (int64_t(Ly.n_pad) + kT - 1) / kT;
        }
        sg.first[sg.n] = blocks;
        if (sg.n != 2 * (nh + 1)) {
            st = fail(DF_E_UNSUPPORTED, std::string(who) + ": too many layers for one Adam launch");
        } else {
            hipLaunchKernelGGL(adam_all_kernel, dim3(unsigned(blocks)), dim3(kT), 0, s, sg, ao.lr, ao.beta1,
                               ao.beta2, ao.eps, bc1, bc2);
            chk("Adam");
        }
    }
    if (prev != d->device) (void)hipSetDevice(prev);
    return st;
}

df_status df_dnn_trainer_get(const df_trainer *t, int32_t layer, int32_t what, float *dst, void *hip_stream) {
    clear_error();
    if (!t || !dst || layer < 0 || layer > t->nh || what < 0 || what > 3)
        return fail(DF_E_INVALID, "df_dnn_trainer_get: bad arguments");
    const DnnLayer &Ly = t->dnn->layers[layer];
    const float *src = (what == 0) ? t->W[layer] : (what == 1) ? t->b[layer] : (what == 2) ? t->gW[layer] : t->gb[layer];
    const bool mat = (what == 0 || what == 2);
    const hipError_t e =
        mat ? hipMemcpy2DAsync(dst, size_t(Ly.n_in) * 4, src, size_t(Ly.k_pad) * 4, size_t(Ly.n_in) * 4, Ly.n_out,
                               hipMemcpyDeviceToDevice, static_cast<hipStream_t>(hip_stream))
            : hipMemcpyAsync(dst, src, size_t(Ly.n_out) * 4, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("df_dnn_trainer_get: ") + hipGetErrorString(e));
    return DF_OK;
}

df_status df_dnn_trainer_set(df_trainer *t, int32_t layer, int32_t what, const float *src, void *hip_stream) {
    clear_error();
    if (!t || !src || layer < 0 || layer > t->nh || what < 0 || what > 1)
        return fail(DF_E_INVALID, "df_dnn_trainer_set: bad arguments");
    DnnLayer &Ly = t->dnn->layers[layer];
    auto s = static_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if (what == 0) {
        e = hipMemcpy2DAsync(t->W[layer], size_t(Ly.k_pad) * 4, src, size_t(Ly.n_in) * 4, size_t(Ly.n_in) * 4,
                             Ly.n_out, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) {
            const int64_t nw = int64_t(Ly.n_pad) * Ly.k_pad;
            hipLaunchKernelGGL(refresh_bf16_kernel, dim3(unsigned((nw + kT - 1) / kT)), dim3(kT), 0, s, t->W[layer],
                               Ly.n_pad, Ly.k_pad, Ly.W, t->WT[layer]);
            e = hipGetLastError();
        }
    } else {
        e = hipMemcpyAsync(t->b[layer], src, size_t(Ly.n_out) * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(Ly.b, src, size_t(Ly.n_out) * 4, hipMemcpyDeviceToDevice, s);
    }
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("df_dnn_trainer_set: ") + hipGetErrorString(e));
    return DF_OK;
}

df_status df_dnn_make_batch(const df_dnn *d, int64_t n, int64_t ld, const double *p, const double *T, const double *Y0,
                            const double *Y1, float *x, float *target, int32_t *valid, void *hip_stream) {
    clear_error();
    if (!d || n < 0 || ld < n) return fail(DF_E_INVALID, "df_dnn_make_batch: bad arguments");
    if (n > 0 && (!p || !T || !Y0 || !Y1 || !x || !target))
        return fail(DF_E_INVALID, "df_dnn_make_batch: null array");
    if (d->K != 9) return fail(DF_E_UNSUPPORTED, "df_dnn_make_batch: compiled for 9 species");
    if (n == 0) return DF_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, "df_dnn_make_batch: hipGetDevice failed");
    if (prev != d->device && hipSetDevice(d->device) != hipSuccess)
        return fail(DF_E_HIP, "df_dnn_make_batch: cannot select the network's device");
    hipLaunchKernelGGL(make_batch_kernel<9>, dim3(unsigned((n + kT - 1) / kT)), dim3(kT), 0,
                       static_cast<hipStream_t>(hip_stream), d->prm, n, ld, p, T, Y0, Y1, x, target, valid);
    const hipError_t e = hipGetLastError();
    if (prev != d->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("df_dnn_make_batch: ") + hipGetErrorString(e));
    return DF_OK;
}

}  // extern "C"
