// Dense layers of the DNN chemistry integrator on gfx950 matrix cores.
//
// C[M][N] = act(A[M][K] . B[N][K]^T + bias[N]), A = activations (one row per
// cell), B = weights (out x in, row-major), bf16 inputs, fp32 accumulation
// with v_mfma_f32_16x16x32_bf16, GELU epilogue, bf16 output.
// Block tile 128 x 160 with four wave64s in a 2 x 2 arrangement, each wave
// owning a 64 x 80 sub-tile (4 x 5 MFMA tiles); operands are staged through
// LDS 32 or 64 deep in K (64 where K allows it) with the next stage's global
// loads issued before the current stage's MFMAs.  The MFMAs take the weight
// fragment as their first operand, so that each lane ends with four consecutive
// outputs of one row, converted with one packed bf16 conversion pair: the GELU
// epilogues (inference, with GELU from an LDS table, and the training forward and
// backward) stage them per wave in LDS and write 16-byte row pieces; the linear
// epilogue writes them with one 8-byte store.  Tiles sharing the same rows of A are mapped to the same XCD so the A
// panel is fetched into that XCD's L2 once.
#include <algorithm>
#include <cmath>

#include "df_fp8.h"
#include "df_internal.h"
#include "df_phi_table.h"

namespace df {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = kGemmBM, BN = kGemmBN, BK = kGemmBK;
constexpr int kThreads = 256;
constexpr int WM = 64, WN = 80;          // per-wave sub-tile
constexpr int TM = WM / 16, TN = WN / 16;  // MFMA tiles per wave

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// GELU(x) = x Phi(x) of the inference and training epilogues without branches: Phi(x) = erfc(-x/sqrt 2) / 2,
// with erfc(a) for a >= 0 from the Chebyshev fit erfcc of Press et al., Numerical Recipes
// (Sec. 6.2), erfc(a) = t exp(-a^2 + P(t)), t = 1 / (1 + a/2), fractional error below 1.2e-7
// for every a >= 0; for x >= 0, Phi = 1 - erfc(x/sqrt 2) / 2.  Its error is far below the bf16
// rounding that follows.  NaN stays NaN; GELU(+inf) = +inf, GELU(-inf) = NaN as x Phi(x) gives.
__device__ __forceinline__ float phi_erfc(float x) {
    const float z = x * 0.70710678118654752f;
    const float a = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.5f * a);
    float q = 0.17087277f;
    q = fmaf(q, t, -0.82215223f);
    q = fmaf(q, t, 1.48851587f);
    q = fmaf(q, t, -1.13520398f);
    q = fmaf(q, t, 0.27886807f);
    q = fmaf(q, t, -0.18628806f);
    q = fmaf(q, t, 0.09678418f);
    q = fmaf(q, t, 0.37409196f);
    q = fmaf(q, t, 1.00002368f);
    q = fmaf(q, t, -1.26551223f);
    const float h = 0.5f * t * __expf(fmaf(-a, a, q));  // erfc(a) / 2
    return (z >= 0.0f) ? 1.0f - h : h;
}
__device__ __forceinline__ float gelu_erfc(float x) { return x * phi_erfc(x); }

// four floats to bf16 with two packed conversions (v_cvt_pk_bf16_f32): round to nearest even and
// NaN kept, except that fp32 subnormal inputs (|x| < 2^-126) are rounded toward zero, at most one
// bf16 subnormal unit (2^-133) from the nearest-even result
__device__ __forceinline__ bf16x4 to_bf16x4(floatx4 v) { return __builtin_convertvector(v, bf16x4); }

// d GELU / dx = Phi(x) + x phi(x), Phi as in gelu_erfc (no branches)
__device__ __forceinline__ float gelu_grad(float x) {
    return fmaf(x * 0.39894228040143268f, __expf(-0.5f * x * x), phi_erfc(x));
}

// GELU of the inference epilogues, GELU(x) = x Phi(x), with Phi from the table of one cubic per
// interval of 12/256 on [-6, 6] (kPhiTable, from erfc in double), which the block keeps in LDS.
// Interpolation error 1.5e-9; the position s = x 256/12 is rounded relative to x, so with the
// float32 evaluation the result is within about 1e-7 of x Phi(x), as close as gelu_erfc, so that
// the bf16 rounding that follows differs from that of the exact value as rarely.  Beyond the table
// Phi is 0 (x < -6 - 12/256, where the exact value is below 7e-10) or 1 (x >= 6).  NaN stays NaN;
// GELU(+inf) = +inf and GELU(-inf) = NaN, as x Phi(x) gives.  About 11 VALU instructions and one
// 16-byte LDS read per value, against about 28 instruction slots for gelu_erfc (reciprocal and
// exponential at a quarter of the rate).
constexpr int kPhiLdsFloats = 4 * kPhiEntries;  // 4,128 bytes of LDS per block

__device__ __forceinline__ float gelu_tab(float x, const float *__restrict__ tab) {
    constexpr float kScale = float(kPhiIntervals) / 12.0f, kHalf = 0.5f * float(kPhiIntervals);
    // position in intervals from 0, clamped to the table: entry 0 (zeros) below -6, entries
    // 1 .. kPhiIntervals the cubics, entry kPhiIntervals + 1 from 6 on; fmaxf maps NaN to entry 0
    const float s = fminf(fmaxf(x * kScale, -kHalf - 1.0f), kHalf);
    const int k = int(floorf(s)) + int(kHalf) + 1;  // 0 .. kPhiIntervals + 1
    const float u = __builtin_amdgcn_fractf(s);
    const floatx4 c = *reinterpret_cast<const floatx4 *>(tab + 4 * k);
    return x * fmaf(fmaf(fmaf(c[3], u, c[2]), u, c[1]), u, c[0]);
}

// copies the table into the block's LDS copy in 16-byte pieces; a barrier must follow before the
// first gelu_tab
__device__ __forceinline__ void copy_phi_table(float *__restrict__ lds, int t) {
    const u32x4 *src = reinterpret_cast<const u32x4 *>(kPhiTable);
    u32x4 *dst = reinterpret_cast<u32x4 *>(lds);
    for (int i = t; i < kPhiLdsFloats / 4; i += kThreads) dst[i] = src[i];
}

// Output staging of the inference epilogues: a wave writes rows of 160 output bytes (80 bf16 or
// 160 FP8 values) into its own LDS region, stride 176 bytes, and then stores them as 16-byte
// pieces, consecutive lanes along a row.  In the MFMA layout a store covers 16 rows x 32 bytes
// (bf16) or 16 bytes (FP8); a store-only probe of the first layer's tiles measured that 1.7 times
// slower than row pieces (65,536 x 1600 bf16: 55.4 against 32.5 us, a plain stream 32.5 us).
constexpr int kStgRowB = 160, kStgStrideB = kStgRowB + 16;

// the wave's own LDS region: its LDS operations execute in order, so reads after writes see them
// and later writes follow earlier reads; the fences keep the compiler from moving LDS accesses
// across
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ROWS staged rows to dst (the first row's first byte, 16-byte aligned), ld_bytes apart
template <int ROWS>
__device__ __forceinline__ void stage_flush(const uint8_t *stg, uint8_t *dst, int64_t ld_bytes, int lane) {
    constexpr int kPer = kStgRowB / 16, kPieces = ROWS * kPer;
    static_assert(kPieces % 64 == 0, "whole waves of pieces");
    wave_lds_fence();
#pragma unroll
    for (int p0 = 0; p0 < kPieces; p0 += 64) {
        const int c = p0 + lane, r = c / kPer, ch = c % kPer;
        const u32x4 v = *reinterpret_cast<const u32x4 *>(stg + r * kStgStrideB + ch * 16);
        *reinterpret_cast<u32x4 *>(dst + r * ld_bytes + ch * 16) = v;
    }
    wave_lds_fence();
}

// Epilogues: inference (bias, GELU); training forward (bias, GELU, and the pre-activation
// stored to P with C's layout); training backward (the product times GELU'(P), no bias).
enum { kEpiGelu = 0, kEpiLinear = 1, kEpiGeluSave = 2, kEpiGeluGrad = 3 };

// KD: reduction depth staged per barrier pair (32, or 64 where K allows it)
// (the 32-deep kernel at three blocks per CU: at most 168 registers, measured 4-6 % faster on
// the 800 -> 400 layer; the 64-deep one keeps two, where the register cap cost 15 %)
template <int EPI, int KD>
__global__ __launch_bounds__(kThreads, KD == 32 ? 3 : 1) void gemm_kernel(const bf16_t *__restrict__ A, int lda,
                                                       const bf16_t *__restrict__ B, int ldb,
                                                       const float *__restrict__ bias, bf16_t *__restrict__ C,
                                                       int ldc, int K, int n_tiles_n, bf16_t *__restrict__ P) {
    constexpr int LDKD = KD + 16;  // LDS row stride in bf16 (96 bytes at KD = 32)
    // the operand stages; after the stage loop the inference epilogue stages its outputs here
    __shared__ __attribute__((aligned(16))) bf16_t ABs[(BM + BN) * LDKD];
    bf16_t *const As = ABs, *const Bs = ABs + BM * LDKD;
    __shared__ __attribute__((aligned(16))) float Ptab[EPI == kEpiGelu ? kPhiLdsFloats : 4];

    // XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs, so
    // block b runs on XCD b % 8; give each XCD a contiguous range of logical tiles.
    const int nb = gridDim.x, b = blockIdx.x;
    const int logical = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int tile_m = logical / n_tiles_n, tile_n = logical % n_tiles_n;
    const int64_t row0 = int64_t(tile_m) * BM;
    const int col0 = tile_n * BN;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;

    // global -> register staging: A has BM*KD/8 16-byte chunks (512 at KD = 32), B has BN*KD/8 (640)
    constexpr int kAChunks = BM * KD / 8, kBChunks = BN * KD / 8;
    constexpr int kAPer = kAChunks / kThreads;
    constexpr int kBPer = (kBChunks + kThreads - 1) / kThreads;
    u32x4 ra[kAPer], rb[kBPer];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < kAPer; ++i) {
            const int c = t + i * kThreads, r = c / (KD / 8), kc = c % (KD / 8);
            ra[i] = *reinterpret_cast<const u32x4 *>(A + (row0 + r) * lda + k0 + kc * 8);
        }
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int c = t + i * kThreads;
            if (c < kBChunks) {
                const int r = c / (KD / 8), kc = c % (KD / 8);
                rb[i] = *reinterpret_cast<const u32x4 *>(B + int64_t(col0 + r) * ldb + k0 + kc * 8);
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < kAPer; ++i) {
            const int c = t + i * kThreads, r = c / (KD / 8), kc = c % (KD / 8);
            *reinterpret_cast<u32x4 *>(As + r * LDKD + kc * 8) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int c = t + i * kThreads;
            if (c < kBChunks) {
                const int r = c / (KD / 8), kc = c % (KD / 8);
                *reinterpret_cast<u32x4 *>(Bs + r * LDKD + kc * 8) = rb[i];
            }
        }
    };

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    // MFMA 16x16x32 operands: lane l supplies row (l % 16) of the A tile and column (l % 16) of
    // the B tile, with 8 consecutive k values starting at 8 * (l / 16)
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    load(0);
    if (EPI == kEpiGelu) copy_phi_table(Ptab, t);  // visible after the stage loop's first barrier
    for (int k0 = 0; k0 < K; k0 += KD) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + KD < K) load(k0 + KD);
        // the staged depth in 32-deep MFMA steps, in k order (the sums are those of KD = 32)
#pragma unroll
        for (int kk = 0; kk < KD; kk += 32) {
            bf16x8 af[TM], bfr[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const bf16x8 *>(As + (wm * WM + i * 16 + fr) * LDKD + kk + fk);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn * WN + j * 16 + fr) * LDKD + kk + fk);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
        }
    }

    // epilogue: with the weights as the first MFMA operand, lane l holds row (l % 16) and the four
    // columns 4 * (l / 16) + r of each 16 x 16 tile
    if constexpr (EPI != kEpiLinear) {
        // staged through the operand buffers, in two halves of 32 rows per wave; the training
        // forward stages its pre-activations (P) first and then its outputs
        static_assert(4 * 32 * kStgStrideB <= (BM + BN) * LDKD * 2 && WN * 2 == kStgRowB, "staging");
        __syncthreads();  // every wave has read its last operand fragments
        uint8_t *const stg = reinterpret_cast<uint8_t *>(ABs) + w * (32 * kStgStrideB);
        const int64_t ldb_c = 2 * int64_t(ldc);
        const int64_t off0 = (row0 + wm * WM) * ldb_c + 2 * (col0 + wn * WN);
        const int fc = (lane >> 4) * 4;  // the lane's first column in a 16 x 16 tile
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            floatx4 v[TN][2];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const floatx4 bc = (EPI == kEpiGeluGrad)
                                       ? floatx4{0.f, 0.f, 0.f, 0.f}
                                       : *reinterpret_cast<const floatx4 *>(bias + col0 + wn * WN + j * 16 + fc);
#pragma unroll
                for (int ii = 0; ii < 2; ++ii) v[j][ii] = acc[2 * hf + ii][j] + bc;
            }
            if constexpr (EPI == kEpiGeluSave) {
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int ii = 0; ii < 2; ++ii)
                        *reinterpret_cast<bf16x4 *>(stg + (ii * 16 + fr) * kStgStrideB + 2 * (j * 16 + fc)) =
                            to_bf16x4(v[j][ii]);
                stage_flush<32>(stg, reinterpret_cast<uint8_t *>(P) + off0 + hf * 32 * ldb_c, ldb_c, lane);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int ii = 0; ii < 2; ++ii) {
                    floatx4 x = v[j][ii];
                    if constexpr (EPI == kEpiGelu) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) x[r] = gelu_tab(x[r], Ptab);
                    } else if constexpr (EPI == kEpiGeluSave) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) x[r] = gelu_erfc(x[r]);
                    } else {
                        const int64_t row = row0 + wm * WM + (2 * hf + ii) * 16 + fr;
                        const bf16x4 pv =
                            *reinterpret_cast<const bf16x4 *>(P + row * ldc + col0 + wn * WN + j * 16 + fc);
#pragma unroll
                        for (int r = 0; r < 4; ++r) x[r] *= gelu_grad(float(pv[r]));
                    }
                    *reinterpret_cast<bf16x4 *>(stg + (ii * 16 + fr) * kStgStrideB + 2 * (j * 16 + fc)) =
                        to_bf16x4(x);
                }
            stage_flush<32>(stg, reinterpret_cast<uint8_t *>(C) + off0 + hf * 32 * ldb_c, ldb_c, lane);
        }
        return;
    }
    // the linear epilogue (bias only) stores in the MFMA layout
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int col = col0 + wn * WN + j * 16 + (lane >> 4) * 4;
        const floatx4 bc = *reinterpret_cast<const floatx4 *>(bias + col);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int64_t row = row0 + wm * WM + i * 16 + fr;
            const int64_t off = row * ldc + col;
            const floatx4 v = acc[i][j] + bc;
            *reinterpret_cast<bf16x4 *>(C + off) = to_bf16x4(v);
        }
    }
}

// A value the E4M3FN conversion takes as is: |x| <= 448 unchanged; 448 < |x| <= 464 rounds to
// 448 (ties to even) and is passed as 448; a value that would round beyond 448, an infinity or a
// NaN becomes NaN, the format's only non-finite value, so that it propagates to the cell's
// status as in the bf16 path.  The block scale keeps every finite scaled value within 448; the
// other cases arise only when the block's maximum itself is not finite.
__device__ __forceinline__ float fp8_in_range(float x) {
    // without branches: clamp to [-448, 448] (leaves |x| <= 448 and -0 as they are), then NaN
    // where |x| > 464 or x is NaN (the comparison is false for NaN)
    const float c = __builtin_amdgcn_fmed3f(x, -448.0f, 448.0f);
    return (fabsf(x) <= 464.0f) ? c : __builtin_nanf("");
}

// E4M3FN bytes of four floats (round to nearest even)
__device__ __forceinline__ uint32_t to_fp8x4(float a, float b, float c, float d) {
    a = fp8_in_range(a);
    b = fp8_in_range(b);
    c = fp8_in_range(c);
    d = fp8_in_range(d);
    int v = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);  // bytes 0, 1
    v = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, v, true);       // bytes 2, 3
    return uint32_t(v);
}

// FP8 output of a layer whose result feeds an FP8 layer, for a wave that owns whole 32-column
// blocks: v0 and v1 are the GELU outputs of the 16 x 16 tiles 2q and 2q + 1 of a 16-row tile
// (lane l: row l % 16, columns 4 (l / 16) + r of each), so a block's 32 values of a row lie with
// the four lanes l % 16 + 16 g'.  Each value is rounded to bf16 first (the hidden activations are
// bf16 values in every precision), the block's largest magnitude is combined over the four lanes
// (NaN ignored), and the values are quantised with the block's scale: the lane's E4M3FN bytes of
// Q[row][c0 .. c0 + 32) as two words (bytes 4 g .. 4 g + 3 and 16 + 4 g .. 16 + 4 g + 3), and the
// E8M0 scale byte to S[row][c0 / 32].
__device__ __forceinline__ void quant_fp8_block(floatx4 v0, floatx4 v1, uint8_t *__restrict__ S, int64_t row,
                                                int sst, int c0, int g, uint32_t &w0, uint32_t &w1) {
    const bf16x4 h0 = to_bf16x4(v0), h1 = to_bf16x4(v1);
    float f[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        f[r] = float(h0[r]);
        f[4 + r] = float(h1[r]);
    }
    float m = 0.0f;
#pragma unroll
    for (int r = 0; r < 8; ++r) m = fmaxf(m, fabsf(f[r]));
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 32));
    const int e = fp8_scale_exp(m);
    const float sc = ldexpf(1.0f, -e);
    if (m <= 3.40282347e38f) {
        // a finite block maximum: the scale keeps every scaled value within 448 (a NaN value
        // stays NaN through the conversion), so the range rule has nothing to do
        int v = __builtin_amdgcn_cvt_pk_fp8_f32(f[0] * sc, f[1] * sc, 0, false);
        w0 = uint32_t(__builtin_amdgcn_cvt_pk_fp8_f32(f[2] * sc, f[3] * sc, v, true));
        v = __builtin_amdgcn_cvt_pk_fp8_f32(f[4] * sc, f[5] * sc, 0, false);
        w1 = uint32_t(__builtin_amdgcn_cvt_pk_fp8_f32(f[6] * sc, f[7] * sc, v, true));
    } else {
        w0 = to_fp8x4(f[0] * sc, f[1] * sc, f[2] * sc, f[3] * sc);
        w1 = to_fp8x4(f[4] * sc, f[5] * sc, f[6] * sc, f[7] * sc);
    }
    if (g == 0) S[row * sst + c0 / kFp8Block] = uint8_t(127 + e);
}

// Inference layer with a shallow reduction (K = KD <= 64, the first hidden layer: the network's
// inputs padded to 32 or 64): no K loop to pipeline, so the time is the GELU epilogue and the
// stores of the M x N outputs.  Each block keeps one 160-column weight panel in registers as MFMA
// fragments and walks down the row tiles tile_m = g, g + G, ... (G = gridDim.x / n_tiles_n),
// loading each tile's activation fragments straight from global memory (16 rows x 64 contiguous
// bytes per load) one tile ahead, so that the loads of the next tile are in flight during the
// epilogue of the current one; LDS holds only the GELU table (one barrier, at the start).  Same tile shape, operand order and
// epilogue (bias, GELU, bf16) as gemm_kernel; with Q8 the output is the FP8 copy the next layer
// reads (quant_fp8_block), and the four waves take 32 rows x 160 columns each so that every
// wave owns whole 32-column blocks.  Each wave writes its outputs (160 bytes per row either way)
// to its own LDS region first and then to memory as 16-byte pieces, consecutive lanes along a
// row: the MFMA layout would give 16 rows x 32 bytes (bf16) or 16 bytes (FP8) per store, which
// measured about 1.7 times slower than row pieces for these outputs.  In the FP8 copy the bias
// row is read from LDS in the epilogue: held in registers (40 of them next to a 160-column weight
// panel) it left none for the staging at KD = 64, which then spilled and ran 14 % slower.
template <int KD, bool Q8>
__global__ __launch_bounds__(kThreads, 2) void gemm_shallow_kernel(const bf16_t *__restrict__ A, int lda,
                                                                const bf16_t *__restrict__ B, int ldb,
                                                                const float *__restrict__ bias,
                                                                bf16_t *__restrict__ C, int ldc,
                                                                uint8_t *__restrict__ S, int sst, int n_tiles_m,
                                                                int n_tiles_n) {
    constexpr int KS = KD / 32;  // 32-deep MFMA steps
    constexpr int WMq = Q8 ? 32 : WM, WNq = Q8 ? 160 : WN, TMq = WMq / 16, TNq = WNq / 16;
    const int tile_n = int(blockIdx.x) % n_tiles_n, g0 = int(blockIdx.x) / n_tiles_n;
    const int G = int(gridDim.x) / n_tiles_n;
    const int col0 = tile_n * BN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = Q8 ? w : w >> 1, wn = Q8 ? 0 : w & 1;
    const int fr = lane & 15, fg = lane >> 4, fk = fg * 8;
    __shared__ __attribute__((aligned(16))) float Ptab[kPhiLdsFloats];
    copy_phi_table(Ptab, t);
    // the wave's staging rows (160 bytes of outputs each)
    static_assert((Q8 ? WNq : 2 * WNq) == kStgRowB, "staging layout");
    __shared__ __attribute__((aligned(16))) uint8_t Stage[4 * WMq * kStgStrideB];
    __shared__ __attribute__((aligned(16))) float Bias[Q8 ? BN : 4];
    if (Q8 && t < BN / 4)
        reinterpret_cast<floatx4 *>(Bias)[t] = reinterpret_cast<const floatx4 *>(bias + col0)[t];
    uint8_t *stg = Stage + w * (WMq * kStgStrideB);
    uint8_t *const Cb = reinterpret_cast<uint8_t *>(C);
    const int col0b = Q8 ? col0 : 2 * (col0 + wn * WNq);  // byte column of the wave's sub-tile
    const int64_t ldcb = Q8 ? ldc : 2 * int64_t(ldc);

    bf16x8 bfr[KS][TNq];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int j = 0; j < TNq; ++j)
            bfr[s][j] = *reinterpret_cast<const bf16x8 *>(B + int64_t(col0 + wn * WNq + j * 16 + fr) * ldb + s * 32 + fk);
    floatx4 bc[Q8 ? 1 : TNq];  // the bf16 path holds its 80-column bias slice in registers
    if constexpr (!Q8) {
#pragma unroll
        for (int j = 0; j < TNq; ++j)
            bc[j] = *reinterpret_cast<const floatx4 *>(bias + col0 + wn * WNq + j * 16 + fg * 4);
    }

    auto load_a = [&](int tm, bf16x8 (&af)[KS][TMq]) {
        const int64_t r0 = int64_t(tm) * BM + wm * WMq + fr;
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int i = 0; i < TMq; ++i)
                af[s][i] = *reinterpret_cast<const bf16x8 *>(A + (r0 + i * 16) * lda + s * 32 + fk);
    };
    bf16x8 an[KS][TMq];
    if (g0 < n_tiles_m) load_a(g0, an);
    __syncthreads();  // the table is in LDS
    for (int tm = g0; tm < n_tiles_m; tm += G) {
        bf16x8 af[KS][TMq];
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int i = 0; i < TMq; ++i) af[s][i] = an[s][i];
        if (tm + G < n_tiles_m) load_a(tm + G, an);
        floatx4 acc[TMq][TNq];
#pragma unroll
        for (int i = 0; i < TMq; ++i)
#pragma unroll
            for (int j = 0; j < TNq; ++j) {
                acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < KS; ++s)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[s][j], af[s][i], acc[i][j], 0, 0, 0);
            }
        const int64_t rowt = int64_t(tm) * BM + wm * WMq;  // first row of the wave's sub-tile
        if constexpr (Q8) {
#pragma unroll
            for (int i = 0; i < TMq; ++i)
#pragma unroll
                for (int q = 0; q < TNq / 2; ++q) {
                    const floatx4 *bl = reinterpret_cast<const floatx4 *>(Bias + 32 * q + fg * 4);
                    floatx4 v0 = acc[i][2 * q] + bl[0], v1 = acc[i][2 * q + 1] + bl[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        v0[r] = gelu_tab(v0[r], Ptab);
                        v1[r] = gelu_tab(v1[r], Ptab);
                    }
                    uint32_t w0, w1;
                    quant_fp8_block(v0, v1, S, rowt + i * 16 + fr, sst, col0 + 32 * q, fg, w0, w1);
                    uint8_t *p = stg + (i * 16 + fr) * kStgStrideB + 32 * q + 4 * fg;
                    *reinterpret_cast<uint32_t *>(p) = w0;
                    *reinterpret_cast<uint32_t *>(p + 16) = w1;
                }
        } else {
#pragma unroll
            for (int j = 0; j < TNq; ++j) {
#pragma unroll
                for (int i = 0; i < TMq; ++i) {
                    floatx4 v = acc[i][j] + bc[j];
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = gelu_tab(v[r], Ptab);
                    *reinterpret_cast<bf16x4 *>(stg + (i * 16 + fr) * kStgStrideB + 2 * (j * 16 + fg * 4)) =
                        to_bf16x4(v);
                }
            }
        }
        stage_flush<WMq>(stg, Cb + rowt * ldcb + col0b, ldcb, lane);
    }
}

// FP8 layer on the block-scaled matrix cores: the tiling of gemm_kernel (128 x 160 block tile,
// 2 x 2 waves of 64 x 80) with 128-deep stages of E4M3FN bytes.  In a 16x16x128 product with
// 8-bit operands, lane l supplies row l % 16 of its operand at the stage's inputs 16 g .. 16 g + 15
// (bytes 0-15) and 64 + 16 g .. 64 + 16 g + 15 (bytes 16-31), g = l / 16, and the E8M0 scale of
// the inputs 32 g .. 32 g + 31 of that row: its two halves lie with lanes g' = 2 (g % 2) and
// 2 (g % 2) + 1 (measured on gfx950 with one-hot data and per-lane scales).  So each lane reads
// the two 16-byte pieces of its row at 16 g and 64 + 16 g, and passes the scale of activation
// block g of the stage (the weight row's scale, 127 + wexp, is the same for all blocks).  Inputs
// at or beyond K (the last stage of a K that is not a multiple of 128) are zeros with scale 2^0.
typedef int i32x8 __attribute__((ext_vector_type(8)));
constexpr int KD8 = 128, LDK8 = KD8 + 16;  // stage depth and LDS row stride in bytes

template <bool Q8>
__global__ __launch_bounds__(kThreads, 2) void gemm_fp8_kernel(const uint8_t *__restrict__ A8, int lda,
                                                           const uint8_t *__restrict__ SA, int sst,
                                                           const uint8_t *__restrict__ W8, int ldb,
                                                           const int32_t *__restrict__ wexp,
                                                           const float *__restrict__ bias, bf16_t *__restrict__ C,
                                                           int ldc, uint8_t *__restrict__ SC, int sstc, int K,
                                                           int n_tiles_n) {
    constexpr int WMq = Q8 ? 32 : WM, WNq = Q8 ? 160 : WN, TMq = WMq / 16, TNq = WNq / 16;
    // the operand stages; after the stage loop the epilogue stages its outputs here
    __shared__ __attribute__((aligned(16))) uint8_t AB8[(BM + BN) * LDK8];
    uint8_t *const As = AB8, *const Bs = AB8 + BM * LDK8;
    __shared__ uint32_t Ss[BM];
    __shared__ __attribute__((aligned(16))) float Ptab[kPhiLdsFloats];

    const int nb = gridDim.x, b = blockIdx.x;
    const int logical = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int tile_m = logical / n_tiles_n, tile_n = logical % n_tiles_n;
    const int64_t row0 = int64_t(tile_m) * BM;
    const int col0 = tile_n * BN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = Q8 ? w : w >> 1, wn = Q8 ? 0 : w & 1;
    const int fr = lane & 15, fg = lane >> 4;

    // 16-byte chunks: A BM*KD8/16 = 1024 (4 per thread), W BN*KD8/16 = 1280 (5 per thread)
    constexpr int kCh = KD8 / 16;
    constexpr int kAPer = BM * kCh / kThreads, kBPer = BN * kCh / kThreads;
    u32x4 ra[kAPer], rb[kBPer];
    uint32_t rs = 0;
    const u32x4 z4 = {0u, 0u, 0u, 0u};
    auto load = [&](int k0) {
        if (k0 + KD8 <= K) {
            // a whole stage within K (the same for the block): no guards, and the four block
            // scales of a row as one little-endian word (4-byte aligned: sst % 16 = 0, k0 % 128 = 0)
#pragma unroll
            for (int i = 0; i < kAPer; ++i) {
                const int c = t + i * kThreads, r = c / kCh, k = k0 + (c % kCh) * 16;
                ra[i] = *reinterpret_cast<const u32x4 *>(A8 + (row0 + r) * lda + k);
            }
#pragma unroll
            for (int i = 0; i < kBPer; ++i) {
                const int c = t + i * kThreads, r = c / kCh, k = k0 + (c % kCh) * 16;
                rb[i] = *reinterpret_cast<const u32x4 *>(W8 + int64_t(col0 + r) * ldb + k);
            }
            if (t < BM) rs = *reinterpret_cast<const uint32_t *>(SA + (row0 + t) * sst + k0 / kFp8Block);
            return;
        }
#pragma unroll
        for (int i = 0; i < kAPer; ++i) {
            const int c = t + i * kThreads, r = c / kCh, k = k0 + (c % kCh) * 16;
            ra[i] = (k < K) ? *reinterpret_cast<const u32x4 *>(A8 + (row0 + r) * lda + k) : z4;
        }
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int c = t + i * kThreads, r = c / kCh, k = k0 + (c % kCh) * 16;
            rb[i] = (k < K) ? *reinterpret_cast<const u32x4 *>(W8 + int64_t(col0 + r) * ldb + k) : z4;
        }
        // the four block scales of a row for this stage; 127 (2^0) for blocks at or beyond K
        if (t < BM) {
            const uint8_t *sp = SA + (row0 + t) * sst + k0 / kFp8Block;
            uint32_t v = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) v |= uint32_t((k0 + q * kFp8Block < K) ? sp[q] : 127) << (8 * q);
            rs = v;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < kAPer; ++i) {
            const int c = t + i * kThreads;
            *reinterpret_cast<u32x4 *>(As + (c / kCh) * LDK8 + (c % kCh) * 16) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int c = t + i * kThreads;
            *reinterpret_cast<u32x4 *>(Bs + (c / kCh) * LDK8 + (c % kCh) * 16) = rb[i];
        }
        if (t < BM) Ss[t] = rs;
    };

    int sw[TNq];  // E8M0 scale of the weight row each lane supplies
#pragma unroll
    for (int j = 0; j < TNq; ++j) sw[j] = 127 + wexp[col0 + wn * WNq + j * 16 + fr];
    floatx4 acc[TMq][TNq];
#pragma unroll
    for (int i = 0; i < TMq; ++i)
#pragma unroll
        for (int j = 0; j < TNq; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    load(0);
    copy_phi_table(Ptab, t);  // visible after the stage loop's first barrier
    for (int k0 = 0; k0 < K; k0 += KD8) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + KD8 < K) load(k0 + KD8);
        auto frag = [&](const uint8_t *row) {
            const u32x4 lo = *reinterpret_cast<const u32x4 *>(row + fg * 16);
            const u32x4 hi = *reinterpret_cast<const u32x4 *>(row + 64 + fg * 16);
            return i32x8{int(lo[0]), int(lo[1]), int(lo[2]), int(lo[3]), int(hi[0]), int(hi[1]), int(hi[2]), int(hi[3])};
        };
        // the activation fragments (fewer than the weight ones) held, the weight fragments one at a time
        i32x8 af[TMq];
        int sa[TMq];
#pragma unroll
        for (int i = 0; i < TMq; ++i) {
            const int r = wm * WMq + i * 16 + fr;
            af[i] = frag(As + r * LDK8);
            sa[i] = int((Ss[r] >> (8 * fg)) & 0xffu);
        }
#pragma unroll
        for (int j = 0; j < TNq; ++j) {
            const i32x8 wf = frag(Bs + (wn * WNq + j * 16 + fr) * LDK8);
#pragma unroll
            for (int i = 0; i < TMq; ++i)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(wf, af[i], acc[i][j], 0, 0, 0, sw[j], 0, sa[i]);
        }
    }

    // outputs staged through the operand buffers: the FP8 copy as one stage of 32 rows x 160
    // bytes per wave, bf16 outputs in two halves of 32 rows x 80 values
    static_assert(4 * 32 * kStgStrideB <= (BM + BN) * LDK8, "staging fits the operand buffers");
    __syncthreads();  // every wave has read its last operand fragments
    uint8_t *const stg = AB8 + w * (32 * kStgStrideB);
    if constexpr (Q8) {
#pragma unroll
        for (int q = 0; q < TNq / 2; ++q) {
            const floatx4 b0 = *reinterpret_cast<const floatx4 *>(bias + col0 + 32 * q + fg * 4);
            const floatx4 b1 = *reinterpret_cast<const floatx4 *>(bias + col0 + 32 * q + 16 + fg * 4);
#pragma unroll
            for (int i = 0; i < TMq; ++i) {
                floatx4 v0 = acc[i][2 * q] + b0, v1 = acc[i][2 * q + 1] + b1;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    v0[r] = gelu_tab(v0[r], Ptab);
                    v1[r] = gelu_tab(v1[r], Ptab);
                }
                uint32_t w0, w1;
                quant_fp8_block(v0, v1, SC, row0 + wm * WMq + i * 16 + fr, sstc, col0 + 32 * q, fg, w0, w1);
                uint8_t *p = stg + (i * 16 + fr) * kStgStrideB + 32 * q + 4 * fg;
                *reinterpret_cast<uint32_t *>(p) = w0;
                *reinterpret_cast<uint32_t *>(p + 16) = w1;
            }
        }
        stage_flush<32>(stg, reinterpret_cast<uint8_t *>(C) + (row0 + wm * WMq) * int64_t(ldc) + col0, ldc, lane);
    } else {
        const int64_t ldb_c = 2 * int64_t(ldc);
        uint8_t *const dst = reinterpret_cast<uint8_t *>(C) + (row0 + wm * WMq) * ldb_c + 2 * (col0 + wn * WNq);
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
            for (int j = 0; j < TNq; ++j) {
                const floatx4 bc = *reinterpret_cast<const floatx4 *>(bias + col0 + wn * WNq + j * 16 + fg * 4);
#pragma unroll
                for (int ii = 0; ii < 2; ++ii) {
                    floatx4 v = acc[2 * hf + ii][j] + bc;
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = gelu_tab(v[r], Ptab);
                    *reinterpret_cast<bf16x4 *>(stg + (ii * 16 + fr) * kStgStrideB + 2 * (j * 16 + fg * 4)) =
                        to_bf16x4(v);
                }
            }
            stage_flush<32>(stg, dst + hf * 32 * ldb_c, ldb_c, lane);
        }
    }
}

// the shallow-reduction layer (K = 32 or 64, shapes checked by the caller): about two blocks per
// CU, each on one 160-column panel and every G-th row tile; S != nullptr: FP8 output (C holds the
// E4M3FN bytes with row stride ldc, S the block scales with row stride sst)
df_status launch_shallow(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C, int ldc,
                         uint8_t *S, int sst, int64_t M, int N, int K, hipStream_t stream) {
    const int64_t tm = M / BM;
    const int tn = N / BN;
    if (tm > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "gemm: too many row tiles");
    // the outputs are written as 16-byte row pieces
    if ((reinterpret_cast<uintptr_t>(C) & 15) || (S ? ldc % 16 : ldc % 8))
        return fail(DF_E_INVALID, "gemm: the output rows must be 16-byte aligned");
    const int G = int(std::max<int64_t>(1, std::min<int64_t>(tm, std::max(1, 512 / tn))));
    const dim3 g = dim3(unsigned(int64_t(G) * tn)), b = dim3(kThreads);
#define DF_SHALLOW(KD, Q)                                                                                        \
    hipLaunchKernelGGL((gemm_shallow_kernel<KD, Q>), g, b, 0, stream, A, lda, B, ldb, bias, C, ldc, S, sst, int(tm), \
                       tn)
    if (K == 32) {
        if (S)
            DF_SHALLOW(32, true);
        else
            DF_SHALLOW(32, false);
    } else {
        if (S)
            DF_SHALLOW(64, true);
        else
            DF_SHALLOW(64, false);
    }
#undef DF_SHALLOW
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("gemm launch: ") + hipGetErrorString(e));
    return DF_OK;
}

}  // namespace

df_status launch_gemm_bf16(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C, int ldc,
                           int64_t M, int N, int K, bool gelu, hipStream_t stream) {
    return launch_gemm_bf16_epi(A, lda, B, ldb, bias, C, ldc, M, N, K, gelu ? GemmEpi::gelu : GemmEpi::linear, nullptr,
                                stream);
}

df_status launch_gemm_bf16_epi(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C,
                               int ldc, int64_t M, int N, int K, GemmEpi epi, bf16_t *P, hipStream_t stream) {
    if (M % BM || N % BN || K % BK || K <= 0 || lda % 8 || ldb % 8)
        return fail(DF_E_INVALID, "gemm: shapes must be multiples of the tile sizes");
    // the outputs of every epilogue but the linear one are written as 16-byte row pieces
    if (epi != GemmEpi::linear && ((reinterpret_cast<uintptr_t>(C) & 15) || ldc % 8 ||
                                   (epi == GemmEpi::gelu_save && (reinterpret_cast<uintptr_t>(P) & 15))))
        return fail(DF_E_INVALID, "gemm: the output rows must be 16-byte aligned");
    if ((epi == GemmEpi::gelu_save || epi == GemmEpi::gelu_grad) && !P)
        return fail(DF_E_INVALID, "gemm: the epilogue needs the pre-activation array");
    if (M == 0) return DF_OK;
    const int64_t tiles = (M / BM) * (N / BN);
    if (tiles > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "gemm: too many tiles");
    if (epi == GemmEpi::gelu && (K == 32 || K == 64))
        return launch_shallow(A, lda, B, ldb, bias, C, ldc, nullptr, 0, M, N, K, stream);
    const dim3 g = dim3(unsigned(tiles)), b = dim3(kThreads);
    const bool deep = K % 64 == 0;
#define DF_GEMM(E)                                                                                              \
    if (deep)                                                                                                   \
        hipLaunchKernelGGL((gemm_kernel<E, 64>), g, b, 0, stream, A, lda, B, ldb, bias, C, ldc, K, N / BN, P);  \
    else                                                                                                        \
        hipLaunchKernelGGL((gemm_kernel<E, 32>), g, b, 0, stream, A, lda, B, ldb, bias, C, ldc, K, N / BN, P);
    switch (epi) {
        case GemmEpi::gelu:
            DF_GEMM(kEpiGelu)
            break;
        case GemmEpi::linear:
            DF_GEMM(kEpiLinear)
            break;
        case GemmEpi::gelu_save:
            DF_GEMM(kEpiGeluSave)
            break;
        case GemmEpi::gelu_grad:
            DF_GEMM(kEpiGeluGrad)
            break;
    }
#undef DF_GEMM
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("gemm launch: ") + hipGetErrorString(e));
    return DF_OK;
}

df_status launch_gemm_bf16_fp8out(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, uint8_t *Q,
                                  int ldq, uint8_t *S, int sst, int64_t M, int N, int K, hipStream_t stream) {
    if (M % BM || N % BN || lda % 8 || ldb % 8 || ldq % 16 || sst % 16 || sst < N / kFp8Block || !Q || !S)
        return fail(DF_E_INVALID, "gemm: shapes must be multiples of the tile sizes");
    if (K != 32 && K != 64) return fail(DF_E_UNSUPPORTED, "gemm with FP8 output: only a reduction depth of 32 or 64");
    if (M == 0) return DF_OK;
    return launch_shallow(A, lda, B, ldb, bias, reinterpret_cast<bf16_t *>(Q), ldq, S, sst, M, N, K, stream);
}

df_status launch_gemm_fp8(const uint8_t *A8, int lda, const uint8_t *S, int sst, const uint8_t *W8, int ldb,
                          const int32_t *wexp, const float *bias, bf16_t *C, int ldc, uint8_t *SC, int sstc,
                          int64_t M, int N, int K, hipStream_t stream) {
    if (M % BM || N % BN || K % kFp8Block || K <= 0 || lda % 16 || ldb % 16 || sst % 16 || lda < K || ldb < K ||
        sst < K / kFp8Block || (SC && (ldc % 16 || sstc % 16 || sstc < N / kFp8Block)))
        return fail(DF_E_INVALID, "gemm fp8: shapes must be multiples of the tile sizes (rows of 16 bytes)");
    if (!A8 || !S || !W8 || !wexp) return fail(DF_E_INVALID, "gemm fp8: null activation, scale, weight or exponent array");
    if (reinterpret_cast<uintptr_t>(S) & 3) return fail(DF_E_INVALID, "gemm fp8: the scale array must be 4-byte aligned");
    if ((reinterpret_cast<uintptr_t>(C) & 15) || ldc % 8)  // outputs written as 16-byte row pieces
        return fail(DF_E_INVALID, "gemm fp8: the output rows must be 16-byte aligned");
    if (M == 0) return DF_OK;
    const int64_t tiles = (M / BM) * (N / BN);
    if (tiles > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "gemm fp8: too many tiles");
    if (SC)
        hipLaunchKernelGGL(gemm_fp8_kernel<true>, dim3(unsigned(tiles)), dim3(kThreads), 0, stream, A8, lda, S, sst, W8,
                           ldb, wexp, bias, C, ldc, SC, sstc, K, N / BN);
    else
        hipLaunchKernelGGL(gemm_fp8_kernel<false>, dim3(unsigned(tiles)), dim3(kThreads), 0, stream, A8, lda, S, sst,
                           W8, ldb, wexp, bias, C, ldc, SC, sstc, K, N / BN);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("gemm fp8 launch: ") + hipGetErrorString(e));
    return DF_OK;
}

}  // namespace df
