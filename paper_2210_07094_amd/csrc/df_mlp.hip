// Dense layers of the DNN chemistry integrator on gfx950 matrix cores.
//
// C[M][N] = act(A[M][K] . B[N][K]^T + bias[N]), A = activations (one row per
// cell), B = weights (out x in, row-major), bf16 inputs, fp32 accumulation
// with v_mfma_f32_16x16x32_bf16, exact-erf GELU epilogue, bf16 output.
// Block tile 128 x 160 with four wave64s in a 2 x 2 arrangement, each wave
// owning a 64 x 80 sub-tile (4 x 5 MFMA tiles); operands are staged through
// LDS with the next tile's global loads issued before the current tile's
// MFMAs.  Tiles sharing the same rows of A are mapped to the same XCD so the
// A panel is fetched into that XCD's L2 once.
#include <cmath>

#include "df_internal.h"

namespace df {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = kGemmBM, BN = kGemmBN, BK = kGemmBK;
constexpr int LDK = BK + 8;  // LDS row stride in bf16 (80 bytes) to spread rows over banks
constexpr int kThreads = 256;
constexpr int WM = 64, WN = 80;          // per-wave sub-tile
constexpr int TM = WM / 16, TN = WN / 16;  // MFMA tiles per wave

// float -> bf16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ bf16_t to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16_t((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16_t(u >> 16);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

// d GELU / dx = Phi(x) + x phi(x)
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__device__ __forceinline__ float bf_to_f(bf16_t h) { return __uint_as_float(unsigned(h) << 16); }

// Epilogues: inference (bias, GELU); training forward (bias, GELU, and the pre-activation
// stored to P with C's layout); training backward (the product times GELU'(P), no bias).
enum { kEpiGelu = 0, kEpiLinear = 1, kEpiGeluSave = 2, kEpiGeluGrad = 3 };

template <int EPI>
__global__ __launch_bounds__(kThreads) void gemm_kernel(const bf16_t *__restrict__ A, int lda,
                                                       const bf16_t *__restrict__ B, int ldb,
                                                       const float *__restrict__ bias, bf16_t *__restrict__ C,
                                                       int ldc, int K, int n_tiles_n, bf16_t *__restrict__ P) {
    __shared__ __attribute__((aligned(16))) bf16_t As[BM * LDK];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[BN * LDK];

    // XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs, so
    // block b runs on XCD b % 8; give each XCD a contiguous range of logical tiles.
    const int nb = gridDim.x, b = blockIdx.x;
    const int logical = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int tile_m = logical / n_tiles_n, tile_n = logical % n_tiles_n;
    const int64_t row0 = int64_t(tile_m) * BM;
    const int col0 = tile_n * BN;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;

    // global -> register staging: A has BM*BK/8 = 512 16-byte chunks, B has 640
    constexpr int kAChunks = BM * BK / 8, kBChunks = BN * BK / 8;
    constexpr int kAPer = kAChunks / kThreads;                      // 2
    constexpr int kBPer = (kBChunks + kThreads - 1) / kThreads;     // 3
    u32x4 ra[kAPer], rb[kBPer];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < kAPer; ++i) {
            const int c = t + i * kThreads, r = c / (BK / 8), kc = c % (BK / 8);
            ra[i] = *reinterpret_cast<const u32x4 *>(A + (row0 + r) * lda + k0 + kc * 8);
        }
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int c = t + i * kThreads;
            if (c < kBChunks) {
                const int r = c / (BK / 8), kc = c % (BK / 8);
                rb[i] = *reinterpret_cast<const u32x4 *>(B + int64_t(col0 + r) * ldb + k0 + kc * 8);
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < kAPer; ++i) {
            const int c = t + i * kThreads, r = c / (BK / 8), kc = c % (BK / 8);
            *reinterpret_cast<u32x4 *>(As + r * LDK + kc * 8) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int c = t + i * kThreads;
            if (c < kBChunks) {
                const int r = c / (BK / 8), kc = c % (BK / 8);
                *reinterpret_cast<u32x4 *>(Bs + r * LDK + kc * 8) = rb[i];
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
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + BK < K) load(k0 + BK);
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
            af[i] = *reinterpret_cast<const bf16x8 *>(As + (wm * WM + i * 16 + fr) * LDK + fk);
#pragma unroll
        for (int j = 0; j < TN; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn * WN + j * 16 + fr) * LDK + fk);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }

    // epilogue: lane l holds column (l % 16) and rows 4 * (l / 16) + r of each 16 x 16 tile
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int col = col0 + wn * WN + j * 16 + fr;
        const float bc = (EPI == kEpiGeluGrad) ? 0.0f : bias[col];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wm * WM + i * 16 + (lane >> 4) * 4 + r;
                float v = acc[i][j][r] + bc;
                if (EPI == kEpiGeluSave) P[row * ldc + col] = to_bf16(v);
                if (EPI == kEpiGelu || EPI == kEpiGeluSave) v = gelu(v);
                if (EPI == kEpiGeluGrad) v *= gelu_grad(bf_to_f(P[row * ldc + col]));
                C[row * ldc + col] = to_bf16(v);
            }
        }
    }
}

}  // namespace

df_status launch_gemm_bf16(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C, int ldc,
                           int64_t M, int N, int K, bool gelu, hipStream_t stream) {
    return launch_gemm_bf16_epi(A, lda, B, ldb, bias, C, ldc, M, N, K, gelu ? GemmEpi::gelu : GemmEpi::linear, nullptr,
                                stream);
}

df_status launch_gemm_bf16_epi(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C,
                               int ldc, int64_t M, int N, int K, GemmEpi epi, bf16_t *P, hipStream_t stream) {
    if (M % BM || N % BN || K % BK || lda % 8 || ldb % 8)
        return fail(DF_E_INVALID, "gemm: shapes must be multiples of the tile sizes");
    if ((epi == GemmEpi::gelu_save || epi == GemmEpi::gelu_grad) && !P)
        return fail(DF_E_INVALID, "gemm: the epilogue needs the pre-activation array");
    if (M == 0) return DF_OK;
    const int64_t tiles = (M / BM) * (N / BN);
    if (tiles > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "gemm: too many tiles");
    const dim3 g = dim3(unsigned(tiles)), b = dim3(kThreads);
    switch (epi) {
        case GemmEpi::gelu:
            hipLaunchKernelGGL(gemm_kernel<kEpiGelu>, g, b, 0, stream, A, lda, B, ldb, bias, C, ldc, K, N / BN, P);
            break;
        case GemmEpi::linear:
            hipLaunchKernelGGL(gemm_kernel<kEpiLinear>, g, b, 0, stream, A, lda, B, ldb, bias, C, ldc, K, N / BN, P);
            break;
        case GemmEpi::gelu_save:
            hipLaunchKernelGGL(gemm_kernel<kEpiGeluSave>, g, b, 0, stream, A, lda, B, ldb, bias, C, ldc, K, N / BN, P);
            break;
        case GemmEpi::gelu_grad:
            hipLaunchKernelGGL(gemm_kernel<kEpiGeluGrad>, g, b, 0, stream, A, lda, B, ldb, bias, C, ldc, K, N / BN, P);
            break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("gemm launch: ") + hipGetErrorString(e));
    return DF_OK;
}

}  // namespace df
