// FP8 inference of the DNN form: the layers between two hidden layers run on the E4M3FN
// matrix cores of gfx950 (OCP 8-bit floating point: 4 exponent bits with bias 7, 3 mantissa
// bits, largest magnitude 448, no infinities), as block-scaled products
// (v_mfma_scale_f32_16x16x128_f8f6f4).
//
// Scales are powers of two, so that applying and removing them is exact:
//  * activations: each row of a layer's input in blocks of 32 consecutive values, block q of row
//    i with the scale 2^e, e the smallest integer with max |block| <= 448 * 2^e (0 for a block of
//    zeros or one holding a non-finite value's maximum, at least -127), applied by the layer that
//    produces the activations to their bf16 values, which it writes as E4M3FN bytes [M][ld] and
//    E8M0 scale bytes (127 + e) [M][sst];
//  * weights: one scale per output row, by the same rule over the row, quantised once at load.
// The matrix cores take both scales with each 128-deep product and sum in fp32; the epilogue
// adds the bias, applies GELU and rounds to bf16.
#pragma once

#include <cstdint>

#include "df_internal.h"

namespace df {

constexpr int kFp8Block = 32;  // activations per block scale

// smallest e with amax <= 448 * 2^e for the float amax (0 for amax 0 or not finite), at least
// -127 (the smallest E8M0 scale); exact
__host__ __device__ inline int fp8_scale_exp(float amax) {
    if (!(amax > 0.0f) || !(amax <= 3.40282347e38f)) return 0;  // zero, NaN or infinite
    int k = 0;
    const float f = frexpf(amax, &k);  // amax = f * 2^k, f in [0.5, 1); 448 = 0.875 * 2^9
    const int e = (f <= 0.875f) ? k - 9 : k - 8;
    return e < -127 ? -127 : e;
}

// bytes per row of the scale array of an FP8 activation buffer of width ld (16-byte rows)
inline int fp8_scale_stride(int ld) { return (ld / kFp8Block + 15) / 16 * 16; }

// C[M][N] = GELU(sum_q 2^(e_a[m][q] + wexp[n]) (Q_a . W8^T over block q)[m][n] + bias[n]) in bf16,
// over the K (% 32 == 0) inputs in 128-deep steps (inputs from K to the next multiple of 128 read
// as zeros).  Q_a: [M][lda] E4M3FN bytes, S_a: [M][sst] E8M0 block scales of blocks 0 .. K/32 - 1;
// W8: [N][ldb] E4M3FN bytes, wexp: [N] row exponents (-127 .. 127).  M % 128 == 0, N % 160 == 0,
// lda, ldb multiples of 16, sst of 16.  With SC != nullptr the output is instead the FP8 copy the
// next FP8 layer reads: C holds E4M3FN bytes (row stride ldc bytes) and SC the block scales (row
// stride sstc), each value rounded to bf16 before it is quantised.
df_status launch_gemm_fp8(const uint8_t *A8, int lda, const uint8_t *S, int sst, const uint8_t *W8, int ldb,
                          const int32_t *wexp, const float *bias, bf16_t *C, int ldc, uint8_t *SC, int sstc,
                          int64_t M, int N, int K, hipStream_t stream);

// The first layer with an FP8 output: GELU(A . B^T + bias) as launch_gemm_bf16 for K = 32 or 64
// (DF_E_UNSUPPORTED otherwise), written as the FP8 copy (E4M3FN bytes Q[M][ldq], block scales
// S[M][sst]) of the bf16 values.
df_status launch_gemm_bf16_fp8out(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, uint8_t *Q,
                                  int ldq, uint8_t *S, int sst, int64_t M, int N, int K, hipStream_t stream);

}  // namespace df
