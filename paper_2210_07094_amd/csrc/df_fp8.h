// FP8 inference of the DNN form: the layers between two hidden layers run on the E4M3FN
// matrix cores of gfx950 (OCP 8-bit floating point: 4 exponent bits with bias 7, 3 mantissa
// bits, largest magnitude 448, no infinities).
//
// Scales are powers of two, so that applying and removing them is exact:
//  * activations: one scale 2^e per layer input over the whole call, e the smallest integer with
//    amax <= 448 * 2^e, where amax is the largest |value| over the rows of the call's cells
//    (the producing layer's epilogue reduces it into kAmaxSlots 32-bit words holding float bits,
//    wave w of block b into word (4 b + w) % kAmaxSlots, so that the atomics of a launch do not
//    queue on one address; the reading layer takes the max of the words);
//  * weights: one scale per output row, by the same rule over the row, quantised once at load.
// The products of the quantised values are summed in fp32 by the MFMA; the epilogue multiplies
// by 2^(e_a + e_w[col]), adds the bias, applies GELU and rounds to bf16.
#pragma once

#include <cstdint>

#include "df_internal.h"

namespace df {

constexpr int kAmaxSlots = 32;  // words of one activation maximum

// smallest e with amax <= 448 * 2^e for the float amax (0 for amax 0 or not finite); exact
__host__ __device__ inline int fp8_scale_exp(float amax) {
    if (!(amax > 0.0f) || !(amax <= 3.40282347e38f)) return 0;  // zero, NaN or infinite
    int k = 0;
    const float f = frexpf(amax, &k);  // amax = f * 2^k, f in [0.5, 1); 448 = 0.875 * 2^9
    return (f <= 0.875f) ? k - 9 : k - 8;
}

// The inference GEMM of launch_gemm_bf16 (GELU epilogue) that also reduces max |C| over rows
// < m_valid into amax[0..kAmaxSlots) (float bits, combined with atomicMax; the words must start
// at 0).
df_status launch_gemm_bf16_amax(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C,
                                int ldc, int64_t M, int N, int K, uint32_t *amax, int64_t m_valid,
                                hipStream_t stream);

// C[M][N] = GELU(2^(e_a + wexp[n]) * (Q(A 2^-e_a) . W8^T)[m][n] + bias[n]) in bf16, e_a from the
// max of amax_in[0..kAmaxSlots) (the scale rule above), Q the E4M3FN rounding (ties to even) of
// the bf16 activations.
// W8: [N][K] E4M3FN bytes (row stride ldb bytes), wexp: [N] row exponents.  amax_out (nullable):
// max |C| over rows < m_valid for the next FP8 layer.  Shapes as launch_gemm_bf16, ldb % 16 == 0.
df_status launch_gemm_fp8(const bf16_t *A, int lda, const uint32_t *amax_in, const uint8_t *W8, int ldb,
                          const int32_t *wexp, const float *bias, bf16_t *C, int ldc, int64_t M, int N, int K,
                          uint32_t *amax_out, int64_t m_valid, hipStream_t stream);

}  // namespace df
