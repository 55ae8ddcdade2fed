// Summary of a finished chemistry step (the outcome dfChemistryModel::solve() reports for the
// whole mesh, Sec. "Description of the new classes"): cells per status code, failed cells,
// sub-step totals and the costliest cell, and the smallest mass fraction written, reduced on the
// device from the per-cell outputs of df_chem_step / df_dnn_step.
//
// One grid-stride pass: each block reduces its cells in registers and LDS and merges into the
// caller's df_stats with one atomic per field; the costliest cell is kept as one 64-bit key
// (attempts in the high word, the complement of the index in the low word, so that the largest
// key is the lowest index among the largest counts) and the smallest Y as the order-preserving
// 64-bit image of its bits, both in the struct's own storage, turned into plain fields by a
// last one-thread kernel.
#include <cmath>
#include <cstddef>

#include "df_internal.h"

namespace df {
namespace {

constexpr int kStThreads = 256;
constexpr int kStBlocksMax = 1024;
constexpr int kStCodes = 8;

static_assert(offsetof(df_stats, max_attempts) % 8 == 0 && offsetof(df_stats, max_cell) == offsetof(df_stats, max_attempts) + 4,
              "max_attempts and max_cell share one 64-bit word during the reduction");
static_assert(sizeof(((df_stats *)nullptr)->count) == kStCodes * sizeof(int64_t), "one counter per status code");

// order-preserving unsigned image of a double (NaN excluded by the caller)
__device__ __forceinline__ unsigned long long ord_bits(double x) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ord(unsigned long long o) {
    const unsigned long long b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __longlong_as_double(static_cast<long long>(b));
}

__device__ __forceinline__ unsigned long long *key_word(df_stats *s) {
    return reinterpret_cast<unsigned long long *>(&s->max_attempts);
}
__device__ __forceinline__ unsigned long long *ymin_word(df_stats *s) {
    return reinterpret_cast<unsigned long long *>(&s->min_Y);
}

__global__ __launch_bounds__(kStThreads) void stats_zero(df_stats *s, int64_t n) {
    const int t = threadIdx.x;
    if (t < kStCodes) s->count[t] = 0;
    if (t == 0) {
        s->n_cells = n;
        s->failed = s->accepted = s->rejected = 0;
        *key_word(s) = 0ull;
        *ymin_word(s) = ord_bits(INFINITY);
    }
}

__global__ __launch_bounds__(kStThreads) void stats_reduce(int64_t n, int64_t ld, int K,
                                                           const int32_t *__restrict__ status,
                                                           const int32_t *__restrict__ nsteps,
                                                           const double *__restrict__ Y, df_stats *s) {
    __shared__ unsigned long long cnt[kStCodes + 3];  // per code, failed, accepted, rejected
    __shared__ unsigned long long key, ymin;
    const int t = threadIdx.x;
    if (t < kStCodes + 3) cnt[t] = 0ull;
    if (t == 0) {
        key = 0ull;
        ymin = ord_bits(INFINITY);
    }
    __syncthreads();
    unsigned long long acc = 0, rej = 0, fl = 0, k_loc = 0, y_loc = ord_bits(INFINITY);
    for (int64_t i = int64_t(blockIdx.x) * kStThreads + t; i < n; i += int64_t(gridDim.x) * kStThreads) {
        if (status) {
            const int32_t c = status[i];
            if (c >= 0 && c < kStCodes) atomicAdd(&cnt[c], 1ull);
            fl += (c == DF_CELL_MAX_STEPS || c == DF_CELL_H_UNDERFLOW || c == DF_CELL_NONFINITE ||
                   c == DF_CELL_TAPE_FULL)
                      ? 1ull
                      : 0ull;
        }
        if (nsteps) {
            const unsigned a = unsigned(nsteps[i]), r = unsigned(nsteps[n + i]);
            acc += a;
            rej += r;
            const unsigned long long kk = (static_cast<unsigned long long>(a + r) << 32) | (0xffffffffu - unsigned(i));
            k_loc = kk > k_loc ? kk : k_loc;
        }
        if (Y)
            for (int k = 0; k < K; ++k) {
                const double y = Y[int64_t(k) * ld + i];
                if (y == y) {
                    const unsigned long long o = ord_bits(y);
                    y_loc = o < y_loc ? o : y_loc;
                }
            }
    }
    if (fl) atomicAdd(&cnt[kStCodes], fl);
    if (acc) atomicAdd(&cnt[kStCodes + 1], acc);
    if (rej) atomicAdd(&cnt[kStCodes + 2], rej);
    if (nsteps) atomicMax(&key, k_loc);
    if (Y) atomicMin(&ymin, y_loc);
    __syncthreads();
    if (t < kStCodes && cnt[t]) atomicAdd(reinterpret_cast<unsigned long long *>(&s->count[t]), cnt[t]);
    if (t == kStCodes && cnt[t]) atomicAdd(reinterpret_cast<unsigned long long *>(&s->failed), cnt[t]);
    if (t == kStCodes + 1 && cnt[t]) atomicAdd(reinterpret_cast<unsigned long long *>(&s->accepted), cnt[t]);
    if (t == kStCodes + 2 && cnt[t]) atomicAdd(reinterpret_cast<unsigned long long *>(&s->rejected), cnt[t]);
    if (t == 0 && nsteps) atomicMax(key_word(s), key);
    if (t == 0 && Y) atomicMin(ymin_word(s), ymin);
}

__global__ void stats_finish(df_stats *s, int have_steps) {
    if (threadIdx.x != 0) return;
    const unsigned long long k = *key_word(s);
    const double ym = from_ord(*ymin_word(s));
    const bool any = have_steps && s->n_cells > 0;
    s->max_attempts = any ? int32_t(k >> 32) : 0;
    s->max_cell = any ? int32_t(0xffffffffu - unsigned(k & 0xffffffffull)) : -1;
    s->min_Y = ym;
}

}  // namespace
}  // namespace df

extern "C" df_status df_step_stats(int64_t n_cells, int64_t ld, int32_t n_species, const int32_t *cell_status,
                                   const int32_t *n_steps, const double *Y, df_stats *stats_dev, df_stats *stats_host,
                                   void *hip_stream) {
    using namespace df;
    clear_error();
    const char *who = "df_step_stats";
    if (!stats_dev) return fail(DF_E_INVALID, std::string(who) + ": null stats_dev");
    if (reinterpret_cast<uintptr_t>(stats_dev) % 8 != 0) return fail(DF_E_INVALID, std::string(who) + ": stats_dev not 8-byte aligned");
    if (n_cells < 0 || n_cells > 0x7fffffff) return fail(DF_E_INVALID, std::string(who) + ": need 0 <= n_cells < 2^31");
    if (Y && (n_species < 1 || ld < n_cells)) return fail(DF_E_INVALID, std::string(who) + ": Y needs n_species >= 1 and ld >= n_cells");
    auto s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(stats_zero, dim3(1), dim3(kStThreads), 0, s, stats_dev, n_cells);
    if (n_cells > 0) {
        int64_t blocks = (n_cells + kStThreads - 1) / kStThreads;
        blocks = blocks > kStBlocksMax ? kStBlocksMax : blocks;
        hipLaunchKernelGGL(stats_reduce, dim3(unsigned(blocks)), dim3(kStThreads), 0, s, n_cells, ld, int(n_species),
                           cell_status, n_steps, Y, stats_dev);
    }
    hipLaunchKernelGGL(stats_finish, dim3(1), dim3(64), 0, s, stats_dev, n_steps ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": launch: " + hipGetErrorString(e));
    if (!stats_host) return DF_OK;
    e = hipMemcpyAsync(stats_host, stats_dev, sizeof(df_stats), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": read: " + hipGetErrorString(e));
    return stats_host->failed > 0 ? DF_CELL_FAILURES : DF_OK;
}
