// DNN form of the chemistry step (the paper's DNNInferencer::inference in three
// stages, Sec. "Description of the new classes"; network structure from Sec.
// "Chemistry Integration"):
//   1. pre   : x = (T, p, BoxCox(Y)), training-range test, z-score, bf16
//   2. layers: hidden layers as bf16 MFMA GEMMs with GELU (df_mlp.hip), output
//              layer on the matrix cores inside the post kernel; with FP8 precision the
//              layers between two hidden layers run on block-scaled E4M3FN operands (df_fp8.h)
//   3. post  : inverse normalisation and Box-Cox, optional renormalisation of Y,
//              T from enthalpy conservation at fixed p (FP64 Newton), rr
// Cells outside the training range are compacted into an index list and
// advanced by the integrator kernel in the same stream (status DNN_FALLBACK).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>

#include "df_fp8.h"
#include "df_internal.h"

namespace df {
namespace {

constexpr int kPreThreads = 256;

__device__ __forceinline__ bf16_t f2bf(float x) {
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16_t((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16_t(u >> 16);
}

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(unsigned(h) << 16); }

__device__ __forceinline__ double boxcox(double Y, double lam) { return (pow(fmax(Y, 0.0), lam) - 1.0) / lam; }

// x^n for 1 <= n by repeated squaring (the inverse Box-Cox power when 1/lambda is an integer)
__device__ __forceinline__ double ipow(double x, int n) {
    double r = 1.0;
    while (n) {
        if (n & 1) r *= x;
        x *= x;
        n >>= 1;
    }
    return r;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Normalised network inputs and flags: 1 = network, 0 = fallback (out of training range),
// 2 = non-finite input.  Cell i's row of in_pad bf16 inputs (zero beyond the K + 2 features, and
// for the padding rows i >= n) is written as 16-byte pieces.  The thread of cell 0 also clears
// the fallback counter, which the output kernel (a later launch) advances.
template <int K>
__global__ __launch_bounds__(kPreThreads) void pre_kernel(DnnDevParams prm, int64_t n, int64_t n_pad, int64_t ld,
                                                          const double *__restrict__ p, const double *__restrict__ T,
                                                          const double *__restrict__ Y, bf16_t *__restrict__ xb,
                                                          int in_pad, int8_t *__restrict__ flag,
                                                          int32_t *__restrict__ count,
                                                          int32_t *__restrict__ status, double *__restrict__ rr,
                                                          int fallback) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    if (i == 0) *count = 0;
    u32x4 *row = reinterpret_cast<u32x4 *>(xb + i * in_pad);
    if (i >= n) {
        for (int c = 0; c < in_pad / 8; ++c) row[c] = u32x4{0u, 0u, 0u, 0u};
        return;
    }
    constexpr int NI = K + 2;
    double x[NI];
    x[0] = T[i];
    x[1] = p[i];
    bool finite = isfinite(x[0]) && x[0] > 0.0 && isfinite(x[1]) && x[1] > 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double y = Y[k * ld + i];
        finite = finite && isfinite(y);
        x[2 + k] = boxcox(y, prm.lambda);
    }
    int f = 1;
    if (!finite) {
        f = 2;
    } else {
#pragma unroll
        for (int c = 0; c < NI; ++c)
            if (!(x[c] >= prm.lo[c] && x[c] <= prm.hi[c])) f = 0;
    }
    flag[i] = int8_t(f);
    unsigned xr[(NI + 1) / 2];
#pragma unroll
    for (int c = 0; c < NI; c += 2) {
        const double x0 = (x[c] - prm.mu_in[c]) / prm.sig_in[c];
        const unsigned b0 = (f == 1) ? unsigned(f2bf(float(x0))) : 0u;
        unsigned b1 = 0u;
        if (c + 1 < NI) {
            const double x1 = (x[c + 1] - prm.mu_in[c + 1]) / prm.sig_in[c + 1];
            b1 = (f == 1) ? unsigned(f2bf(float(x1))) : 0u;
        }
        xr[c / 2] = b0 | (b1 << 16);
    }
    constexpr int NQ = (NI + 7) / 8;  // 16-byte pieces holding features
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        u32x4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (4 * q + e < (NI + 1) / 2) ? xr[4 * q + e] : 0u;
        row[q] = v;
    }
    for (int q = NQ; q < in_pad / 8; ++q) row[q] = u32x4{0u, 0u, 0u, 0u};
    if (f != 1 && !(f == 0 && fallback)) {
        // non-finite input, or out of range with the fallback switched off: state left as is
        if (status) status[i] = (f == 2) ? DF_CELL_NONFINITE : DF_CELL_DNN_FALLBACK;
        if (rr)
            for (int k = 0; k < K; ++k) rr[k * ld + i] = 0.0;
    }
}

// output layer + stage 3.  The output layer u = W h (bf16 operands, fp32 sums) runs on the matrix
// cores as 16 x 16 x 32 MFMAs over groups of 64 consecutive cells, with the weight rows (zero
// beyond the K outputs) as the first operand, so that lane l ends with outputs 4 (l / 16) + r of
// cell l % 16 of each 16-cell tile; the products go through LDS to one lane per cell, which then
// runs stage 3 in FP64.  The activation rows are read as 16-byte fragments, 16 rows x 64
// contiguous bytes per load.  With at most 16 outputs (one output tile) the four waves of a block
// share one group of 64 cells and split the reduction, wave w taking the 32-deep steps w, w + 4,
// ...; their partial sums meet in LDS and are added in wave order, and wave 0 runs stage 3.  The
// chain of dependent load-and-product steps of a wave is then a quarter as long, and a launch has
// four times as many waves (65,536 cells: 4,096 instead of 1,024).  With more outputs each wave
// takes its own 64 cells: there stage 3 holds the most registers and the longest chain.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kPostThreads = 256;
template <int K>
constexpr int post_ksplit() { return (K + 15) / 16 == 1 ? 4 : 1; }
template <int K>
constexpr int post_cells_per_block() { return kPostThreads / post_ksplit<K>(); }

template <int K>
__global__ __launch_bounds__(kPostThreads) void post_kernel(DnnDevParams prm, MechDev m, int64_t n, int64_t ld,
                                                            double dt, const bf16_t *__restrict__ h, int h_ld,
                                                            const bf16_t *__restrict__ W, const float *__restrict__ b,
                                                            int k_in, const int8_t *__restrict__ flag,
                                                            const double *__restrict__ p, double *__restrict__ T,
                                                            double *__restrict__ Y, double *__restrict__ rr,
                                                            int32_t *__restrict__ status, int renormalise,
                                                            int32_t *__restrict__ idx, int32_t *__restrict__ count,
                                                            int fallback) {
    constexpr int NT = (K + 15) / 16;          // 16-output tiles
    constexpr int NP = (K % 2) ? K : K + 1;    // LDS row stride in floats (odd: conflict-free reads)
    constexpr int KS = post_ksplit<K>();       // waves sharing a group of 64 cells
    __shared__ float su[kPostThreads / 64][64 * NP];
    const int lane = int(threadIdx.x) & 63, wv = int(threadIdx.x) >> 6;
    const int fr = lane & 15, fg = lane >> 4;
    const int64_t cell0 = int64_t(blockIdx.x) * post_cells_per_block<K>() + (KS == 1 ? int64_t(wv) * 64 : 0);
    {
        floatx4 acc[4][NT];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        const bf16x8 zero = {};
        for (int k0 = (KS == 1 ? 0 : 32 * wv); k0 < k_in; k0 += 32 * KS) {
            bf16x8 wf[NT], hf[4];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int o = nt * 16 + fr;
                wf[nt] = (o < K) ? *reinterpret_cast<const bf16x8 *>(W + int64_t(o) * k_in + k0 + fg * 8) : zero;
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int64_t c = cell0 + mt * 16 + fr;
                hf[mt] = (c < n) ? *reinterpret_cast<const bf16x8 *>(h + c * h_ld + k0 + fg * 8) : zero;
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[nt], hf[mt], acc[mt][nt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = nt * 16 + fg * 4 + r;
                    if (o < K) su[wv][(mt * 16 + fr) * NP + o] = acc[mt][nt][r];
                }
    }
    __syncthreads();
    if (KS > 1 && wv > 0) return;  // wave 0 finishes the shared group
    const int64_t i = cell0 + lane;
    if (i >= n) return;
    const int fl = flag[i];
    if (fl != 1) {
        // the fallback list for the integrator's launch (its order does not change any cell's result)
        if (fl == 0 && fallback) idx[atomicAdd(count, 1)] = int32_t(i);
        return;
    }
    float u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        u[k] = su[wv][lane * NP + k];
#pragma unroll
        for (int w = 1; w < KS; ++w) u[k] += su[w][lane * NP + k];
    }
    // ---- stage 3, FP64
    const double T0 = T[i], iT0 = 1.0 / T0;
    // 1/lambda as an exact small integer (lambda = 0.1 gives 10): the power by squaring
    const int n_inv = (prm.inv_lambda == rint(prm.inv_lambda) && prm.inv_lambda >= 1.0 && prm.inv_lambda <= 64.0)
                          ? int(prm.inv_lambda)
                          : 0;
    double Y0[K], Yn[K];
    double sYW = 0.0, h0 = 0.0, sum = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        Y0[k] = Y[k * ld + i];
        const double *r = m.sp + k * kSpTab;
        sYW += Y0[k] * r[1];
        const double hRT = r[2] + T0 * (r[9] + T0 * (r[10] + T0 * (r[11] + T0 * r[12]))) + r[7] * iT0;
        h0 += Y0[k] * hRT * r[1];
        const double z1 = boxcox(Y0[k], prm.lambda) + (double(u[k] + b[k]) * prm.sig_out[k] + prm.mu_out[k]);
        // the base clamped at 0 from below; a NaN (a non-finite network output) stays NaN, so
        // that the cell's temperature recovery fails and it is flagged non-finite
        const double b1 = 1.0 + prm.lambda * z1;
        const double base = (b1 < 0.0) ? 0.0 : b1;
        Yn[k] = n_inv ? ipow(base, n_inv) : pow(base, prm.inv_lambda);
        sum += Yn[k];
    }
    h0 *= kR * T0;
    if (renormalise && sum > 0.0) {
        const double is = 1.0 / sum;
#pragma unroll
        for (int k = 0; k < K; ++k) Yn[k] *= is;
    }
    // T from h(T, Yn) = h0: Newton with dh/dT = cp
    double Tn = T0;
    bool conv = false;
    for (int it = 0; it < 20; ++it) {
        double hm = 0.0, cp = 0.0;
        const double iTn = 1.0 / Tn;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double *r = m.sp + k * kSpTab;
            const double cpR = r[2] + Tn * (r[3] + Tn * (r[4] + Tn * (r[5] + Tn * r[6])));
            const double hRT = r[2] + Tn * (r[9] + Tn * (r[10] + Tn * (r[11] + Tn * r[12]))) + r[7] * iTn;
            hm += Yn[k] * hRT * r[1];
            cp += Yn[k] * cpR * r[1];
        }
        const double dT = (hm * Tn - h0 / kR) / cp;
        Tn -= dT;
        if (!isfinite(Tn)) break;
        if (fabs(dT) <= 1e-9) {
            conv = true;
            break;
        }
    }
    if (rr) {
        const double rdt = p[i] / (sYW * kR * T0) / dt;
#pragma unroll
        for (int k = 0; k < K; ++k) rr[k * ld + i] = rdt * (Yn[k] - Y0[k]);
    }
    T[i] = Tn;
#pragma unroll
    for (int k = 0; k < K; ++k) Y[k * ld + i] = Yn[k];
    if (status) status[i] = conv ? DF_CELL_OK : DF_CELL_NONFINITE;
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

struct WsLayout {
    int64_t n_pad;
    size_t o_x, o_a, o_b, o_flag, o_idx, o_cnt, total;
    int wa, wb;  // widths of the two activation buffers
};

WsLayout workspace_layout(const df_dnn *d, int64_t n) {
    WsLayout w{};
    w.n_pad = round_up(std::max<int64_t>(n, 1), kGemmBM);
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const int nh = int(d->layers.size()) - 1;
    w.wa = w.wb = 0;
    for (int l = 0; l < nh; ++l) {
        if (l % 2 == 0)
            w.wa = std::max(w.wa, d->layers[l].n_pad);
        else
            w.wb = std::max(w.wb, d->layers[l].n_pad);
    }
    size_t o = 0;
    w.o_x = o;
    o = al(o + size_t(w.n_pad) * d->layers[0].k_pad * 2);
    w.o_a = o;
    o = al(o + size_t(w.n_pad) * w.wa * 2);
    w.o_b = o;
    o = al(o + size_t(w.n_pad) * w.wb * 2);
    w.o_flag = o;
    o = al(o + size_t(w.n_pad));
    w.o_idx = o;
    o = al(o + size_t(w.n_pad) * 4);
    w.o_cnt = o;
    o = al(o + 4);
    w.total = o;
    return w;
}

// Device blob of a network: per layer the bf16 weights [n_pad][k_pad] and fp32 biases [n_pad],
// the normalisation parameters, then per layer between two hidden layers the E4M3FN weights
// [n_pad][k_pad] and their row exponents [n_pad] (int32).  Offsets follow from the widths alone.
struct BlobLayout {
    std::vector<size_t> W, b, w8, e8;
    size_t prm = 0, total = 0;
};

BlobLayout blob_layout(const std::vector<DnnLayer> &layers, int n_in) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const int L = int(layers.size());
    BlobLayout bl;
    bl.W.assign(L, 0);
    bl.b.assign(L, 0);
    bl.w8.assign(L, 0);
    bl.e8.assign(L, 0);
    size_t o = 0;
    for (int l = 0; l < L; ++l) {
        bl.W[l] = o;
        o = al(o + size_t(layers[l].n_pad) * layers[l].k_pad * 2);
        bl.b[l] = o;
        o = al(o + size_t(layers[l].n_pad) * 4);
    }
    bl.prm = o;
    o = al(o + size_t(6) * n_in * 8);
    for (int l = 1; l + 1 < L; ++l) {
        bl.w8[l] = o;
        o = al(o + size_t(layers[l].n_pad) * layers[l].k_pad);
        bl.e8[l] = o;
        o = al(o + size_t(layers[l].n_pad) * 4);
    }
    bl.total = o;
    return bl;
}

// E4M3FN byte of v, |v| <= 448: round to nearest, ties to even; a non-finite v gives the
// format's NaN (the format has no infinity), so that it propagates as in the bf16 path
uint8_t e4m3_byte(float v) {
    const uint8_t sgn = std::signbit(v) ? 0x80 : 0x00;
    if (!std::isfinite(v)) return uint8_t(sgn | 0x7f);
    const float a = std::fabs(v);
    if (!(a > 0.0f)) return sgn;
    int k = 0;
    (void)std::frexp(a, &k);               // a = f 2^k, f in [0.5, 1): floor(log2 a) = k - 1
    int E = std::max(k - 1, -6);           // below 2^-6 the spacing stays 2^-9
    int m = int(std::nearbyint(std::ldexp(a, 3 - E)));  // a / 2^(E-3), exact before rounding
    if (E == -6 && m < 8) return uint8_t(sgn | m);     // subnormal
    if (m == 16) {
        m = 8;
        ++E;
    }
    return uint8_t(sgn | ((E + 7) << 3) | (m - 8));
}

template <int K>
df_status launch_dnn_k(const df_dnn *d, const df_mech *m, int64_t n, int64_t ld, double dt, const double *p,
                       double *T, double *Y, double *rr, int32_t *status, void *ws, const df_dnn_opts &o,
                       const df_chem_opts &fo, hipStream_t s) {
    const WsLayout w = workspace_layout(d, n);
    auto *base = static_cast<unsigned char *>(ws);
    auto *xb = reinterpret_cast<bf16_t *>(base + w.o_x);
    auto *ba = reinterpret_cast<bf16_t *>(base + w.o_a);
    auto *bb = reinterpret_cast<bf16_t *>(base + w.o_b);
    auto *flag = reinterpret_cast<int8_t *>(base + w.o_flag);
    auto *idx = reinterpret_cast<int32_t *>(base + w.o_idx);
    auto *cnt = reinterpret_cast<int32_t *>(base + w.o_cnt);
    const int in_pad = d->layers[0].k_pad;
    hipLaunchKernelGGL(pre_kernel<K>, dim3(unsigned((w.n_pad + kPreThreads - 1) / kPreThreads)), dim3(kPreThreads), 0,
                       s, d->prm, n, w.n_pad, ld, p, T, Y, xb, in_pad, flag, cnt, status, rr, o.fallback);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("dnn pre launch: ") + hipGetErrorString(e));
    // hidden layers
    const bf16_t *in = xb;
    int in_ld = in_pad;
    const int nh = int(d->layers.size()) - 1;
    const bool fp8 = (o.precision == 1);
    const BlobLayout bl = fp8 ? blob_layout(d->layers, d->prm.n_in) : BlobLayout{};
    auto *blob = static_cast<unsigned char *>(d->dev_blob);
    // FP8 input of the current layer (E4M3FN bytes and block scales), when its producer wrote one
    const uint8_t *a8 = nullptr, *a8s = nullptr;
    int a8_sst = 0;
    for (int l = 0; l < nh; ++l) {
        const DnnLayer &L = d->layers[l];
        bf16_t *out = (l % 2 == 0) ? ba : bb;
        const int out_ld = (l % 2 == 0) ? w.wa : w.wb;
        // layers 1..nh-1 (between two hidden layers) in FP8: each reads the E4M3FN copy of its
        // input (bytes and block scales), written by the layer before it (the first layer, whose
        // K is 32 or 64 for every compiled species count, or an FP8 layer).  An FP8 copy fills
        // the layer's activation buffer as bytes [n_pad][out_ld] followed by the scales
        // [n_pad][sst].
        const bool q_next = fp8 && l + 1 < nh;
        auto *o8 = reinterpret_cast<uint8_t *>(out);
        uint8_t *o8s = o8 + size_t(w.n_pad) * out_ld;
        const int o8_sst = fp8_scale_stride(out_ld);
        df_status st;
        bool wrote8 = false;
        if (fp8 && l >= 1) {
            if (!a8) return fail(DF_E_UNSUPPORTED, "dnn step: FP8 needs a first layer with 32 or 64 padded inputs");
            st = launch_gemm_fp8(a8, in_ld, a8s, a8_sst, blob + bl.w8[l], L.k_pad,
                                 reinterpret_cast<const int32_t *>(blob + bl.e8[l]), L.b, out, out_ld,
                                 q_next ? o8s : nullptr, o8_sst, w.n_pad, L.n_pad, L.k_pad, s);
            wrote8 = q_next;
        } else if (q_next) {
            st = launch_gemm_bf16_fp8out(in, in_ld, L.W, L.k_pad, L.b, o8, out_ld, o8s, o8_sst, w.n_pad, L.n_pad,
                                         L.k_pad, s);
            wrote8 = true;
        } else {
            st = launch_gemm_bf16(in, in_ld, L.W, L.k_pad, L.b, out, out_ld, w.n_pad, L.n_pad, L.k_pad, true, s);
        }
        if (st != DF_OK) return st;
        a8 = wrote8 ? o8 : nullptr;
        a8s = wrote8 ? o8s : nullptr;
        a8_sst = o8_sst;
        in = out;
        in_ld = out_ld;
    }
    const DnnLayer &Lo = d->layers.back();
    constexpr int kCpb = post_cells_per_block<K>();
    hipLaunchKernelGGL(post_kernel<K>, dim3(unsigned((n + kCpb - 1) / kCpb)), dim3(kPostThreads), 0, s,
                       d->prm, m->dev, n, ld, dt, in, in_ld, Lo.W, Lo.b, Lo.k_pad, flag, p, T, Y, rr, status,
                       o.renormalise, idx, cnt, o.fallback);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("dnn post launch: ") + hipGetErrorString(e));
    if (o.fallback) {
        const StepArgs a{n, ld, dt, nullptr, p, T, Y, nullptr, rr, status, nullptr, kernel_opts(fo),
                         DF_CELL_DNN_FALLBACK};
        return launch_chem_step(m->dev, a, fo.mapping, idx, cnt, s);
    }
    return DF_OK;
}

template <class T>
bool rd(std::ifstream &f, T *v, size_t n) {
    f.read(reinterpret_cast<char *>(v), std::streamsize(sizeof(T) * n));
    return bool(f);
}

}  // namespace
}  // namespace df

using namespace df;

extern "C" {

df_status df_dnn_load(const char *path, const df_mech *mech, int32_t device, df_dnn **out) {
    clear_error();
    if (!path || !mech || !out) return fail(DF_E_INVALID, "df_dnn_load: null path, mechanism or out");
    *out = nullptr;
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(DF_E_IO, std::string("cannot open DNN file ") + path);
    char magic[8];
    int32_t L = 0, K = 0, reserved = 0;
    if (!rd(f, magic, 8) || std::memcmp(magic, "DFDNN01", 7) != 0 || !rd(f, &L, 1) || L < 2 || L > 15)
        return fail(DF_E_FORMAT, std::string(path) + ": not a DFDNN01 file with 2..15 layers");
    std::vector<int32_t> dims(L + 1);
    double lam = 0, dtt = 0;
    if (!rd(f, dims.data(), dims.size()) || !rd(f, &K, 1) || !rd(f, &reserved, 1) || !rd(f, &lam, 1) ||
        !rd(f, &dtt, 1))
        return fail(DF_E_FORMAT, std::string(path) + ": truncated header");
    if (K != mech->host.K || dims[0] != K + 2 || dims[L] != K)
        return fail(DF_E_INVALID, "df_dnn_load: network widths do not match the mechanism's species count");
    for (int l = 0; l <= L; ++l)
        if (dims[l] < 1 || dims[l] > 65536) return fail(DF_E_FORMAT, "df_dnn_load: bad layer width");
    if (!(lam > 0) || !(dtt > 0)) return fail(DF_E_FORMAT, "df_dnn_load: lambda and dt_train must be > 0");
    const int ni = K + 2;
    std::vector<double> prm_h(size_t(6) * ni, 0.0);  // mu_in, sig_in, mu_out, sig_out, lo, hi
    for (int a = 0; a < 6; ++a) {
        const int cnt = (a == 2 || a == 3) ? K : ni;
        if (!rd(f, &prm_h[size_t(a) * ni], cnt)) return fail(DF_E_FORMAT, "df_dnn_load: truncated parameters");
    }
    for (int c = 0; c < ni; ++c)
        if (!(prm_h[size_t(ni) + c] > 0)) return fail(DF_E_FORMAT, "df_dnn_load: sig_in must be > 0");
    auto *d = new df_dnn;
    d->device = device;
    d->K = K;
    d->L = L;
    d->dims.assign(dims.begin(), dims.end());
    d->lambda = lam;
    d->dt_train = dtt;
    // padded device layout
    std::vector<std::vector<bf16_t>> Wh(L);
    std::vector<std::vector<float>> bh(L);
    int prev_pad = int(round_up(dims[0], kGemmBK));
    d->layers.resize(L);
    for (int l = 0; l < L; ++l) {
        DnnLayer &Ly = d->layers[l];
        Ly.n_in = dims[l];
        Ly.n_out = dims[l + 1];
        Ly.k_pad = prev_pad;
        Ly.n_pad = (l < L - 1) ? int(round_up(dims[l + 1], kGemmBN)) : dims[l + 1];
        std::vector<bf16_t> w(size_t(Ly.n_out) * Ly.n_in);
        std::vector<float> b(Ly.n_out);
        if (!rd(f, w.data(), w.size()) || !rd(f, b.data(), b.size())) {
            delete d;
            return fail(DF_E_FORMAT, std::string(path) + ": truncated weights");
        }
        Wh[l].assign(size_t(Ly.n_pad) * Ly.k_pad, 0);
        bh[l].assign(Ly.n_pad, 0.0f);
        for (int o = 0; o < Ly.n_out; ++o) {
            std::memcpy(&Wh[l][size_t(o) * Ly.k_pad], &w[size_t(o) * Ly.n_in], sizeof(bf16_t) * Ly.n_in);
            bh[l][o] = b[o];
        }
        prev_pad = Ly.n_pad;
    }
    // one device allocation
    const BlobLayout bl = blob_layout(d->layers, ni);
    const std::vector<size_t> &offW = bl.W, &offb = bl.b;
    const size_t offP = bl.prm, o = bl.total;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
        delete d;
        return fail(DF_E_HIP, "df_dnn_load: cannot select device");
    }
    void *blob = nullptr;
    hipError_t e = hipMalloc(&blob, o);
    if (e == hipSuccess) {
        std::vector<unsigned char> h(o, 0);
        for (int l = 0; l < L; ++l) {
            std::memcpy(h.data() + offW[l], Wh[l].data(), Wh[l].size() * 2);
            std::memcpy(h.data() + offb[l], bh[l].data(), bh[l].size() * 4);
        }
        std::memcpy(h.data() + offP, prm_h.data(), prm_h.size() * 8);
        // E4M3FN copies of the weights between two hidden layers, one power-of-two scale per row
        for (int l = 1; l + 1 < L; ++l) {
            const DnnLayer &Ly = d->layers[l];
            auto *e8 = reinterpret_cast<int32_t *>(h.data() + bl.e8[l]);
            for (int r = 0; r < Ly.n_pad; ++r) {
                const bf16_t *wr = &Wh[l][size_t(r) * Ly.k_pad];
                auto bf = [](bf16_t x) {
                    uint32_t u = uint32_t(x) << 16;
                    float f;
                    std::memcpy(&f, &u, 4);
                    return f;
                };
                float wmax = 0.0f;
                for (int c = 0; c < Ly.k_pad; ++c) wmax = std::max(wmax, std::fabs(bf(wr[c])));
                const int e = fp8_scale_exp(wmax);
                e8[r] = e;
                uint8_t *q = h.data() + bl.w8[l] + size_t(r) * Ly.k_pad;
                for (int c = 0; c < Ly.k_pad; ++c) q[c] = e4m3_byte(std::ldexp(bf(wr[c]), -e));
            }
        }
        e = hipMemcpy(blob, h.data(), o, hipMemcpyHostToDevice);
    }
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        if (blob) (void)hipFree(blob);
        delete d;
        return fail(DF_E_HIP, std::string("df_dnn_load: ") + hipGetErrorString(e));
    }
    d->dev_blob = blob;
    auto *base = static_cast<unsigned char *>(blob);
    for (int l = 0; l < L; ++l) {
        d->layers[l].W = reinterpret_cast<bf16_t *>(base + offW[l]);
        d->layers[l].b = reinterpret_cast<float *>(base + offb[l]);
    }
    const double *P = reinterpret_cast<const double *>(base + offP);
    d->prm = DnnDevParams{K, ni, lam, 1.0 / lam, P, P + ni, P + 2 * ni, P + 3 * ni, P + 4 * ni, P + 5 * ni};
    *out = d;
    return DF_OK;
}

void df_dnn_free(df_dnn *d) {
    if (!d) return;
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(d->device) == hipSuccess) {
        (void)hipFree(d->dev_blob);
        (void)hipSetDevice(prev);
    }
    delete d;
}

df_status df_dnn_info(const df_dnn *d, int32_t *n_layers, int32_t *dims, double *lambda, double *dt_train) {
    clear_error();
    if (!d) return fail(DF_E_INVALID, "df_dnn_info: null handle");
    if (n_layers) *n_layers = d->L;
    if (dims)
        for (int l = 0; l <= d->L; ++l) dims[l] = d->dims[l];
    if (lambda) *lambda = d->lambda;
    if (dt_train) *dt_train = d->dt_train;
    return DF_OK;
}

df_status df_dnn_workspace_size(const df_dnn *d, int64_t n_cells, size_t *bytes) {
    clear_error();
    if (!d || !bytes || n_cells < 0) return fail(DF_E_INVALID, "df_dnn_workspace_size: bad arguments");
    *bytes = workspace_layout(d, n_cells).total;
    return DF_OK;
}

#define DF_DNN_SPECIES_LIST(X) X(2) X(4) X(9) X(53)

df_status df_dnn_step(const df_dnn *d, const df_mech *m, int64_t n, int64_t ld, double dt, const double *p, double *T,
                      double *Y, double *rr, int32_t *status, void *ws, size_t ws_bytes, const df_dnn_opts *opts,
                      const df_chem_opts *fallback_opts, void *hip_stream) {
    clear_error();
    if (!d || !m) return fail(DF_E_INVALID, "df_dnn_step: null DNN or mechanism handle");
    if (d->K != m->host.K || d->device != m->device)
        return fail(DF_E_INVALID, "df_dnn_step: DNN and mechanism differ in species count or device");
    if (n < 0 || ld < n) return fail(DF_E_INVALID, "df_dnn_step: need 0 <= n_cells <= ld");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DF_E_INVALID, "df_dnn_step: dt must be finite and > 0");
    if (std::fabs(dt - d->dt_train) > 1e-12 * d->dt_train)
        return fail(DF_E_UNSUPPORTED, "df_dnn_step: dt differs from the time step the network was trained for");
    if (n > 0 && (!p || !T || !Y)) return fail(DF_E_INVALID, "df_dnn_step: null p, T or Y");
    if (n > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "df_dnn_step: more than 2^31-1 cells");
    df_dnn_opts o;
    df_dnn_default_opts(&o);
    if (opts) o = *opts;
    if ((o.renormalise != 0 && o.renormalise != 1) || (o.fallback != 0 && o.fallback != 1) ||
        (o.precision != 0 && o.precision != 1) || o.reserved1)
        return fail(DF_E_INVALID, "df_dnn_opts: renormalise, fallback and precision must be 0 or 1, reserved 0");
    df_chem_opts fo;
    df_chem_default_opts(&fo);
    if (fallback_opts) fo = *fallback_opts;
    df_status st = validate_chem_opts(fo);
    if (st != DF_OK) return st;
    if (n == 0) return DF_OK;
    const size_t need = workspace_layout(d, n).total;
    if (!ws || ws_bytes < need)
        return fail(DF_E_INVALID, "df_dnn_step: workspace missing or smaller than df_dnn_workspace_size");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(DF_E_INVALID, "df_dnn_step: workspace not 256-byte aligned");
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, "df_dnn_step: hipGetDevice failed");
    if (prev != d->device && hipSetDevice(d->device) != hipSuccess)
        return fail(DF_E_HIP, "df_dnn_step: cannot select the device");
    auto s = static_cast<hipStream_t>(hip_stream);
    switch (d->K) {
#define DF_CASE(k)                                                                \
    case k:                                                                       \
        st = launch_dnn_k<k>(d, m, n, ld, dt, p, T, Y, rr, status, ws, o, fo, s); \
        break;
        DF_DNN_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            st = fail(DF_E_UNSUPPORTED, "df_dnn_step: no compiled kernels for " + std::to_string(d->K) + " species");
    }
    if (prev != d->device) (void)hipSetDevice(prev);
    return st;
}

}  // extern "C"
