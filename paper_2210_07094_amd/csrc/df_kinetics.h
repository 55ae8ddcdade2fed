// Device-side pieces shared by the integrator kernels: the RODAS4 tableau, the
// integrator options and the forward rate constant (Arrhenius, Lindemann/Troe).
#pragma once

#include "df_internal.h"

namespace df {

// ---- RODAS4, transformed coefficients: (I/(g h) - J) u_i = f(y + sum a_ij u_j) + sum (c_ij/h) u_j
struct Rodas4 {
    static constexpr double g = 0.25;
    static constexpr double a[6][5] = {
        {0, 0, 0, 0, 0},
        {1.544, 0, 0, 0, 0},
        {0.9466785280815826, 0.2557011698983284, 0, 0, 0},
        {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0},
        {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0},
        {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0},
    };
    static constexpr double c[6][5] = {
        {0, 0, 0, 0, 0},
        {-5.6688, 0, 0, 0, 0},
        {-2.430093356833875, -0.2063599157091915, 0, 0, 0},
        {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0},
        {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0},
        {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136, -6.058818238834054},
    };
    // stage 6 starts from the embedded (order 3) solution; the order-4 solution adds u6,
    // so the error estimate is u6 itself.
};

constexpr double kInvLn10 = 0.43429448190325182765;
constexpr double kLn10 = 2.30258509299404568402;

// Reciprocal and quotient for normal finite divisors: the hardware reciprocal estimate refined
// by two Newton steps (each doubles the correct bits), and one residual correction of the
// quotient; within an ulp of the rounded result, at about half the instructions of the
// IEEE division sequence.  A zero or infinite divisor gives NaN.
__device__ __forceinline__ double frcp(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double fdiv(double a, double b) {
    const double r = frcp(b);
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}

// Natural logarithm for positive finite x, at about half the latency of the library call:
// x = 2^e m with m in [1/sqrt(2), sqrt(2)), ln m = 2 atanh(s) with s = (m - 1)/(m + 1), so
// |s| <= 0.1716 and the odd power series of atanh through s^21 leaves a truncation error
// below 2e-19 relative; e ln 2 is added in two parts (the high part has trailing zero bits,
// so e * kLn2Hi is exact).  Zero gives -inf, negative or NaN input NaN, +inf gives +inf.
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;

__device__ __forceinline__ double dlog(double x) {
    int e;
    double m = frexp(x, &e);
    const bool lo = m < 0.70710678118654752440;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const double s = fdiv(m - 1.0, m + 1.0);
    const double z = s * s;
    double q = 1.0 / 21;
    q = fma(q, z, 1.0 / 19);
    q = fma(q, z, 1.0 / 17);
    q = fma(q, z, 1.0 / 15);
    q = fma(q, z, 1.0 / 13);
    q = fma(q, z, 1.0 / 11);
    q = fma(q, z, 1.0 / 9);
    q = fma(q, z, 1.0 / 7);
    q = fma(q, z, 1.0 / 5);
    q = fma(q, z, 1.0 / 3);
    const double t = s + s;
    const double lm = fma(t * z, q, t);  // 2 s (1 + z/3 + z^2/5 + ...)
    const double de = double(e);
    double r = fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
    r = (x == 0.0) ? -INFINITY : r;
    r = (x > 0.0 || x == 0.0) ? r : NAN;
    r = (x == INFINITY) ? INFINITY : r;
    return r;
}

// claim from the front (+1) or the back (+2^32) of the queue; the cell index or -1
// Claims are ordered by the atomic: until the queue is exhausted every front claim is valid
// and the back claims are valid while t < tail_max, so the cells taken so far are
// h + min(t, tail_max); a claim takes the next cell while that is below n.
__device__ __forceinline__ int64_t queue_claim(const CellQueue &q, int64_t n, bool front) {
    const unsigned long long old = atomicAdd(q.ctr, front ? 1ull : (1ull << 32));
    const int64_t h = int64_t(old & 0xffffffffull), t = int64_t(old >> 32);
    const int64_t tm = int64_t(*q.tail_max);
    if (front) return (h + (t < tm ? t : tm) < n) ? int64_t(q.order[h]) : -1;
    return (t < tm && h + t < n) ? int64_t(q.order[n - 1 - t]) : -1;
}


// Forward rate constant of one reaction row (rd = ln A, b, Ta, ln A0, b0, Ta0, alpha,
// 1/T***, 1/T*, T**, ...): Arrhenius k = A T^b exp(-Ta/T); for Troe rows the
// Lindemann form k_inf Pr/(1+Pr) times the broadening factor F, Pr = k_0 [M]/k_inf.
// With DERIV also d ln kf/dT at fixed [M] and d kf/d[M].
template <bool DERIV>
__device__ __forceinline__ double rate_constant(const double *rd, int type, double T, double iT, double lT, double Mc,
                                                double &dlnkf, double &dkfdM) {
    const double kinf = exp(rd[0] + rd[1] * lT - rd[2] * iT);
    const double dlninf = (rd[1] + rd[2] * iT) * iT;
    if (type != 2) {
        if (DERIV) {
            dlnkf = dlninf;
            dkfdM = 0.0;
        }
        return kinf;
    }
    const double k0 = exp(rd[3] + rd[4] * lT - rd[5] * iT);
    const double al = rd[6], i3 = rd[7], i1 = rd[8], T2 = rd[9];
    const double e3 = exp(-T * i3), e1 = exp(-T * i1), e2 = exp(-T2 * iT);
    const double Fc = (1.0 - al) * e3 + al * e1 + e2;
    const double lFc = log(Fc) * kInvLn10;
    const double Pr = k0 * Mc / kinf;
    const double lPr = log(Pr) * kInvLn10;
    const double cc = -0.4 - 0.67 * lFc;
    const double nn = 0.75 - 1.27 * lFc;
    const double x = lPr + cc;
    const double iden = 1.0 / (nn - 0.14 * x);
    const double f1 = x * iden;
    const double q1 = 1.0 / (1.0 + f1 * f1);
    const double F = exp(lFc * q1 * kLn10);
    const double iPr1 = 1.0 / (1.0 + Pr);
    const double kf = kinf * Pr * iPr1 * F;
    if (DERIV) {
        const double dlnk0 = (rd[4] + rd[5] * iT) * iT;
        const double gq = 2.0 * f1 * q1 * q1;
        const double dlF_dlPr = -lFc * gq * nn * iden * iden;
        const double dlF_dlFc = q1 - lFc * gq * (1.27 * x - 0.67 * nn) * iden * iden;
        const double dFc = -(1.0 - al) * i3 * e3 - al * i1 * e1 + T2 * iT * iT * e2;
        const double dlFc_dT = dFc / Fc * kInvLn10;
        dlnkf = dlninf + (iPr1 + dlF_dlPr) * (dlnk0 - dlninf) + kLn10 * dlF_dlFc * dlFc_dT;
        dkfdM = k0 * F * iPr1 * (iPr1 + dlF_dlPr);
    }
    return kf;
}

// (p0/RT)^(-dnu) from p0/RT and its inverse: the reverse rate constant is kf / Kc with
// Kc = prod_k exp(-G_k/RT)^nu_k (p0/RT)^dnu in mol/cm^3 units
__device__ __forceinline__ double cref_pow(double cref, double icref, int dnu) {
    double r = 1.0;
    if (dnu > 0)
        for (int i = 0; i < dnu; ++i) r *= icref;
    else
        for (int i = 0; i < -dnu; ++i) r *= cref;
    return r;
}

}  // namespace df
