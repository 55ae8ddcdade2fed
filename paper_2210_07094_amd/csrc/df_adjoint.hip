// Discrete adjoint of the detailed-chemistry step on gfx950: eight lanes per cell, FP64.
//
// The step y0 = (T0, Y0) -> y(dt) is the sequence of accepted RODAS4 sub-steps of the taped
// forward integration (df_chem_step_taped), with the step lengths held fixed: the
// controller's choices are part of the sequence and are not differentiated.  One sub-step
// from y with length h is
//   W = I/(g h) - J(y),   Y_i = y + sum_{j<i} a_ij u_j,
//   W u_i = f(Y_i) + (1/h) sum_{j<i} c_ij u_j,   y_new = y + sum_i b_i u_i
// (b_i = a_5i for i < 5, b_5 = 1: the new state is the stage-6 state plus u_5).  The tape
// holds, per accepted sub-step, y, h, W^-1 and the six stage vectors u_i.  Given the adjoint
// lam of y_new, the reverse sweep over the sub-steps, last to first, sets
//   ubar_i = b_i lam,  ybar = lam;  for i = 5 .. 0:
//     rbar = W^-T ubar_i
//     v = J(Y_i)^T rbar:  ybar += v,  ubar_j += a_ij v + (c_ij / h) rbar   (j < i)
//     thbar += (df/dlnA)(Y_i)^T rbar
//     ybar += grad_y <rbar, J(y) u_i>,  thbar += grad_lnA <rbar, J(y) u_i>
//   lam = ybar
// The last line is the derivative of the iteration matrix: W depends on y through J.  The
// first-order products use the analytic Jacobian at the five stage states (formed in parallel,
// one stage per lane), so the sequential chain is a string of small matrix products.  The
// second-order terms are a vector-Jacobian product of f written out in reverse mode and
// evaluated in dual-number arithmetic at y + eps u_i, whose eps part is the directional
// derivative (a Hessian-vector product of <rbar, f>).  ln A is the natural log of the
// pre-exponential factor of each reaction, k_inf's for falloff rows.
#include <algorithm>
#include <cmath>

#include "df_internal.h"
#include "df_kinetics.h"
#include "df_lane.h"

namespace df {
namespace {

// columns of the equilibrium-constant rows the products read (the sweep's LDS copy keeps these)
constexpr int kAdjCr = 16;

// ---- dual numbers: value v and derivative d along one direction
struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, fma(a.v, b.d, a.d * b.v)}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual &operator+=(Dual &a, Dual b) { return a = a + b; }
__device__ __forceinline__ Dual &operator-=(Dual &a, Dual b) { return a = a - b; }
__device__ __forceinline__ Dual rcp(Dual a) {
    const double r = 1.0 / a.v;
    return {r, -a.d * r * r};
}
__device__ __forceinline__ double rcp(double a) { return 1.0 / a; }
__device__ __forceinline__ Dual sexp(Dual a) {
    const double e = exp(a.v);
    return {e, a.d * e};
}
__device__ __forceinline__ double sexp(double a) { return exp(a); }
__device__ __forceinline__ Dual slog(Dual a) { return {log(a.v), a.d / a.v}; }
__device__ __forceinline__ double slog(double a) { return log(a); }
template <class S>
__device__ __forceinline__ S mk(double v) {
    return S(v);
}
template <>
__device__ __forceinline__ Dual mk<Dual>(double v) {
    return Dual{v, 0.0};
}
// the part of a product accumulated into a gradient: the value for plain numbers; for duals the
// derivative, plus the value when the first-order term is wanted too
__device__ __forceinline__ double part(double x, bool) { return x; }
__device__ __forceinline__ double part(Dual x, bool with_value) { return with_value ? x.v + x.d : x.d; }

// LDS of one lane: element k of an array at base[k * kWave]
template <class S>
__device__ __forceinline__ S &at(S *base, int k) {
    return base[k * kWave];
}
// the concentration arrays of the products are laid out as one dual per lane and slot; the
// plain-number product uses the value half of its lane's slots (element k at base[k * 2 kWave])
template <class S>
__device__ __forceinline__ S &slot(S *base, int k) {
    return base[k * kWave * int(sizeof(Dual) / sizeof(S))];
}
// Per-species arrays of the products (the adjoint weights and the production rates) live in the
// lane's LDS rows (see rget()), plain numbers and duals alike: the registers go to the reaction
// loop's temporaries (in registers, both arrays spilled to scratch memory in the chain).
template <int K, class S>
struct SpArr {
    double *b;
    __device__ SpArr(double *base) : b(base) {}
    __device__ double get(int k) const { return b[k * kWave]; }
    __device__ void put(int k, double x) { b[k * kWave] = x; }
};
template <int K>
struct SpArr<K, Dual> {
    double *b;
    __device__ SpArr(double *base) : b(base) {}
    __device__ Dual get(int k) const;
    __device__ void put(int k, Dual x);
};
// arrays in the Cell region keep its layout, one double per lane in each wave-wide row: a plain
// number takes row k, a dual rows 2k (value) and 2k + 1 (derivative)
__device__ __forceinline__ double rget(const double *b, int k, double) { return b[k * kWave]; }
__device__ __forceinline__ Dual rget(const double *b, int k, Dual) { return {b[2 * k * kWave], b[(2 * k + 1) * kWave]}; }
__device__ __forceinline__ void rput(double *b, int k, double x) { b[k * kWave] = x; }
__device__ __forceinline__ void rput(double *b, int k, Dual x) {
    b[2 * k * kWave] = x.v;
    b[(2 * k + 1) * kWave] = x.d;
}
template <int K>
__device__ __forceinline__ Dual SpArr<K, Dual>::get(int k) const {
    return rget(b, k, Dual());
}
template <int K>
__device__ __forceinline__ void SpArr<K, Dual>::put(int k, Dual x) {
    rput(b, k, x);
}

// Reverse-mode product of lam with the Jacobian of f at y (the reactor right-hand side of
// Cell<K>::rhs): yb = J(y)^T lam, and for each reaction j (stored order)
// th[j] += part(lam . df/dlnA_j).  cs, cb: the lane's LDS slots (see slot()) of concentrations
// and their adjoints (N elements, element 0 the neutral slot); om, wd: the lane's rows (see
// rget()) of the adjoint weights of the production rates and the production rates (K
// elements); th: M doubles.
//   f_k = (1e6/rho) W_k wd_k,  f_T = -sum_k hm_k f_k / cp,  wd_k = sum_j nu_kj q_j,
//   q_j = Mq (kf prod c^nu' - kf/Kc prod c^nu''),  c_k = 1e-6 rho Y_k / W_k.
// The equilibrium constant and the reaction enthalpy come from the per-reaction coefficient
// rows over (1, ln T, 1/T, T, .., T^4), so no per-species thermo is live in the reaction loop.
template <int K, class S>
__device__ void vjp(const MechDev &m, double p, const S (&y)[K + 1], const double (&lam)[K + 1], S *cs, S *cb,
                    double *om, double *wd, double *th, bool with_value, S (&yb)[K + 1]) {
    const S T = y[0];
    const S iT = rcp(T);
    const S lT = slog(T);
    const S T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    auto cpR_of = [&](const double *r) { return r[2] + T * (r[3] + T * (r[4] + T * (r[5] + T * r[6]))); };
    auto hRT_of = [&](const double *r) {
        return r[2] + T * (r[9] + T * (r[10] + T * (r[11] + T * r[12]))) + r[7] * iT;
    };
    S sYW = mk<S>(0.0), cpm = mk<S>(0.0), dcpm = mk<S>(0.0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double *r = m.sp + k * kSpTab;
        sYW += y[1 + k] * r[1];
        cpm += y[1 + k] * cpR_of(r) * r[1];
        dcpm += y[1 + k] * (r[3] + T * (r[16] + T * (r[17] + T * r[18]))) * r[1];
    }
    const S Wbar = rcp(sYW);
    const S rho = (p / kR) * Wbar * iT;
    const S irho = rcp(rho);
    const S fy = 1e6 * irho;
    const S cp = kR * cpm;
    const S icp = rcp(cp);
    const S cfac = 1e-6 * rho;
    slot(cs, 0) = mk<S>(1.0);
    slot(cb, 0) = mk<S>(0.0);
    SpArr<K, S> oms(om), wds(wd);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double *r = m.sp + k * kSpTab;
        slot(cs, 1 + k) = cfac * y[1 + k] * r[1];
        slot(cb, 1 + k) = mk<S>(0.0);
        // adjoint weight of wd_k: (lam_k - lam_T hm_k / cp) (1e6/rho) W_k, hm_k = h_k/RT * R T / W_k
        const S hm = hRT_of(r) * T * (kR * r[1]);
        oms.put(k, (lam[1 + k] - lam[0] * hm * icp) * fy * r[0]);
        wds.put(k, mk<S>(0.0));
    }
    S cbd[K];
#pragma unroll
    for (int k = 0; k < K; ++k) cbd[k] = mk<S>(0.0);
    S Tb = mk<S>(0.0);
    // the species table entries read above are read again after the reaction loop rather than
    // kept live across it (compiler barrier)
    __asm__ volatile("" ::: "memory");
    for (int j = 0; j < m.M; ++j) {
        const int *ri = m.rx + j * kRxInt;
        const double *rd = m.rk + j * kRxDbl;
        const double *cr = m.cr + j * kAdjCr;
        const int type = ri[0];
        const int r0 = ri[1], r1 = ri[2], r2 = ri[3], p0 = ri[4], p1 = ri[5], p2 = ri[6], dnu = ri[7];
        const double *ef = m.eff + j * K;
        const int *nuj = m.nu + j * K;
        S Mc = mk<S>(0.0);
        if (type != 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) Mc += ef[k] * slot(cs, 1 + k);
        }
        // forward rate constant, d ln kf/dT at fixed [M], d kf/d[M], d ln kf/d ln A
        const S kinf = sexp(rd[0] + rd[1] * lT - rd[2] * iT);
        const S dlninf = (rd[1] + rd[2] * iT) * iT;
        S kf = kinf, dlnkf = dlninf, dkfdM = mk<S>(0.0), rA = mk<S>(1.0);
        if (type == 2) {
            const S k0 = sexp(rd[3] + rd[4] * lT - rd[5] * iT);
            const double al = rd[6], i3 = rd[7], i1 = rd[8], Tss = rd[9];
            const S e3 = sexp(-i3 * T), e1 = sexp(-i1 * T), e2 = sexp(-Tss * iT);
            const S Fc = (1.0 - al) * e3 + al * e1 + e2;
            const S lFc = kInvLn10 * slog(Fc);
            const S Pr = k0 * Mc * rcp(kinf);
            const S lPr = kInvLn10 * slog(Pr);
            const S cc = -0.4 - 0.67 * lFc;
            const S nn = 0.75 - 1.27 * lFc;
            const S x = lPr + cc;
            const S iden = rcp(nn - 0.14 * x);
            const S f1 = x * iden;
            const S q1 = rcp(1.0 + f1 * f1);
            const S F = sexp(kLn10 * (lFc * q1));
            const S iPr1 = rcp(1.0 + Pr);
            kf = kinf * Pr * iPr1 * F;
            const S dlnk0 = (rd[4] + rd[5] * iT) * iT;
            const S gq = 2.0 * f1 * q1 * q1;
            const S dlF_dlPr = -1.0 * (lFc * gq * nn * iden * iden);
            const S dlF_dlFc = q1 - lFc * gq * (1.27 * x - 0.67 * nn) * iden * iden;
            const S dFc = -(1.0 - al) * i3 * e3 - al * i1 * e1 + Tss * iT * iT * e2;
            const S dlFc_dT = kInvLn10 * (dFc * rcp(Fc));
            dlnkf = dlninf + (iPr1 + dlF_dlPr) * (dlnk0 - dlninf) + kLn10 * (dlF_dlFc * dlFc_dT);
            dkfdM = k0 * F * iPr1 * (iPr1 + dlF_dlPr);
            rA = 1.0 - iPr1 - dlF_dlPr;
        }
        // 1/Kc = k_r / k_f from the rows of ln k_r and ln k_f; d ln Kc/dT = (sum nu H/RT - dnu)/T
        const S iKc = sexp((cr[3] - cr[0]) + (cr[4] - cr[1]) * lT + (cr[5] - cr[2]) * iT + cr[6] * T + cr[7] * T2 +
                           cr[8] * T3 + cr[9] * T4);
        const S dlnKc = (cr[10] + cr[11] * T + cr[12] * T2 + cr[13] * T3 + cr[14] * T4 + cr[15] * iT - double(dnu)) * iT;
        S Qb = mk<S>(0.0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int nk = nuj[k];
            if (nk != 0) Qb += double(nk) * oms.get(k);  // wave-uniform branch
        }
        const S kr = kf * iKc;
        const S c0 = slot(cs, r0), c1 = slot(cs, r1), c2 = slot(cs, r2);
        const S d0 = slot(cs, p0), d1 = slot(cs, p1), d2 = slot(cs, p2);
        const S Pf = c0 * c1 * c2, Pb = d0 * d1 * d2;
        const S fwd = kf * Pf, rev = kr * Pb, X = fwd - rev;
        const S Mq = (type == 1) ? Mc : mk<S>(1.0);
        const S q = Mq * X;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int nk = nuj[k];
            if (nk != 0) wds.put(k, wds.get(k) + double(nk) * q);
        }
        // adjoint of q_j: T at fixed c, the concentrations of its slots, [M], ln A
        Tb += Qb * Mq * (fwd * dlnkf - rev * (dlnkf - dlnKc));
        const S af = Qb * Mq * kf, ar = Qb * Mq * kr;
        slot(cb, r0) += af * c1 * c2;
        slot(cb, r1) += af * c0 * c2;
        slot(cb, r2) += af * c0 * c1;
        slot(cb, p0) -= ar * d1 * d2;
        slot(cb, p1) -= ar * d0 * d2;
        slot(cb, p2) -= ar * d0 * d1;
        if (type != 0) {
            const S G = Qb * ((type == 1) ? X : dkfdM * (Pf - Pb * iKc));
#pragma unroll
            for (int k = 0; k < K; ++k) cbd[k] += G * ef[k];
        }
        at(th, j) += part(Qb * q * rA, with_value);
    }
    __asm__ volatile("" ::: "memory");
    // mixture: f_k, f_T and the adjoints of fy, hm_k, cp, rho
    S fyb = mk<S>(0.0), H = mk<S>(0.0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double *r = m.sp + k * kSpTab;
        const S hm = hRT_of(r) * T * (kR * r[1]);
        const S wk = wds.get(k);
        H += hm * (fy * r[0] * wk);
        fyb += (lam[1 + k] - lam[0] * hm * icp) * r[0] * wk;
    }
    const S fT = -1.0 * (H * icp);
    const S cpb = -lam[0] * fT * icp;
    S rhob = -1.0 * (fyb * fy * irho);
    S T_hm = mk<S>(0.0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double *r = m.sp + k * kSpTab;
        const S cbk = slot(cb, 1 + k) + cbd[k];
        cbd[k] = cbk;
        rhob += cbk * slot(cs, 1 + k) * irho;
        const S fk = fy * r[0] * wds.get(k);
        T_hm += (-lam[0] * fk * icp) * cpR_of(r) * (kR * r[1]);  // hm_k' = cp_k (mass)
    }
    yb[0] = Tb + T_hm + cpb * (kR * dcpm) - rhob * rho * iT;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double *r = m.sp + k * kSpTab;
        yb[1 + k] = (cbd[k] * cfac + cpb * kR * cpR_of(r) - rhob * rho * Wbar) * r[1];
    }
}

struct AdjArgs {
    int64_t n, ld;
    const double *p;
    const double *tape;
    int32_t cap;
    const double *Tb, *Yb;   // seeds, [n] and [K][ld]
    double *T0b, *Y0b;       // [n], [K][ld]
    double *thc;             // [M][ld] per-cell ln A adjoints in file order, or nullptr
    double *wth;             // [M][n] per-cell ln A adjoints in stored order (for the sum)
};

constexpr int kAdjLanes = 8;                  // lanes per cell
constexpr int kAdjCells = kWave / kAdjLanes;  // cells per block (one wave)

// Per-block LDS of the sweep, in doubles.  Per lane, rows of one double per lane (element k at
// base[k * kWave]): a work area of P = max(4N + 4K, 5N + M) rows, then the ln A adjoints (M).
// The work area holds, at different times of a sub-step, the analytic Jacobian's thermo and
// scatter rows (5N) with the per-reaction ln A factors after them (M), and the products' dual
// concentrations and their adjoints (4N) with the production-rate weights and rates (4K).  Per
// cell: the stage adjoints ubar (6N; after the chain, the second-order parts of the six
// stages), the transposed products' results rbar (6N), the state adjoint (N), the product
// J^T rbar (N) and the sub-step's tape record (N^2 + 7N).  Then a copy of the mechanism tables
// the reaction loops read (species rows, reaction rows, third-body efficiencies, the first
// kAdjCr columns of the equilibrium rows, stoichiometry): read with wave-uniform addresses,
// they are broadcast LDS reads instead of memory loads on the loops' dependency chains.
template <int K>
struct AdjLds {
    static constexpr int N = K + 1;
    static constexpr int kTapeRec = N * N + 7 * N;  // a sub-step's W^-1, y and six stage vectors
    static constexpr int kCell = 14 * N + kTapeRec;
    __host__ __device__ static int work_rows(int M) { return 4 * N + 4 * K > 5 * N + M ? 4 * N + 4 * K : 5 * N + M; }
    // doubles of the per-lane rows and the cell regions (the mechanism copy follows them)
    __host__ __device__ static int front(int M) { return kWave * (work_rows(M) + M) + kAdjCells * kCell; }
};

// One cell per group of 8 lanes.  Per sub-step, last to first:
//  1. the lanes stage the sub-step's tape record in LDS;
//  2. lanes 0..4 form J(Y_i) of stages i = 1..5 with the analytic Jacobian (lane i - 1 keeps its
//     stage's Jacobian in registers), with the factors of df/dlnA;
//  3. the chain, stage 5 to 0: rbar_i = W^-T ubar_i with the eight lanes taking the columns,
//     v = J(Y_i)^T rbar_i on the lane that holds J(Y_i), and the ubar and ybar updates with the
//     lanes taking the species;
//  4. lanes 0..4 add (df/dlnA)(Y_i)^T rbar_i to the ln A adjoints;
//  5. lanes 0..5 each take one stage's second-order term (the dual product at y + eps u_i);
//     every lane adds them up into the new lam.
template <int K>
__global__ __launch_bounds__(kWave) void adjoint_kernel(MechDev m, AdjArgs a) {
    constexpr int N = K + 1;
    extern __shared__ double lds[];
    const int lane = threadIdx.x, r = lane % kAdjLanes, g = lane / kAdjLanes;
    const int P = AdjLds<K>::work_rows(m.M);
    Dual *cs = reinterpret_cast<Dual *>(lds) + lane;
    Dual *cb = cs + N * kWave;
    double *omr = lds + 4 * N * kWave + lane, *wdr = omr + 2 * K * kWave;
    double *shr = lds + lane;                 // the Jacobian's rows
    double *lnar = lds + 5 * N * kWave + lane;  // its ln A factors
    double *th = lds + P * kWave + lane;
    double *cell = lds + (P + m.M) * kWave + g * AdjLds<K>::kCell;
    double *ub = cell, *rbs = cell + 6 * N, *yba = cell + 12 * N, *vt = cell + 13 * N;
    double *ybp = ub;  // the stage adjoints are dead once the chain is done
    double *tw = cell + 14 * N, *ty = tw + N * N, *tu = ty + N;  // the sub-step's tape record
    // the mechanism copy: doubles (species, reaction rows, efficiencies, equilibrium rows), then ints
    MechDev ml = m;
    {
        double *md = lds + AdjLds<K>::front(m.M);
        double *lsp = md, *lrk = lsp + K * kSpTab, *leff = lrk + m.M * kRxDbl, *lcr = leff + m.M * K;
        int *lrx = reinterpret_cast<int *>(lcr + m.M * kAdjCr), *lnu = lrx + m.M * kRxInt;
        for (int e = lane; e < K * kSpTab; e += kWave) lsp[e] = m.sp[e];
        for (int e = lane; e < m.M * kRxDbl; e += kWave) lrk[e] = m.rk[e];
        for (int e = lane; e < m.M * K; e += kWave) leff[e] = m.eff[e];
        for (int e = lane; e < m.M * kAdjCr; e += kWave) lcr[e] = m.cr[(e / kAdjCr) * kCrDbl + e % kAdjCr];
        for (int e = lane; e < m.M * kRxInt; e += kWave) lrx[e] = m.rx[e];
        for (int e = lane; e < m.M * K; e += kWave) lnu[e] = m.nu[e];
        ml.sp = lsp;
        ml.rk = lrk;
        ml.eff = leff;
        ml.cr = lcr;
        ml.rx = lrx;
        ml.nu = lnu;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const int64_t i = int64_t(blockIdx.x) * kAdjCells + g;
    if (i >= a.n) return;  // the lanes of a cell leave together
    const int64_t ld = a.ld;
    const Tape tp(K, a.n, a.cap);
    const int32_t cnt = tp.count(a.tape)[i];
    const double *T = a.tape + i;
    double lam[N];
    lam[0] = a.Tb[i];
#pragma unroll
    for (int k = 0; k < K; ++k) lam[1 + k] = a.Yb[k * ld + i];
    for (int j = 0; j < m.M; ++j) at(th, j) = 0.0;
    const double p = a.p[i];
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // the species (or columns) of the lane in the spread phases: r and r + 8
    constexpr int kSpread = (N + kAdjLanes - 1) / kAdjLanes;
    constexpr int kRec = AdjLds<K>::kTapeRec, kPer = (kRec + kAdjLanes - 1) / kAdjLanes;
    for (int64_t s = int64_t(cnt > 0 ? cnt : 0) - 1; s >= 0; --s) {
        // 1. the cell's 8 lanes stage the sub-step's tape record with all loads in flight together
        {
            double v[kPer];
#pragma unroll
            for (int t = 0; t < kPer; ++t) {
                const int e = r + kAdjLanes * t;
                v[t] = (e < N * N) ? T[tp.w(s, e)] : (e < N * N + N) ? T[tp.y(s, e - N * N)]
                                                   : (e < kRec) ? T[tp.u(s, e - N * N - N)] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < kPer; ++t) {
                const int e = r + kAdjLanes * t;
                if (e < kRec) tw[e] = v[t];
            }
        }
        const double ih = 1.0 / T[tp.h(s)];
        wave_sync();
        // ubar_i = b_i lam, ybar = lam (the lanes take species r, r + 8); lam is dead from here
        // until the sub-step's end, while the stage Jacobians take the registers
#pragma unroll
        for (int t = 0; t < kSpread; ++t) {
            const int k = r + kAdjLanes * t;
            if (k < N) {
                double lk = lam[0];
#pragma unroll
                for (int kk = 1; kk < N; ++kk) lk = (k == kk) ? lam[kk] : lk;
                yba[k] = lk;
#pragma unroll
                for (int si = 0; si < 6; ++si) ub[si * N + k] = (si < 5 ? Rodas4::a[5][si] : 1.0) * lk;
            }
        }
        // 2. lane r < 5: J at the state of stage r + 1, Y = y + sum_{j < r+1} a_{r+1,j} u_j (y and
        //    the u_j read from the staged record)
        double J[N][N], mix[2];
        if (r < 5) {
            const int si = r + 1;
            double ys[N], f[N];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double w = ty[k];
#pragma unroll
                for (int jj = 0; jj < 5; ++jj) w = fma(Rodas4::a[si][jj], tu[jj * N + k], w);  // a_ij = 0 for j >= i
                ys[k] = w;
            }
            Cell<K>::init_lds(shr);
            Cell<K>::template jacobian<true>(ml, p, ys, shr, J, f, lnar, mix);
        }
        wave_sync();
        // 3. the chain
#pragma unroll 1
        for (int si = 5; si >= 0; --si) {
            // rbar = W^-T ubar_i: lane r takes columns r, r + 8
#pragma unroll
            for (int t = 0; t < kSpread; ++t) {
                const int c = r + kAdjLanes * t;
                if (c < N) {
                    double acc = 0.0;
#pragma unroll
                    for (int q = 0; q < N; ++q) acc = fma(tw[q * N + c], ub[si * N + q], acc);
                    rbs[si * N + c] = acc;
                }
            }
            wave_sync();
            if (si > 0) {
                // v = J(Y_i)^T rbar on lane i - 1
                if (r == si - 1) {
                    double rb[N];
#pragma unroll
                    for (int k = 0; k < N; ++k) rb[k] = rbs[si * N + k];
#pragma unroll
                    for (int l = 0; l < N; ++l) {
                        double acc = 0.0;
#pragma unroll
                        for (int k = 0; k < N; ++k) acc = fma(J[k][l], rb[k], acc);
                        vt[l] = acc;
                    }
                }
                wave_sync();
                // ybar += v;  ubar_j += a_ij v + (c_ij / h) rbar  (j < i)
#pragma unroll
                for (int t = 0; t < kSpread; ++t) {
                    const int k = r + kAdjLanes * t;
                    if (k < N) {
                        const double vk = vt[k], rk = rbs[si * N + k];
                        yba[k] += vk;
                        for (int jj = 0; jj < si; ++jj)
                            ub[jj * N + k] += Rodas4::a[si][jj] * vk + Rodas4::c[si][jj] * ih * rk;
                    }
                }
                wave_sync();
            }
        }
        // 4. lane r < 5: the first-order ln A terms of stage r + 1, lnA_bar_j += Qb_j q_j dlnkf_j/dlnA_j
        //    with Qb_j = sum_k nu_kj om_k, om_k = fy W_k rbar_k - (fy R T / cp) (H_k/RT) rbar_T (the
        //    H/RT rows of the stage state are still in the lane's Jacobian rows)
        if (r < 5) {
            const int si = r + 1;
            double om[K];
            const double rT = rbs[si * N] * mix[1];
#pragma unroll
            for (int k = 0; k < K; ++k)
                om[k] = mix[0] * ml.sp[k * kSpTab] * rbs[si * N + 1 + k] - rT * at(shr, Cell<K>::kH + 1 + k);
            for (int j = 0; j < m.M; ++j) {
                const int *nuj = ml.nu + j * K;
                double Qb = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int nk = nuj[k];
                    if (nk != 0) Qb = fma(double(nk), om[k], Qb);  // wave-uniform branch
                }
                at(th, j) = fma(Qb, at(lnar, j), at(th, j));
            }
        }
        // 5. derivative of W through J(y): the dual product at y + eps u_i with seed rbar_i (stage 0
        //    also takes the first-order term J(y)^T rbar_0, the value part)
        if (r < 6) {
            Dual yd[N], vd[N];
            double rb[N];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                yd[k] = Dual{ty[k], tu[r * N + k]};
                rb[k] = rbs[r * N + k];
            }
            vjp<K, Dual>(ml, p, yd, rb, cs, cb, omr, wdr, th, r == 0, vd);
#pragma unroll
            for (int k = 0; k < N; ++k) ybp[r * N + k] = (r == 0) ? vd[k].v + vd[k].d : vd[k].d;
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double v = yba[k];
#pragma unroll
            for (int q = 0; q < 6; ++q) v += ybp[q * N + k];
            lam[k] = v;
        }
        wave_sync();
    }
    const bool ok = cnt > 0;
    if (r == 0) {
        a.T0b[i] = ok ? lam[0] : 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) a.Y0b[k * ld + i] = ok ? lam[1 + k] : 0.0;
    }
    // ln A adjoints: the six lanes' partial sums; lane r takes reactions r, r + 8, ...
    for (int j = r; j < m.M; j += kAdjLanes) {
        double v = 0.0;
        for (int q = 0; q < 6; ++q) v += lds[(P + j) * kWave + g * kAdjLanes + q];
        v = ok ? v : 0.0;
        a.wth[int64_t(j) * a.n + i] = v;
        if (a.thc) a.thc[int64_t(m.src[j]) * ld + i] = v;
    }
}

// lnA_bar[src[j]] = sum over cells of the per-cell adjoints of stored reaction j: one block per
// reaction, a fixed-order tree over a fixed-stride partition (deterministic)
__global__ __launch_bounds__(256) void sum_cells_kernel(const double *__restrict__ wth, int64_t n,
                                                        const int *__restrict__ src, double *__restrict__ out) {
    extern __shared__ double part_sum[];  // 256 doubles
    const int j = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < n; i += 256) s += wth[int64_t(j) * n + i];
    part_sum[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part_sum[t] += part_sum[t + w];
        __syncthreads();
    }
    if (t == 0) out[src[j]] = part_sum[0];
}

size_t adj_ws_bytes(int, int M, int64_t n) { return size_t(8) * size_t(M) * size_t(n); }

size_t adj_lds_bytes(int K, int M) {
    const size_t N = size_t(K + 1), Ms = size_t(M), Ks = size_t(K);
    const size_t P = std::max(4 * N + 4 * Ks, 5 * N + Ms);
    const size_t front = size_t(kWave) * (P + Ms) + size_t(kAdjCells) * (21 * N + N * N);
    const size_t mech_dbl = Ks * kSpTab + Ms * (kRxDbl + Ks + kAdjCr), mech_int = Ms * (kRxInt + Ks);
    return size_t(8) * (front + mech_dbl) + size_t(4) * mech_int;
}

constexpr size_t kAdjLdsMax = 80 * 1024;  // two blocks (waves) per CU

template <int K>
df_status launch_adjoint_k(const MechDev &m, const AdjArgs &a, hipStream_t s) {
    const int64_t blocks = (a.n + kAdjCells - 1) / kAdjCells;
    const size_t lds = adj_lds_bytes(K, m.M);
    if (lds > 64 * 1024) {
        const hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void *>(adjoint_kernel<K>),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (ea != hipSuccess)
            return fail(DF_E_HIP, std::string("df_chem_adjoint: LDS size: ") + hipGetErrorString(ea));
    }
    hipLaunchKernelGGL(adjoint_kernel<K>, dim3(unsigned(blocks)), dim3(kWave), lds, s, m, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("df_chem_adjoint launch: ") + hipGetErrorString(e));
    return DF_OK;
}

// species counts with a compiled adjoint kernel
#define DF_ADJ_SPECIES_LIST(X) X(2) X(4) X(9)

bool adjoint_supported(const MechDev &m) {
    bool k_ok = false;
#define DF_CASE(k) k_ok = k_ok || m.K == k;
    DF_ADJ_SPECIES_LIST(DF_CASE)
#undef DF_CASE
    return k_ok && adj_lds_bytes(m.K, m.M) <= kAdjLdsMax && chem_coop_supported(m);
}

struct DeviceScope {
    int prev = 0;
    bool changed = false;
    df_status st = DF_OK;
    DeviceScope(int dev, const char *who) {
        if (hipGetDevice(&prev) != hipSuccess) {
            st = fail(DF_E_HIP, std::string(who) + ": hipGetDevice failed");
            return;
        }
        if (prev != dev) {
            if (hipSetDevice(dev) != hipSuccess) {
                st = fail(DF_E_HIP, std::string(who) + ": cannot select the mechanism's device");
                return;
            }
            changed = true;
        }
    }
    ~DeviceScope() {
        if (changed) (void)hipSetDevice(prev);
    }
};

}  // namespace
}  // namespace df

extern "C" df_status df_chem_tape_size(const df_mech *mech, int64_t n_cells, int32_t max_substeps, size_t *bytes) {
    using namespace df;
    clear_error();
    if (!mech || !bytes || n_cells < 0 || max_substeps < 1)
        return fail(DF_E_INVALID, "df_chem_tape_size: bad arguments");
    *bytes = tape_bytes(mech->host.K, n_cells, max_substeps);
    return DF_OK;
}

extern "C" df_status df_chem_step_taped(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *p,
                                        double *T, double *Y, int32_t *cell_status, int32_t *n_steps, void *tape,
                                        size_t tape_size, int32_t max_substeps, const df_chem_opts *opts,
                                        void *hip_stream) {
    using namespace df;
    clear_error();
    const char *who = "df_chem_step_taped";
    if (!mech) return fail(DF_E_INVALID, std::string(who) + ": null mechanism handle");
    if (n_cells < 0 || ld < n_cells) return fail(DF_E_INVALID, std::string(who) + ": need 0 <= n_cells <= ld");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DF_E_INVALID, std::string(who) + ": dt must be finite and > 0");
    if (max_substeps < 1) return fail(DF_E_INVALID, std::string(who) + ": max_substeps must be >= 1");
    if (n_cells > 0 && (!p || !T || !Y || !tape)) return fail(DF_E_INVALID, std::string(who) + ": null p, T, Y or tape");
    if (n_cells > 0x7fffffff) return fail(DF_E_UNSUPPORTED, std::string(who) + ": more than 2^31-1 cells");
    if (n_cells > 0 && (tape_size < tape_bytes(mech->host.K, n_cells, max_substeps) ||
                        reinterpret_cast<uintptr_t>(tape) % 256 != 0))
        return fail(DF_E_INVALID, std::string(who) + ": tape smaller than df_chem_tape_size or not 256-byte aligned");
    if (!adjoint_supported(mech->dev))
        return fail(DF_E_UNSUPPORTED, std::string(who) + ": no adjoint kernel for this mechanism");
    df_chem_opts o;
    df_chem_default_opts(&o);
    if (opts) o = *opts;
    df_status st = validate_chem_opts(o);
    if (st != DF_OK) return st;
    if (n_cells == 0) return DF_OK;
    DeviceScope dev(mech->device, who);
    if (dev.st != DF_OK) return dev.st;
    StepArgs a{n_cells, ld, dt, nullptr, p, T, Y, nullptr, nullptr, cell_status, n_steps, kernel_opts(o), DF_CELL_OK};
    a.tape = static_cast<double *>(tape);
    a.tape_cap = max_substeps;
    return launch_chem_coop(mech->dev, a, CellQueue{nullptr, nullptr, nullptr, nullptr, nullptr, 0},
                            static_cast<hipStream_t>(hip_stream));
}

extern "C" df_status df_chem_adjoint_workspace_size(const df_mech *mech, int64_t n_cells, size_t *bytes) {
    using namespace df;
    clear_error();
    if (!mech || !bytes || n_cells < 0) return fail(DF_E_INVALID, "df_chem_adjoint_workspace_size: bad arguments");
    *bytes = adj_ws_bytes(mech->host.K, mech->host.M, n_cells);
    return DF_OK;
}

extern "C" df_status df_chem_adjoint(const df_mech *mech, int64_t n_cells, int64_t ld, const double *p,
                                     const void *tape, size_t tape_size, int32_t max_substeps, const double *T_bar,
                                     const double *Y_bar, double *T0_bar, double *Y0_bar, double *lnA_bar_cells,
                                     double *lnA_bar, void *workspace, size_t ws_bytes, void *hip_stream) {
    using namespace df;
    clear_error();
    const char *who = "df_chem_adjoint";
    if (!mech) return fail(DF_E_INVALID, std::string(who) + ": null mechanism handle");
    if (n_cells < 0 || ld < n_cells) return fail(DF_E_INVALID, std::string(who) + ": need 0 <= n_cells <= ld");
    if (max_substeps < 1) return fail(DF_E_INVALID, std::string(who) + ": max_substeps must be >= 1");
    if (n_cells > 0 && (!p || !tape || !T_bar || !Y_bar || !T0_bar || !Y0_bar || !workspace))
        return fail(DF_E_INVALID, std::string(who) + ": null p, tape, seed, output or workspace");
    if (n_cells > 0x7fffffff) return fail(DF_E_UNSUPPORTED, std::string(who) + ": more than 2^31-1 cells");
    const int K = mech->host.K, M = mech->host.M;
    if (n_cells > 0 && (tape_size < tape_bytes(K, n_cells, max_substeps) ||
                        reinterpret_cast<uintptr_t>(tape) % 256 != 0))
        return fail(DF_E_INVALID, std::string(who) + ": tape smaller than df_chem_tape_size or not 256-byte aligned");
    if (n_cells > 0 && (ws_bytes < adj_ws_bytes(K, M, n_cells) || reinterpret_cast<uintptr_t>(workspace) % 256 != 0))
        return fail(DF_E_INVALID,
                    std::string(who) + ": workspace smaller than df_chem_adjoint_workspace_size or not 256-byte aligned");
    if (!adjoint_supported(mech->dev))
        return fail(DF_E_UNSUPPORTED, std::string(who) + ": no adjoint kernel for this mechanism");
    if (n_cells == 0) {
        if (lnA_bar && M > 0) {
            DeviceScope dev(mech->device, who);
            if (dev.st != DF_OK) return dev.st;
            if (hipMemsetAsync(lnA_bar, 0, size_t(M) * 8, static_cast<hipStream_t>(hip_stream)) != hipSuccess)
                return fail(DF_E_HIP, std::string(who) + ": clearing lnA_bar failed");
        }
        return DF_OK;
    }
    DeviceScope dev(mech->device, who);
    if (dev.st != DF_OK) return dev.st;
    auto s = static_cast<hipStream_t>(hip_stream);
    const AdjArgs a{n_cells, ld,     p,      static_cast<const double *>(tape), max_substeps, T_bar, Y_bar,
                    T0_bar,  Y0_bar, lnA_bar_cells, static_cast<double *>(workspace)};
    df_status st = DF_OK;
    switch (K) {
#define DF_CASE(k)                                   \
    case k:                                          \
        st = launch_adjoint_k<k>(mech->dev, a, s);   \
        break;
        DF_ADJ_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            st = fail(DF_E_UNSUPPORTED, std::string(who) + ": no adjoint kernel for this mechanism");
    }
    if (st == DF_OK && lnA_bar && M > 0) {
        const double *wth = static_cast<const double *>(workspace);
        hipLaunchKernelGGL(sum_cells_kernel, dim3(unsigned(M)), dim3(256), 256 * sizeof(double), s, wth, n_cells,
                           mech->dev.src, lnA_bar);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = fail(DF_E_HIP, std::string(who) + ": reduction launch: " + hipGetErrorString(e));
    }
    return st;
}
