// Detailed-chemistry step with one wavefront per cell, for mechanisms of up to 63 species
// (the size of the hydrocarbon mechanisms for which the paper expects the DNN's gain to
// grow): FP64 throughout.
//
// The reactor (constant-pressure adiabatic, the species source term of the paper's Sec.
// "Chemistry Integration" with its density written out), the RODAS4 method, its error norm
// and its step-size controller are those of the one-cell-per-lane and 16-lane kernels.  What
// changes is how one cell occupies the 64 lanes of a wave:
//  * rates: lane t evaluates reactions t, t + 64, ... (ln k_f and ln k_r as coefficient rows
//    over functions of T, third-body sums, Troe falloff; the tables are column-major, so the
//    lanes' loads are contiguous) into per-reaction LDS arrays, with the Jacobian the
//    derivative of each rate of progress with respect to the concentration in each slot;
//  * production rates: lane 1 + k gathers species k's reactions from its list;
//  * Jacobian: the sparse entries are grouped by target on the host, so each lane sums whole
//    entries of an LDS-staged N x N matrix (no two lanes write one entry); third-body and
//    falloff rows add their dense efficiency terms one species row at a time, together with
//    the map to the (T, Y) variables;
//  * factorisation: lane r holds row r of W = I/(g h) - J in registers.  Gaussian elimination
//    with partial pivoting takes the pivot row by a wave-wide arg-max and never moves a row:
//    the pivot row is broadcast to the other lanes by readlane, and each lane remembers the
//    step at which its row was the pivot;
//  * solves: forward and back substitution in pivot order, one readlane broadcast per step;
//    component k of the solution ends in lane k.
// Wave-wide sums and maxima give every lane the same bits, so the control flow stays uniform.
// The block's barrier orders the LDS phases of one cell.
//
// This file is compiled with the AMDGPU scheduler's max-memory-clause strategy: -O2 and -O3
// builds of the 53-species instantiation with the default strategy returned garbage states on
// gfx950 (every attempt rejected), while -O1, -O3 with the scheduler off or with the max-ILP or
// max-memory-clause strategy, and the CPU build of the same source under AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_cpu_emu.py, which also fails a cross-lane operation in
// divergent code) reproduced the oracle's sub-step sequences exactly.  The optimised IR of this
// file holds no undefined value, so the difference arises in code generation, not in the source.
#include <cmath>

#include "df_internal.h"
#include "df_kinetics.h"

namespace df {
namespace {

constexpr int kW = 64;

// value of v in lane l (l wave-uniform)
__device__ __forceinline__ double rdlane(double v, int l) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffull), l));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), l));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// v of another lane of the same row of 16 by a DPP control (quad_perm, row_mirror, ...)
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffull), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(
        static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo)));
}

// Wave-wide sum and maximum: within each row of 16 lanes exchange with the lane at xor 1, xor 2,
// the mirrored lane of the half row and of the row (each pairing combines the same two numbers
// in either order, so all 16 lanes of a row end with the same bits), then combine the four rows'
// values read from lanes 0, 16, 32 and 48; every lane gets the same result.
__device__ __forceinline__ double wsum(double v) {
    v += dppd<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v += dppd<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v += dppd<0x141>(v);  // row_half_mirror
    v += dppd<0x140>(v);  // row_mirror
    return (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
}

__device__ __forceinline__ double wmax(double v) {
    v = fmax(v, dppd<0xb1>(v));
    v = fmax(v, dppd<0x4e>(v));
    v = fmax(v, dppd<0x141>(v));
    v = fmax(v, dppd<0x140>(v));
    return fmax(fmax(rdlane(v, 0), rdlane(v, 16)), fmax(rdlane(v, 32), rdlane(v, 48)));
}

// packed table entries: index | (coefficient + 8) << 20
constexpr int kPad = 8 << 20;  // index 0, coefficient 0
__device__ __forceinline__ int ent_idx(int v) { return v & 0xfffff; }
__device__ __forceinline__ int ent_nu(int v) { return (v >> 20) - 8; }

// CV: the constant-volume reactor (density given where the pressure is otherwise, internal
// energies and cv in the energy equation, concentrations independent of T and Wbar)
template <int K, bool CV = false>
struct Wave {
    static constexpr int N = K + 1;
    static_assert(N <= kW, "one wavefront holds a cell of at most 63 species");
    static constexpr int LDJ = N + 1;  // row stride of the staged Jacobian (doubles)

    // LDS of one cell (doubles): area A [max(N LDJ, 3 M)] holding the staged J, or before the
    // matrix is formed q, S (sum_m c_m dq/dc_m) and dq/dT of every reaction (q alone in f(y));
    // concentrations [kW] (slot 0 = 1, slot 1 + k = species k, mol/cm^3); D [(wsr + wsp) M], the
    // derivative of q with respect to the concentration in each slot in use; G [M], the
    // coefficient of a reaction's dense third-body term.
    struct Lds {
        double *J, *q, *S, *dT, *c, *D, *G;
    };
    __host__ __device__ static size_t area(int M) { return size_t(N) * LDJ > 3 * size_t(M) ? size_t(N) * LDJ : 3 * size_t(M); }
    static size_t lds_doubles(const MechDev &m) {
        return area(m.M) + kW + size_t(m.wsr + m.wsp + 1) * size_t(m.M);
    }
    __device__ static Lds layout(double *base, const MechDev &m) {
        const int M = m.M;
        Lds L;
        L.J = base;
        L.q = base;
        L.S = base + M;
        L.dT = base + 2 * M;
        L.c = base + area(M);
        L.D = L.c + kW;
        L.G = L.D + (m.wsr + m.wsp) * M;
        return L;
    }

    // thermo of the lane's species (lane 1 + k holds species k) and the mixture
    struct Mix {
        double T, iT, lT, T2, T3, T4;
        double rho, Wbar, cp;
        double W, iW, cpR, hRT, Yk;
        bool spl;
        const double *sr;
    };

    __device__ static void state(const MechDev &m, const Lds &L, double p, double y, int lane, Mix &s) {
        s.T = rdlane(y, 0);
        s.iT = 1.0 / s.T;
        s.lT = log(s.T);
        s.T2 = s.T * s.T;
        s.T3 = s.T2 * s.T;
        s.T4 = s.T2 * s.T2;
        s.spl = lane >= 1 && lane <= K;
        const int k = s.spl ? lane - 1 : 0;
        const double *r = m.sp + k * kSpTab;
        s.sr = r;
        const double T = s.T;
        s.W = r[0];
        s.iW = r[1];
        s.cpR = r[2] + T * (r[3] + T * (r[4] + T * (r[5] + T * r[6])));
        s.hRT = r[2] + T * (r[9] + T * (r[10] + T * (r[11] + T * r[12]))) + r[7] * s.iT;
        s.Yk = s.spl ? y : 0.0;
        const double sYW = wsum(s.Yk * s.iW);
        const double cpm = wsum(s.Yk * s.cpR * s.iW);
        s.Wbar = 1.0 / sYW;
        s.rho = CV ? p : p * s.Wbar * s.iT * (1.0 / kR);
        s.cp = CV ? (cpm - sYW) * kR : cpm * kR;
        L.c[lane] = (lane == 0) ? 1.0 : 1e-6 * s.rho * s.Yk * s.iW;
    }

    struct Rate {
        double q, G, S, dqdT, D[6];
    };

    // reaction jd at the concentrations in LDS; with DER the derivative terms
    // the table fields every reaction needs, loaded ahead of the arithmetic
    struct Pre {
        double a[10];
        int type, sl[6];
    };
    __device__ __forceinline__ static void pre_load(const MechDev &m, int jd, Pre &pr) {
        const int M = m.M;
#pragma unroll
        for (int f = 0; f < 10; ++f) pr.a[f] = m.wcr[f * M + jd];
        pr.type = m.wci[jd];
#pragma unroll
        for (int f = 0; f < 6; ++f) pr.sl[f] = m.wci[(1 + f) * M + jd];
    }

    template <bool DER>
    __device__ static void rate(const MechDev &m, const Lds &L, const Mix &s, int jd, Rate &o) {
        Pre pr;
        pre_load(m, jd, pr);
        rate_from<DER>(m, L, s, jd, pr, o);
    }

    template <bool DER>
    __device__ static void rate_from(const MechDev &m, const Lds &L, const Mix &s, int jd, const Pre &pr, Rate &o) {
        const int M = m.M;
        const double *cr = m.wcr + jd;
        const int type = pr.type;
        double lf = fma(pr.a[1], s.lT, fma(pr.a[2], s.iT, pr.a[0]));
        double lr = fma(pr.a[4], s.lT, fma(pr.a[5], s.iT, pr.a[3]));
        lr = fma(pr.a[6], s.T, lr);
        lr = fma(pr.a[7], s.T2, lr);
        lr = fma(pr.a[8], s.T3, lr);
        lr = fma(pr.a[9], s.T4, lr);
        double Mc = 0.0;
        if (type != 0) {  // third-body concentration sum_k eff_k c_k
            const double *ef = m.weff + jd;
            double m0 = 0.0, m1 = 0.0;
#pragma unroll 8
            for (int k = 0; k + 1 < K; k += 2) {
                m0 = fma(ef[k * M], L.c[1 + k], m0);
                m1 = fma(ef[(k + 1) * M], L.c[2 + k], m1);
            }
            if (K & 1) m0 = fma(ef[(K - 1) * M], L.c[K], m0);
            Mc = m0 + m1;
        }
        double phi = 1.0, dphiM = 0.0, dlphi = 0.0;
        if (type == 2) {
            // Lindemann form times the Troe broadening factor F (ln F folded into both
            // exponentials), phi = Pr/(1 + Pr)
            const double c20 = cr[20 * M], c21 = cr[21 * M], c22 = cr[22 * M];
            const double e3 = exp(c20 * s.T), e1 = exp(c21 * s.T), e2 = exp(c22 * s.iT);
            const double ek0 = exp(fma(cr[17 * M], s.lT, fma(cr[18 * M], s.iT, cr[16 * M])));  // k0 / k_inf
            const double al = cr[19 * M];
            const double Fc = fma(1.0 - al, e3, fma(al, e1, e2));
            const double Pr = ek0 * Mc;
            const double lFc = dlog(Fc) * kInvLn10;
            const double lPr = dlog(Pr) * kInvLn10;
            const double cc = -0.4 - 0.67 * lFc;
            const double nn = 0.75 - 1.27 * lFc;
            const double x = lPr + cc;
            const double iden = frcp(nn - 0.14 * x);
            const double f1 = x * iden;
            const double q1 = frcp(1.0 + f1 * f1);
            const double lF = lFc * q1;
            const double iPr1 = frcp(1.0 + Pr);
            lf = fma(kLn10, lF, lf);
            lr = fma(kLn10, lF, lr);
            phi = Pr * iPr1;
            if (DER) {
                const double gq = 2.0 * f1 * q1 * q1;
                const double dlF_dlPr = -lFc * gq * nn * iden * iden;
                const double dlF_dlFc = q1 - lFc * gq * (1.27 * x - 0.67 * nn) * iden * iden;
                const double dFc = (1.0 - al) * c20 * e3 + al * c21 * e1 - c22 * s.iT * s.iT * e2;
                const double dlnPr = (cr[17 * M] - cr[18 * M] * s.iT) * s.iT;
                dlphi = (iPr1 + dlF_dlPr) * dlnPr + dlF_dlFc * fdiv(dFc, Fc);
                dphiM = ek0 * iPr1 * (iPr1 + dlF_dlPr);
            }
        }
        const double Ef = exp(lf), Er = exp(lr);
        const double kf = Ef * phi, kr = Er * phi;
        const double c0 = L.c[pr.sl[0]], c1 = L.c[pr.sl[1]], c2 = L.c[pr.sl[2]];
        const double d0 = L.c[pr.sl[3]], d1 = L.c[pr.sl[4]], d2 = L.c[pr.sl[5]];
        const double Pf = c0 * c1 * c2, Pb = d0 * d1 * d2;
        const double fwd = kf * Pf, rev = kr * Pb, X = fwd - rev;
        const double Mq = (type == 1) ? Mc : 1.0;
        o.q = Mq * X;
        if (DER) {
            const double dlf = (pr.a[1] - pr.a[2] * s.iT) * s.iT + dlphi;
            const double dlr = (pr.a[4] - pr.a[5] * s.iT) * s.iT +
                               fma(s.T, fma(s.T, fma(4.0 * pr.a[9], s.T, 3.0 * pr.a[8]), 2.0 * pr.a[7]), pr.a[6]) +
                               dlphi;
            o.dqdT = Mq * (fwd * dlf - rev * dlr);
            o.G = (type == 1) ? X : ((type == 2) ? (Ef * dphiM) * Pf - (Er * dphiM) * Pb : 0.0);
            o.S = Mq * (cr[23 * M] * fwd - cr[24 * M] * rev) + Mc * o.G;
            const double kfM = Mq * kf, krM = Mq * kr;
            o.D[0] = kfM * c1 * c2;
            o.D[1] = kfM * c0 * c2;
            o.D[2] = kfM * c0 * c1;
            o.D[3] = -krM * d1 * d2;
            o.D[4] = -krM * d0 * d2;
            o.D[5] = -krM * d0 * d1;
        }
    }

    // component `lane` of f(y)
    __device__ static double rhs(const MechDev &m, const Lds &L, double p, double y, int lane) {
        Mix s;
        state(m, L, p, y, lane, s);
        __syncthreads();
        // the next round's table fields are loaded before this round's arithmetic
        {
            const int M = m.M;
            Pre cur, nxt;
            pre_load(m, lane < M ? lane : M - 1, cur);
            for (int jd = lane; jd < M; jd += kW) {
                const int jn = jd + kW;
                pre_load(m, jn < M ? jn : M - 1, nxt);
                Rate o;
                rate_from<false>(m, L, s, jd, cur, o);
                L.q[jd] = o.q;
                cur = nxt;
            }
        }
        __syncthreads();
        double wd = 0.0;
        if (s.spl) {
            const int k = lane - 1;
            const int e1 = m.wlo[k + 1];
            for (int e = m.wlo[k]; e < e1; e += 4) {
                int v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = (e + i < e1) ? m.wlp[e + i] : kPad;
#pragma unroll
                for (int i = 0; i < 4; ++i) wd = fma(double(ent_nu(v[i])), L.q[ent_idx(v[i])], wd);
            }
        }
        const double rho = s.rho;
        const double hs = wsum(s.spl ? (CV ? s.hRT - 1.0 : s.hRT) * wd : 0.0);  // U/RT = H/RT - 1
        __syncthreads();
        if (lane == 0) return -hs * (1e6 * kR) * s.T / (rho * s.cp);
        return s.spl ? (1e6 / rho) * s.W * wd : 0.0;
    }

    // J = df/dy staged in LDS (row-major, stride LDJ) and f(y) in lane order
    __device__ static double jacobian(const MechDev &m, const Lds &L, double p, double y, int lane) {
        const int M = m.M;
        Mix s;
        state(m, L, p, y, lane, s);
        __syncthreads();
        for (int jd = lane; jd < M; jd += kW) {
            Rate o;
            rate<true>(m, L, s, jd, o);
            L.q[jd] = o.q;
            L.S[jd] = o.S;
            L.dT[jd] = o.dqdT;
            L.G[jd] = o.G;
            // the slot derivatives of the slots in use
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < m.wsr) L.D[i * M + jd] = o.D[i];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < m.wsp) L.D[(m.wsr + i) * M + jd] = o.D[3 + i];
        }
        __syncthreads();
        // per species: production rate, sum_m c_m dq/dc_m and dq/dT at fixed c
        double wd = 0.0, sq = 0.0, dt = 0.0;
        if (s.spl) {
            const int k = lane - 1;
            const int e1 = m.wlo[k + 1];
            for (int e = m.wlo[k]; e < e1; e += 4) {
                int v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = (e + i < e1) ? m.wlp[e + i] : kPad;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = ent_idx(v[i]);
                    const double nu = double(ent_nu(v[i]));
                    wd = fma(nu, L.q[j], wd);
                    sq = fma(nu, L.S[j], sq);
                    dt = fma(nu, L.dT[j], dt);
                }
            }
        }
        __syncthreads();
        for (int e = lane; e < N * LDJ; e += kW) L.J[e] = 0.0;
        __syncthreads();
        // concentration-space derivatives A_kl = sum_j nu_kj dq_j/dc_l: whole entries per lane
        for (int r = 0; r < m.wnr; ++r) {
            const int t = r * kW + lane;
            const int *ep = m.well + m.wrb[r] + lane;
            const int cm = m.wrc[r];
            double acc = 0.0;
            for (int e0 = 0; e0 < cm; e0 += 8) {
                int v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = (e0 + i < cm) ? ep[(e0 + i) * kW] : kPad;
#pragma unroll
                for (int i = 0; i < 8; ++i) acc = fma(double(ent_nu(v[i])), L.D[ent_idx(v[i])], acc);
            }
            if (t < m.wnt) L.J[m.wtk[t]] = acc;
        }
        __syncthreads();
        const double T = s.T;
        const double coef = (1e6 / s.rho) * s.W;
        // at constant pressure c depends on T and Wbar; at constant volume it does not
        const double gk = CV ? 0.0 : coef * s.Wbar * (wd - sq);
        const double fk = s.spl ? coef * wd : 0.0;
        const double hm = s.spl ? (CV ? s.hRT - 1.0 : s.hRT) * kR * T * s.iW : 0.0;  // J/kg: h_k, or u_k
        const double cpm = s.spl ? (CV ? s.cpR - 1.0 : s.cpR) * kR * s.iW : 0.0;     // J/kg/K: cp_k, or cv_k
        const double *r = s.sr;
        const double dcpR = r[3] + T * (r[16] + T * (r[17] + T * r[18]));
        const double dcpdT = wsum(s.spl ? s.Yk * dcpR * kR * s.iW : 0.0);
        const double icp = 1.0 / s.cp;
        const double fT = -wsum(hm * fk) * icp;
        const double cf = wsum(cpm * fk);
        // species rows: the dense third-body terms (dq/dc_l gains eff_l G), over the flat list of
        // (row, reaction) pairs in batches, the row of entry e being the number of rows 1..K-1
        // starting at or before e; then the map to (T, Y) with
        // dc_m/dY_l = 1e-6 rho delta_ml / W_m - c_m Wbar / W_l and dc_m/dT = -c_m / T at
        // constant pressure
        const double iWl = (lane < K) ? m.sp[lane * kSpTab + 1] : 0.0;
        const double *effl = m.ceff + ((lane < K) ? lane : 0);
        const int row_start = (lane >= 1 && lane < K) ? m.wdo[lane] : 0x7fffffff;
        const int nd = m.wdo[K];
        for (int e0 = 0; e0 < nd; e0 += 8) {
            int v[8], kr[8];
            double ef[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = e0 + i;
                v[i] = (e < nd) ? m.wdp[e] : kPad;
                kr[i] = __popcll(__ballot(row_start <= e));
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) ef[i] = effl[size_t(ent_idx(v[i])) * (K + 4)];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (lane < K) {
                    double &Jkl = L.J[(1 + kr[i]) * LDJ + 1 + lane];
                    Jkl = fma(double(ent_nu(v[i])) * L.G[ent_idx(v[i])], ef[i], Jkl);
                }
        }
        for (int k = 0; k < K; ++k) {
            const double Wk = m.sp[k * kSpTab];
            const double g = rdlane(gk, 1 + k);
            if (lane < K) {
                double &Jkl = L.J[(1 + k) * LDJ + 1 + lane];
                Jkl = (Wk * Jkl + g) * iWl;
            }
        }
        if (s.spl) L.J[lane * LDJ] = CV ? coef * dt : coef * (dt + (wd - sq) * s.iT);
        __syncthreads();
        // temperature row: f_T = -sum_k h_k f_k / cp
        double acc = 0.0;
        for (int k = 1; k <= K; ++k) {
            const double h = rdlane(hm, k);
            if (lane < N) acc = fma(h, L.J[k * LDJ + lane], acc);
        }
        if (lane == 0) acc += cf;
        const double dcp = (lane == 0) ? dcpdT : cpm;
        if (lane < N) L.J[lane] = -(acc + fT * dcp) * icp;
        __syncthreads();
        return (lane == 0) ? fT : fk;
    }

    // row `lane` of W = ig I - J from the staged J
    __device__ static void load_rows(const Lds &L, double ig, int lane, double (&a)[N]) {
        const bool act = lane < N;
        const double *row = L.J + (act ? lane : 0) * LDJ;
#pragma unroll
        for (int c = 0; c < N; ++c) a[c] = act ? ((c == lane ? ig : 0.0) - row[c]) : 0.0;
    }

    // Gaussian elimination with partial pivoting (largest magnitude, ties to the lowest lane);
    // rows stay in their lanes.  On return lane r holds, in columns below its pivot step pos,
    // the multipliers of the steps it was eliminated in, at pos the reciprocal of its pivot and
    // beyond it its row of U.  perm[k] is the lane of step k's pivot.
    __device__ static void lu(double (&a)[N], int lane, int (&perm)[N], int &pos) {
        bool used = lane >= N;
        pos = used ? -1 : 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double cand = used ? -1.0 : fabs(a[k]);
            const double mx = wmax(cand);
            unsigned long long bal = __ballot(!used && cand == mx);
            if (bal == 0ull) bal = __ballot(!used);  // a column of NaN: any row not yet a pivot
            const int p = __ffsll(static_cast<long long>(bal)) - 1;
            perm[k] = p;
            const double inv = 1.0 / rdlane(a[k], p);
            const bool me = lane == p;
            const bool upd = !used && !me;
            const double l = upd ? a[k] * inv : 0.0;
#pragma unroll
            for (int c = k + 1; c < N; ++c) a[c] = fma(-l, rdlane(a[c], p), a[c]);
            a[k] = me ? inv : (upd ? l : a[k]);
            pos = me ? k : pos;
            used = used || me;
        }
    }

    // solve W x = b, b given by component in lane order; returns x in lane order
    __device__ static double solve(const double (&a)[N], const int (&perm)[N], int pos, int lane, double b) {
        // forward: component of pivot step k is final after steps < k
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            const double yk = rdlane(b, perm[k]);
            b = fma(-((pos > k) ? a[k] : 0.0), yk, b);
        }
        double x = 0.0;
#pragma unroll
        for (int k = N - 1; k >= 0; --k) {
            const double xk = rdlane(b * a[k], perm[k]);
            x = (lane == k) ? xk : x;
            if (k > 0) b = fma(-((pos >= 0 && pos < k) ? a[k] : 0.0), xk, b);
        }
        return x;
    }
};

template <int K, bool CV>
__global__ __launch_bounds__(kW) void chem_wave_kernel(MechDev m, StepArgs a, const int32_t *__restrict__ cidx,
                                                       const int32_t *__restrict__ dcount) {
    using Wv = Wave<K, CV>;
    constexpr int N = K + 1;
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int64_t slot = blockIdx.x;
    const int64_t limit = dcount ? int64_t(*dcount) : a.n;
    if (slot >= limit) return;
    const int64_t i = cidx ? int64_t(cidx[slot]) : slot;
    const typename Wv::Lds L = Wv::layout(lds, m);
    const Opts &o = a.o;

    const double p = a.p[i];
    const double dtc = a.dts ? a.dts[i] : a.dt;
    const double y0 = (lane == 0) ? a.T[i] : ((lane <= K) ? a.Y[(lane - 1) * a.ld + i] : 0.0);
    const bool okl = isfinite(y0) && (lane != 0 || y0 > 0.0);
    const bool ok = __ballot(!okl) == 0ull && isfinite(p) && p > 0.0 && isfinite(dtc) && dtc > 0.0;
    if (!ok) {
        if (lane == 0) {
            if (a.status) a.status[i] = DF_CELL_NONFINITE;
            if (a.nsteps) {
                a.nsteps[i] = 0;
                a.nsteps[a.n + i] = 0;
            }
        }
        if (a.rr && lane >= 1 && lane <= K) a.rr[(lane - 1) * a.ld + i] = 0.0;
        return;
    }
    const double h_in = a.h_io ? a.h_io[i] : 0.0;
    bool fresh = !(h_in > 0.0);
    double h = fresh ? 0.0 : fmin(h_in, dtc);
    if (!fresh && !(h >= o.h_min)) h = o.h_min;
    double t = 0.0, h_final = 0.0;
    int acc = 0, rej = 0, st = DF_CELL_OK;
    bool prev_rej = false;
    double y = y0;
    const double sc_abs = (lane == 0) ? o.atol_T : o.atol_Y;
    const bool act = lane < N;

    while (true) {
        if (acc + rej >= o.max_steps) {
            st = DF_CELL_MAX_STEPS;
            break;
        }
        const double f0 = Wv::jacobian(m, L, p, y, lane);
        if (fresh) {
            // initial sub-step from the weighted norms of y0 and f(y0)
            const double sc = sc_abs + o.rtol * fabs(y);
            const double ny = sqrt(wsum(act ? (y / sc) * (y / sc) : 0.0) / N);
            const double nf = sqrt(wsum(act ? (f0 / sc) * (f0 / sc) : 0.0) / N);
            h = (nf > 0.0) ? fmin(0.01 * ny / nf, dtc) : dtc;
            if (!(h >= o.h_min)) h = o.h_min;
            fresh = false;
        }
        const bool last = (t + h >= dtc);
        const double ht = last ? dtc - t : h;
        double W[N];
        Wv::load_rows(L, 1.0 / (Rodas4::g * ht), lane, W);
        int perm[N], pos;
        Wv::lu(W, lane, perm, pos);
        const double ih = 1.0 / ht;
        double u[6], ys = y;
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            double v;
            if (s == 0) {
                v = f0;
            } else {
                double w = y;
#pragma unroll
                for (int j = 0; j < s; ++j) w = fma(Rodas4::a[s][j], u[j], w);
                ys = w;
                v = Wv::rhs(m, L, p, ys, lane);
                double c = 0.0;
#pragma unroll
                for (int j = 0; j < s; ++j) c = fma(Rodas4::c[s][j], u[j], c);
                v = fma(c, ih, v);
            }
            u[s] = Wv::solve(W, perm, pos, lane, act ? v : 0.0);
        }
        // y_new = (stage-6 state) + u5 ; error = u5
        const double yn = ys + u[5];
        const double sc = sc_abs + o.rtol * fmax(fabs(y), fabs(yn));
        const double rr = u[5] / sc;
        const double err = sqrt(wsum(act ? rr * rr : 0.0) / N);
        const double fmx = prev_rej ? 1.0 : 6.0;
        double fac;
        if (!isfinite(err))
            fac = 0.2;
        else if (err == 0.0)
            fac = fmx;
        else
            fac = fmin(fmx, fmax(0.2, 0.9 * pow(err, -0.25)));
        if (isfinite(err) && err <= 1.0) {
            ++acc;
            y = yn;
            h_final = h;
            prev_rej = false;
            if (last) break;
            t += ht;
            h = ht * fac;
        } else {
            ++rej;
            prev_rej = true;
            h = ht * fac;
            if (h < o.h_min) {
                st = DF_CELL_H_UNDERFLOW;
                break;
            }
        }
    }
    // results; rr = rho0 (Y - Y0) / dt with rho0 the density of the input state
    if (a.rr) {
        const double T0 = rdlane(y0, 0);
        const int k = (lane >= 1 && lane <= K) ? lane - 1 : 0;
        const double sYW = wsum((lane >= 1 && lane <= K) ? y0 * m.sp[k * kSpTab + 1] : 0.0);
        const double rdt = (CV ? p : p / (sYW * kR * T0)) / dtc;  // the density is given at constant volume
        if (lane >= 1 && lane <= K) a.rr[(lane - 1) * a.ld + i] = rdt * (y - y0);
    }
    if (lane == 0) a.T[i] = y;
    if (lane >= 1 && lane <= K) a.Y[(lane - 1) * a.ld + i] = y;
    if (lane == 0) {
        if (a.h_io) a.h_io[i] = (st == DF_CELL_OK) ? h_final : h;
        if (a.status) a.status[i] = (st == DF_CELL_OK) ? a.status_ok : st;
        if (a.nsteps) {
            a.nsteps[i] = acc;
            a.nsteps[a.n + i] = rej;
        }
    }
}

template <int K>
size_t wave_lds_bytes(const MechDev &m) {
    return 8 * Wave<K>::lds_doubles(m);
}

template <int K, bool CV = false>
df_status launch_wave_k(const MechDev &m, const StepArgs &a, const int32_t *cidx, const int32_t *dcount,
                        hipStream_t stream) {
    const size_t lds = wave_lds_bytes<K>(m);
    auto kernel = chem_wave_kernel<K, CV>;
    if (lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(lds)) != hipSuccess)
        return fail(DF_E_HIP, "df_chem_step: cannot raise the LDS limit of the one-wave-per-cell kernel");
    hipLaunchKernelGGL(kernel, dim3(unsigned(a.n)), dim3(kW), lds, stream, m, a, cidx, dcount);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("chem_step wave launch: ") + hipGetErrorString(e));
    return DF_OK;
}

// species counts with a compiled one-wave-per-cell kernel
#define DF_WAVE_SPECIES_LIST(X) X(9) X(53)

}  // namespace

bool chem_wave_supported(const MechDev &m) {
    switch (m.K) {
#define DF_CASE(k) \
    case k:        \
        return wave_lds_bytes<k>(m) <= 160 * 1024;
        DF_WAVE_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return false;
    }
}

df_status launch_chem_wave(const MechDev &m, const StepArgs &a, const int32_t *cidx, const int32_t *dcount,
                           hipStream_t stream) {
    if (a.n == 0) return DF_OK;
    if (a.n > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "df_chem_step: too many cells for one launch");
    if (a.tape) return fail(DF_E_UNSUPPORTED, "df_chem_step: the one-wave-per-cell kernel records no tape");
    if (!chem_wave_supported(m))
        return fail(DF_E_UNSUPPORTED, "df_chem_step: no one-wave-per-cell kernel for " + std::to_string(m.K) +
                                          " species and " + std::to_string(m.M) + " reactions");
    switch (m.K) {
#define DF_CASE(k) \
    case k:        \
        return launch_wave_k<k>(m, a, cidx, dcount, stream);
        DF_WAVE_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return fail(DF_E_UNSUPPORTED, "df_chem_step: no one-wave-per-cell kernel for " + std::to_string(m.K));
    }
}

// the constant-volume reactor on one wavefront per cell (df_chem_step_const_volume for species
// counts without a one-cell-per-lane kernel); a.p holds the density
df_status launch_chem_wave_cv(const MechDev &m, const StepArgs &a, hipStream_t stream) {
    if (a.n == 0) return DF_OK;
    if (a.n > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "df_chem_step_const_volume: too many cells for one launch");
    if (!chem_wave_supported(m))
        return fail(DF_E_UNSUPPORTED, "df_chem_step_const_volume: no kernel for " + std::to_string(m.K) + " species");
    switch (m.K) {
#define DF_CASE(k) \
    case k:        \
        return launch_wave_k<k, true>(m, a, nullptr, nullptr, stream);
        DF_WAVE_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return fail(DF_E_UNSUPPORTED, "df_chem_step_const_volume: no kernel for " + std::to_string(m.K));
    }
}

}  // namespace df
