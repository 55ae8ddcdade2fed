// Detailed-chemistry step on gfx950 with 16 lanes per cell (four cells per wave64).
//
// Same integration as the one-cell-per-lane kernel (constant-pressure reactor,
// RODAS4, identical step-size controller), with the work of one attempt spread
// over the lanes of the cell so that the latency of a sub-step -- which sets
// the time of a stiff cell's hundreds of sequential sub-steps -- shrinks.  The
// wave issues one instruction stream for its 64 lanes, so the cost of a phase is
// the number of instructions any lane needs; the layout keeps every lane on the
// same short stream:
//   * rates: lane l evaluates the reactions stored at l, l + 16, ...; ln k_f and
//     ln k_r = ln k_f - ln K_c are dot products of per-reaction coefficient rows
//     with functions of T (ln T, 1/T, T..T^4), so a rate constant costs one exp and
//     no species data; only the concentrations cross lanes (one LDS exchange);
//   * production rates: species lane k sums nu q over a fixed-length list; lane 0
//     sums the 16 partial sums of q_j dH_j/(R T), which gives dT/dt in the same pass;
//   * Jacobian: each reaction writes one dense record dq/dc (plus dq/dT, q and the
//     density term) to LDS, species lane k assembles row k from its list, and lane c
//     then reads column c and adds the T-row entry;
//   * linear algebra: row i of W = I/(gamma h) - J lives in lane i; Gauss-Jordan
//     elimination with partial pivoting (pivot search as a cross-lane maximum within
//     the 16 lanes, pivot row broadcast through LDS) gives W^-1, so each stage solve is
//     one N-term dot product per lane.
// State vectors are replicated in the lanes of a cell; every scalar that steers
// control flow (error norm, step size, accept/reject) is computed from the same
// LDS data in the same order by all 16 lanes, so a cell's lanes never diverge.
// Cells of a wave communicate only through their own LDS region.
// With two halves per cell (H = 2: 32 lanes, two cells per wave) the second 16 lanes take
// the second slot of reactions, so each lane evaluates half as many rate constants in the
// rate phases that dominate an attempt; every other phase runs replicated in both halves.
// Each reaction's arithmetic and every sum's order are those of the 16-lane layout, so the
// two layouts give the same bits.
#include <cmath>

#include "df_internal.h"
#include "df_kinetics.h"
#include "df_lane.h"

namespace df {
namespace {

constexpr int G = kCoopLanes;       // lanes of a cell that hold the rows (the cell's first half)
constexpr int kCellsPerBlock = 4;   // one wave64 per block, 16-lane cells
constexpr int kMaxRPL = 4;          // reaction slots per lane instantiated (M <= 64)

// Order LDS accesses of the lanes of a wave: the wave executes in lockstep and LDS
// requests of one wave are served in order, so only the compiler must not move
// memory operations across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row strides of LDS tables read by the 16 lanes of a cell at different rows and the
// same column: an odd number of doubles (or ints) puts the 16 reads in 16 banks.
__host__ __device__ constexpr int odd(int x) { return x | 1; }
constexpr int kSpS = kSpTab + 1;  // 21 doubles per species row

// H: halves (of 16 lanes) per cell; the lanes of half h evaluate reaction slots h, h + H, ...
template <int K, int RPL, int H = 1>
struct Coop {
    static_assert(H == 1 || H == 2, "one or two halves per cell");
    static_assert(RPL % H == 0, "the reaction slots divide between the halves");
    static constexpr int N = K + 1;
    static constexpr int GL = G * H;       // lanes per cell
    static constexpr int RL = RPL / H;     // reaction slots per lane
    static constexpr int CPB = kCellsPerBlock / H;  // cells per block
    static constexpr int MP = G * RPL;     // stored reactions incl. inert padding
    static constexpr int RS = odd(K + 4);  // record: dq/dc_0..K-1, q, dq/dT, S, scratch
    static constexpr int EFS = odd(K + 4);
    static constexpr int EWS = odd(K);
    static constexpr int LM = kCoopList;

    // per-cell LDS layout, in doubles
    static constexpr int oC = 0;                 // concentrations (slot 0 = 1)
    static constexpr int oCpt = oC + N;          // y_k cp_k/(R W_k) (slot 0 = 0)
    static constexpr int oHm = oCpt + N;         // h_k in J/kg
    static constexpr int oDcp = oHm + N;         // y_k dcp_k/dT in J/kg/K^2
    static constexpr int oExt = oDcp + N;        // h_k f_k | cp_k f_k
    static constexpr int oQ = oExt + 2 * N;      // q_0..q_{MP-1}, zero, 16 lane partial sums
    static constexpr int oRec = oQ + MP + 1 + G; // records, row MP stays zero
    static constexpr int oRows = oRec + (MP + 1) * RS;
    static constexpr int oProw = oRows + N * N;  // pivot-row broadcast, two buffers
    static constexpr int oVec = oProw + 2 * (2 * N + 1);
    static constexpr int oVec2 = oVec + N;
    static constexpr int oRed = oVec2 + N;
    static constexpr int oClaim = oRed + 3 * N;  // a claimed cell index (int64), broadcast to the group
    static constexpr int oDH = oClaim + 1;       // reaction enthalpies dH_j/(R T) (two halves only)
    static constexpr int kEnd = oDH + (H > 1 ? MP : 0);
    // cells of a wave start 10 doubles (20 banks) apart modulo the 64 banks
    static constexpr int kStride = kEnd + ((10 - kEnd % 32) + 32) % 32;

    // mechanism tables staged in LDS once per block, offsets in bytes
    static constexpr int tSp = 0;
    static constexpr int tCr = tSp + K * kSpS * 8;
    static constexpr int tEff = tCr + MP * kCrDbl * 8;
    static constexpr int tEw = tEff + MP * EFS * 8;
    static constexpr int tCi = tEw + MP * EWS * 8;
    static constexpr int tBytes = (tCi + MP * kCiInt * 4 + 15) & ~15;
    static constexpr size_t lds_bytes() { return size_t(tBytes) + size_t(kStride) * CPB * 8; }

    struct Tab {
        const double *sp, *cr, *eff, *ew;
        const int *ci;
    };

    // functions of the stage state shared by all lanes
    struct St {
        double T, iT, lT, T2, T3, T4, rho, irho, Wbar, c6;
    };

    __device__ __forceinline__ static void state(const Tab &tb, double p, double ip, const double (&y)[N], St &s) {
        s.T = y[0];
        s.iT = frcp(s.T);
        s.lT = dlog(s.T);
        s.T2 = s.T * s.T;
        s.T3 = s.T2 * s.T;
        s.T4 = s.T2 * s.T2;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int k = 0; k < K; k += 2) a0 = fma(y[1 + k], tb.sp[k * kSpS + 1], a0);
#pragma unroll
        for (int k = 1; k < K; k += 2) a1 = fma(y[1 + k], tb.sp[k * kSpS + 1], a1);
        const double sYW = a0 + a1;
        s.Wbar = frcp(sYW);
        s.rho = p * s.Wbar * s.iT * (1.0 / kR);
        s.irho = kR * s.T * sYW * ip;
        s.c6 = 1e-6 * s.rho;
    }

    struct Rate {
        double kf, kr, Mc, dH, dlf, dlr, dkfM, dkrM;
        int type;
        int sl[6];  // reactant and product slots (1 + species index, 0 = empty)
    };

    // rate constants of stored reaction jd (CGS); with D also d ln k/dT at fixed [M] and dk/d[M]
    template <bool D>
    __device__ __forceinline__ static void rate(const Tab &tb, int jd, const St &s, const double (&y)[N], Rate &o) {
        const double *cr = tb.cr + jd * kCrDbl;
        const int *ci = tb.ci + jd * kCiInt;
        const int type = ci[0];
#pragma unroll
        for (int i = 0; i < 6; ++i) o.sl[i] = ci[1 + i];
        // reaction enthalpy sum_k nu_k H_k/(R T)
        o.dH = fma(s.T, fma(s.T, fma(s.T, fma(s.T, cr[14], cr[13]), cr[12]), cr[11]), fma(cr[15], s.iT, cr[10]));
        double lf = fma(cr[1], s.lT, fma(cr[2], s.iT, cr[0]));
        double lr = fma(cr[4], s.lT, fma(cr[5], s.iT, cr[3]));
        lr = fma(cr[6], s.T, lr);
        lr = fma(cr[7], s.T2, lr);
        lr = fma(cr[8], s.T3, lr);
        lr = fma(cr[9], s.T4, lr);
        double Mc = 0.0;
        if (type != 0) {  // third-body concentration sum_k eff_k c_k
            const double *ew = tb.ew + jd * EWS;
            double m0 = 0.0, m1 = 0.0;
#pragma unroll
            for (int k = 0; k < K; k += 2) m0 = fma(ew[k], y[1 + k], m0);
#pragma unroll
            for (int k = 1; k < K; k += 2) m1 = fma(ew[k], y[1 + k], m1);
            Mc = (m0 + m1) * s.c6;
        }
        double phi = 1.0, dphiM = 0.0, dlphi = 0.0;
        if (type == 2) {
            // Lindemann form times the Troe broadening factor F; ln F is folded into the two
            // exponentials, phi = Pr/(1 + Pr)
            const double e3 = exp(cr[20] * s.T), e1 = exp(cr[21] * s.T), e2 = exp(cr[22] * s.iT);
            const double ek0 = exp(fma(cr[17], s.lT, fma(cr[18], s.iT, cr[16])));  // k0 / k_inf
            const double al = cr[19];
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
            if (D) {
                const double gq = 2.0 * f1 * q1 * q1;
                const double dlF_dlPr = -lFc * gq * nn * iden * iden;
                const double dlF_dlFc = q1 - lFc * gq * (1.27 * x - 0.67 * nn) * iden * iden;
                const double dFc = (1.0 - al) * cr[20] * e3 + al * cr[21] * e1 - cr[22] * s.iT * s.iT * e2;
                const double dlnPr = (cr[17] - cr[18] * s.iT) * s.iT;
                dlphi = (iPr1 + dlF_dlPr) * dlnPr + dlF_dlFc * fdiv(dFc, Fc);
                dphiM = ek0 * iPr1 * (iPr1 + dlF_dlPr);
            }
        }
        const double Ef = exp(lf), Er = exp(lr);
        o.kf = Ef * phi;
        o.kr = Er * phi;
        o.Mc = Mc;
        o.type = type;
        if (D) {
            o.dlf = (cr[1] - cr[2] * s.iT) * s.iT + dlphi;
            o.dlr = (cr[4] - cr[5] * s.iT) * s.iT + fma(s.T, fma(s.T, fma(4.0 * cr[9], s.T, 3.0 * cr[8]), 2.0 * cr[7]), cr[6]) +
                    dlphi;
            o.dkfM = Ef * dphiM;
            o.dkrM = Er * dphiM;
        }
    }

    // component r of f(y) in lane r (r < N); yo = y[r]; rl is the lane within the cell
    __device__ static double rhs(const Tab &tb, double *sh, int r, int rl, double p, double ip, const double (&y)[N],
                                 double yo, const int (&li)[LM], const double (&lc)[LM]) {
        St s;
        state(tb, p, ip, y, s);
        const bool spl = (r >= 1 && r <= K);
        const double *sp = tb.sp + (spl ? r - 1 : 0) * kSpS;
        if (spl) {
            const double cpR = fma(s.T, fma(s.T, fma(s.T, fma(s.T, sp[6], sp[5]), sp[4]), sp[3]), sp[2]);
            sh[oC + r] = s.c6 * yo * sp[1];
            sh[oCpt + r] = yo * cpR * sp[1];
        }
        Rate rt[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) rate<false>(tb, rl + GL * q, s, y, rt[q]);
        wave_sync();
        double hs = 0.0;
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            const int jd = rl + GL * q;
            const int *sl = rt[q].sl;
            const double Pf = sh[oC + sl[0]] * sh[oC + sl[1]] * sh[oC + sl[2]];
            const double Pb = sh[oC + sl[3]] * sh[oC + sl[4]] * sh[oC + sl[5]];
            double X = rt[q].kf * Pf - rt[q].kr * Pb;
            X = (rt[q].type == 1) ? X * rt[q].Mc : X;
            if (H == 1) hs = fma(X, rt[q].dH, hs);
            sh[oQ + jd] = X;
            if (H > 1) sh[oDH + jd] = rt[q].dH;
        }
        if (H > 1) {
            // the partial sum of lane r over its reactions r, r + 16, ... in slot order, as the
            // 16-lane layout forms it in registers
            wave_sync();
#pragma unroll
            for (int q = 0; q < RPL; ++q) hs = fma(sh[oQ + r + G * q], sh[oDH + r + G * q], hs);
        }
        sh[oQ + MP + 1 + r] = hs;
        double c0 = 0.0, c1 = 0.0;
#pragma unroll
        for (int k = 1; k <= K; k += 2) c0 += sh[oCpt + k];
#pragma unroll
        for (int k = 2; k <= K; k += 2) c1 += sh[oCpt + k];
        const double icp = frcp(c0 + c1);  // 1/(cp/R) per unit mass
        wave_sync();
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int e = 0; e < LM; e += 2) {
            a0 = fma(lc[e], sh[oQ + li[e]], a0);
            a1 = fma(lc[e + 1], sh[oQ + li[e + 1]], a1);
        }
        const double acc = a0 + a1;
        // dT/dt = -sum_k h_k dY_k/dt / cp = -1e6 T sum_j q_j dH_j/(R T) / (rho cp/R)
        return (r == 0) ? -1e6 * s.T * acc * s.irho * icp : 1e6 * sp[0] * acc * s.irho;
    }

    // the analytic Jacobian J = d f/d y, row-major in LDS (rows), and f_r.  Derivatives are
    // taken in concentration space and mapped to (T, Y); species lane k writes row k, lane c
    // then adds the T-row entry of column c from f_T = -sum_k h_k f_k / cp.
    __device__ static double jacobian(const Tab &tb, double *sh, int r, int rl, double p, double ip,
                                      const double (&y)[N], double yo, const int (&li)[LM], const double (&lc)[LM]) {
        St s;
        state(tb, p, ip, y, s);
        const bool spl = (r >= 1 && r <= K);
        const double *sp = tb.sp + (spl ? r - 1 : 0) * kSpS;
        const double T = s.T;
        const double cpR = fma(T, fma(T, fma(T, fma(T, sp[6], sp[5]), sp[4]), sp[3]), sp[2]);
        const double dcpR = fma(T, fma(T, fma(T, sp[18], sp[17]), sp[16]), sp[3]);
        const double hRT = fma(T, fma(T, fma(T, fma(T, sp[12], sp[11]), sp[10]), sp[9]), sp[2]) + sp[7] * s.iT;
        const double cpm = cpR * kR * sp[1];    // J/kg/K of the lane's species
        const double hm = hRT * kR * T * sp[1]; // J/kg
        if (spl) {
            sh[oC + r] = s.c6 * yo * sp[1];
            sh[oCpt + r] = yo * cpR * sp[1];
            sh[oHm + r] = hm;
            sh[oDcp + r] = yo * dcpR * kR * sp[1];
        }
        Rate rt[RL];
        int ecol[RL][kCoopEnt], emsk[RL][kCoopEnt];
        double eeff[RL][kCoopEnt], nrp[RL][2], effr[RL][K];
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            const int jd = rl + GL * q;
            rate<true>(tb, jd, s, y, rt[q]);
            const int *ci = tb.ci + jd * kCiInt;
            const double *ef = tb.eff + jd * EFS;
#pragma unroll
            for (int e = 0; e < kCoopEnt; ++e) {
                ecol[q][e] = ci[7 + 2 * e];
                emsk[q][e] = ci[8 + 2 * e];
                eeff[q][e] = ef[ecol[q][e]];
            }
#pragma unroll
            for (int l = 0; l < K; ++l) effr[q][l] = ef[l];
            nrp[q][0] = tb.cr[jd * kCrDbl + 23];
            nrp[q][1] = tb.cr[jd * kCrDbl + 24];
        }
        wave_sync();
#pragma unroll
        for (int q = 0; q < RL; ++q) {
            const int jd = rl + GL * q;
            const Rate &k = rt[q];
            const int *sl = k.sl;
            const double c0 = sh[oC + sl[0]], c1 = sh[oC + sl[1]], c2 = sh[oC + sl[2]];
            const double d0 = sh[oC + sl[3]], d1 = sh[oC + sl[4]], d2 = sh[oC + sl[5]];
            const double P0 = c1 * c2, P1 = c0 * c2, P2 = c0 * c1;  // d Pf / d c of reactant slot i
            const double Q0 = d1 * d2, Q1 = d0 * d2, Q2 = d0 * d1;
            const double Pf = c0 * P0, Pb = d0 * Q0;
            const double fwd = k.kf * Pf, rev = k.kr * Pb, X = fwd - rev;
            const double Mq = (k.type == 1) ? k.Mc : 1.0;
            // d q / d [M] (times d[M]/dc_l = eff_l): X for third-body rows, falloff term for Troe rows
            const double Gd = (k.type == 1) ? X : k.dkfM * Pf - k.dkrM * Pb;
            const double S = fma(Gd, k.Mc, Mq * (nrp[q][0] * fwd - nrp[q][1] * rev));  // sum_l c_l dq/dc_l
            double *rc = sh + oRec + jd * RS;
#pragma unroll
            for (int l = 0; l < K; ++l) rc[l] = Gd * effr[q][l];
            const double fk = Mq * k.kf, rk = Mq * k.kr;
#pragma unroll
            for (int e = 0; e < kCoopEnt; ++e) {
                const int msk = emsk[q][e];
                const double dr = ((msk & 1) ? P0 : 0.0) + ((msk & 2) ? P1 : 0.0) + ((msk & 4) ? P2 : 0.0);
                const double dp = ((msk & 8) ? Q0 : 0.0) + ((msk & 16) ? Q1 : 0.0) + ((msk & 32) ? Q2 : 0.0);
                rc[ecol[q][e]] = fma(Gd, eeff[q][e], fk * dr - rk * dp);
            }
            rc[K] = Mq * X;
            rc[K + 1] = Mq * (fwd * k.dlf - rev * k.dlr);
            rc[K + 2] = S;
        }
        wave_sync();
        // species rows: sum of nu times the records of the species' reactions
        double A[K];
#pragma unroll
        for (int l = 0; l < K; ++l) A[l] = 0.0;
        double wd = 0.0, dt = 0.0, sq = 0.0;
#pragma unroll
        for (int e = 0; e < LM; ++e) {
            const int j = li[e] < MP ? li[e] : MP;  // lane 0's entries address the zero record
            const double *rc = sh + oRec + j * RS;
            double v[K + 3];
#pragma unroll
            for (int l = 0; l < K + 3; ++l) v[l] = rc[l];
            const double nu = lc[e];
#pragma unroll
            for (int l = 0; l < K; ++l) A[l] = fma(nu, v[l], A[l]);
            wd = fma(nu, v[K], wd);
            dt = fma(nu, v[K + 1], dt);
            sq = fma(nu, v[K + 2], sq);
        }
        double f = 0.0;
        if (spl) {
            const double Wk = sp[0];
            const double coef = 1e6 * Wk * s.irho;
            const double gk = coef * s.Wbar * (wd - sq);
            sh[oRows + r * N] = coef * (dt + (wd - sq) * s.iT);
#pragma unroll
            for (int l = 0; l < K; ++l) sh[oRows + r * N + 1 + l] = fma(Wk, A[l], gk) * tb.sp[l * kSpS + 1];
            f = coef * wd;
            sh[oExt + r] = hm * f;
            sh[oExt + N + r] = cpm * f;
        }
        wave_sync();
        // T-row entry of column r
        const int rc = (r < N) ? r : 0;
        double acc = 0.0, hf = 0.0, cf = 0.0, cps = 0.0, dcpT = 0.0;
#pragma unroll
        for (int i = 1; i <= K; ++i) {
            acc = fma(sh[oHm + i], sh[oRows + i * N + rc], acc);
            hf += sh[oExt + i];
            cf += sh[oExt + N + i];
            cps += sh[oCpt + i];
            dcpT += sh[oDcp + i];
        }
        const double icp = frcp(kR * cps);
        const double fT = -hf * icp;
        acc += (r == 0) ? cf : 0.0;
        const double dcp = (r == 0) ? dcpT : cpm;
        if (r < N) sh[oRows + r] = -fma(fT, dcp, acc) * icp;
        return (r == 0) ? fT : f;
    }

    // 16-lane maximum of an int (a DPP row is the 16 lanes of a cell): butterfly over
    // quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror and row_mirror
    __device__ __forceinline__ static int row_max(int x) {
        x = max(x, __builtin_amdgcn_update_dpp(0, x, 0xb1, 0xf, 0xf, false));
        x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x4e, 0xf, 0xf, false));
        x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, false));
        return max(x, __builtin_amdgcn_update_dpp(0, x, 0x140, 0xf, 0xf, false));
    }

    // W^-1 for W = I/(g h) - J, from J row-major in LDS.  Row-distributed Gauss-Jordan
    // elimination with partial pivoting: lane i holds row i of [W | I].  At step k the pivot is
    // the unused row of largest |W_ik|, found as a cross-lane maximum of a 32-bit key: the
    // exponent and leading 16 mantissa bits of |W_ik| with the low 4 bits replaced by 15 - i,
    // so candidates that agree to 2^-16 count as ties and go to the lowest row.  Every lane
    // forms 1/W_ik of its own row meanwhile; the pivot lane publishes its row unscaled with
    // that reciprocal, the other rows subtract multiples of it, and pivot rows are scaled at
    // the end and stored as the row of their pivot column.  On return lane r holds row r of
    // W^-1.
    __device__ static void invert(double *sh, int r, double ig, double (&winv)[N]) {
        wave_sync();
        const int rr = (r < N) ? r : 0;
        double a[N], b[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            a[c] = ((c == r) ? ig : 0.0) - sh[oRows + rr * N + c];
            b[c] = (c == r) ? 1.0 : 0.0;
        }
        bool used = (r >= N);
        int mycol = 0;
        double myinv = 1.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double inv = frcp(a[k]);
            const int hi = int(__double_as_longlong(a[k]) >> 32) & 0x7fffffff;
            const int key = row_max(used ? -1 : ((hi & ~15) | (15 - r)));
            int pk = 15 - (key & 15);
            pk = pk < N ? pk : N - 1;
            double *pr = sh + oProw + (k & 1) * (2 * N + 1);
            if (r == pk) {
#pragma unroll
                for (int c = k + 1; c < N; ++c) pr[c] = a[c];
#pragma unroll
                for (int c = 0; c < N; ++c) pr[N + c] = b[c];
                pr[k] = inv;
                used = true;
                mycol = k;
                myinv = inv;
            }
            wave_sync();
            double row[2 * N];
#pragma unroll
            for (int c = k; c < 2 * N; ++c) row[c] = pr[c];
            double f = a[k] * row[k];
            f = (r == pk || r >= N) ? 0.0 : f;
#pragma unroll
            for (int c = k + 1; c < N; ++c) a[c] = fma(-f, row[c], a[c]);
#pragma unroll
            for (int c = 0; c < N; ++c) b[c] = fma(-f, row[N + c], b[c]);
        }
        if (r < N) {
#pragma unroll
            for (int c = 0; c < N; ++c) sh[oRows + mycol * N + c] = b[c] * myinv;
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < N; ++c) winv[c] = (r < N) ? sh[oRows + r * N + c] : 0.0;
    }

    // gather the component held by lane i (i < N) into every lane
    __device__ __forceinline__ static void gather(double *buf, int r, double v, double (&out)[N]) {
        wave_sync();
        if (r < N) buf[r] = v;
        wave_sync();
#pragma unroll
        for (int c = 0; c < N; ++c) out[c] = buf[c];
    }

    // sum over lanes i < N of v (identical result in every lane)
    __device__ __forceinline__ static double lane_sum(double *buf, int r, double v) {
        wave_sync();
        if (r < N) buf[r] = v;
        wave_sync();
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < N; ++c) s += buf[c];
        return s;
    }
};

// Tables staged in LDS once per block (read by all cells of the block), and the constant
// slots of the cell regions.
template <int K, int RPL, int H = 1>
__device__ typename Coop<K, RPL, H>::Tab stage_tables(const MechDev &mg, double *lds, int lane) {
    using C = Coop<K, RPL, H>;
    constexpr int MP = C::MP;
    auto *dst = reinterpret_cast<unsigned char *>(lds);
    // copy rows x cols from a dense table to an LDS table with row stride `st`
    auto cp8 = [&](int off, const double *src, int rows, int cols, int st) {
        double *d8 = reinterpret_cast<double *>(dst + off);
        for (int q = lane; q < rows * cols; q += 64) d8[(q / cols) * st + q % cols] = src[q];
    };
    auto cp4 = [&](int off, const int *src, int rows, int cols, int st) {
        int *d4 = reinterpret_cast<int *>(dst + off);
        for (int q = lane; q < rows * cols; q += 64) d4[(q / cols) * st + q % cols] = src[q];
    };
    cp8(C::tSp, mg.sp, K, kSpTab, kSpS);
    cp8(C::tCr, mg.cr, MP, kCrDbl, kCrDbl);
    cp8(C::tEff, mg.ceff, MP, K + 4, C::EFS);
    cp8(C::tEw, mg.ceffw, MP, K, C::EWS);
    cp4(C::tCi, mg.ci, MP, kCiInt, kCiInt);
    __syncthreads();
    typename C::Tab tb;
    tb.sp = reinterpret_cast<const double *>(dst + C::tSp);
    tb.cr = reinterpret_cast<const double *>(dst + C::tCr);
    tb.eff = reinterpret_cast<const double *>(dst + C::tEff);
    tb.ew = reinterpret_cast<const double *>(dst + C::tEw);
    tb.ci = reinterpret_cast<const int *>(dst + C::tCi);
    return tb;
}

// the lane's production-rate list (index into the per-cell rate array, coefficient)
__device__ __forceinline__ void load_lists(const MechDev &mg, int r, int (&li)[kCoopList], double (&lc)[kCoopList]) {
#pragma unroll
    for (int e = 0; e < kCoopList; ++e) {
        li[e] = mg.cli[r * kCoopList + e];
        lc[e] = mg.clc[r * kCoopList + e];
    }
}

template <int K, int RPL, int H = 1>
__device__ void init_cell_region(double *sh, int r) {
    using C = Coop<K, RPL, H>;
    if (r == 0) {
        sh[C::oC] = 1.0;
        sh[C::oCpt] = 0.0;
        sh[C::oHm] = 0.0;
        sh[C::oDcp] = 0.0;
        sh[C::oQ + C::MP] = 0.0;
    }
    for (int c = r; c < C::RS; c += G) sh[C::oRec + C::MP * C::RS + c] = 0.0;
}

// State of the cell a 16-lane group is integrating: replicated in the group's lanes, except
// the lane's own component yr = y[r] and the quantities derived from it.  The group advances
// it one RODAS4 attempt at a time, so that a group whose cell is done can take another cell
// while the other groups of its wave continue.
template <int K>
struct GroupTask {
    static constexpr int N = K + 1;
    int64_t i;  // cell index
    double y[N];
    double yr, p, ip, dtc, rho0, y0own, atol, t, h, h_final;
    int acc, rej;
    bool prev_rej, fresh;
};

// Load cell i into the group (all 16 lanes).  A cell whose input is unusable (non-finite,
// p or T not positive, or a step length that is not positive and finite) gets status
// DF_CELL_NONFINITE, zero steps and zero rr, and false is returned.
template <int K>
__device__ bool group_load(const StepArgs &a, const double *sp, int r, int64_t i, GroupTask<K> &c) {
    constexpr int N = K + 1;
    c.i = i;
    c.p = a.p[i];
    c.dtc = a.dts ? a.dts[i] : a.dt;
    c.y[0] = a.T[i];
#pragma unroll
    for (int k = 0; k < K; ++k) c.y[1 + k] = a.Y[k * a.ld + i];
    bool ok = isfinite(c.p) && c.p > 0.0 && isfinite(c.y[0]) && c.y[0] > 0.0 && isfinite(c.dtc) && c.dtc > 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) ok = ok && isfinite(c.y[1 + k]);
    if (!ok) {
        if (r == 0) {
            if (a.status) a.status[i] = DF_CELL_NONFINITE;
            if (a.nsteps) {
                a.nsteps[i] = 0;
                a.nsteps[a.n + i] = 0;
            }
        }
        if (a.rr && r >= 1 && r <= K) a.rr[(r - 1) * a.ld + i] = 0.0;
        if (a.tape && r == 0) Tape(K, a.n, a.tape_cap).count(a.tape)[i] = -1;
        return false;
    }
    c.ip = 1.0 / c.p;
    c.yr = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) c.yr = (q == r) ? c.y[q] : c.yr;
    c.y0own = (r >= 1 && r <= K) ? c.yr : 0.0;
    c.rho0 = 0.0;
    if (a.rr) {  // input density, for rr
        double sYW = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) sYW += c.y[1 + k] * sp[k * kSpS + 1];
        c.rho0 = c.p / (sYW * kR * c.y[0]);
    }
    c.atol = (r == 0) ? a.o.atol_T : a.o.atol_Y;
    const double h_in = a.h_io ? a.h_io[i] : 0.0;
    c.fresh = !(h_in > 0.0);
    c.h = c.fresh ? 0.0 : fmin(h_in, c.dtc);
    if (!c.fresh && !(c.h >= a.o.h_min)) c.h = a.o.h_min;
    c.t = 0.0;
    c.h_final = 0.0;
    c.acc = c.rej = 0;
    c.prev_rej = false;
    return true;
}

// write the results of the group's cell: lane 0 the scalars, lanes 1..K their species
template <int K>
__device__ void group_finish(const StepArgs &a, int r, const GroupTask<K> &c, int st) {
    const int64_t i = c.i;
    if (a.tape) {
        // a cell whose accepted sub-steps did not all fit keeps its result but has no tape
        if (st == DF_CELL_OK && c.acc > a.tape_cap) st = DF_CELL_TAPE_FULL;
        if (r == 0) Tape(K, a.n, a.tape_cap).count(a.tape)[i] = (st == DF_CELL_OK) ? c.acc : -1;
    }
    if (r == 0) {
        a.T[i] = c.y[0];
        if (a.h_io) a.h_io[i] = (st == DF_CELL_OK) ? c.h_final : c.h;
        if (a.status) a.status[i] = (st == DF_CELL_OK) ? a.status_ok : st;
        if (a.nsteps) {
            a.nsteps[i] = c.acc;
            a.nsteps[a.n + i] = c.rej;
        }
    } else if (r <= K) {
        if (a.rr) a.rr[(r - 1) * a.ld + i] = c.rho0 * (c.yr - c.y0own) / c.dtc;
        a.Y[(r - 1) * a.ld + i] = c.yr;
    }
}

// One RODAS4 attempt of the group's cell (the first attempt of a cell without a step hint
// also picks the initial step from f(y0)).  Returns true when the cell is done and its
// results have been written.
template <int K, int RPL, int H = 1>
__device__ bool group_attempt(const StepArgs &a, const typename Coop<K, RPL, H>::Tab &tb, double *sh, int r, int rl,
                              const int (&li)[kCoopList], const double (&lc)[kCoopList], GroupTask<K> &c) {
    using C = Coop<K, RPL, H>;
    constexpr int N = K + 1;
    const Opts &o = a.o;
    if (c.acc + c.rej >= o.max_steps) {
        group_finish<K>(a, r, c, DF_CELL_MAX_STEPS);
        return true;
    }
    const double f0 = C::jacobian(tb, sh, r, rl, c.p, c.ip, c.y, c.yr, li, lc);
    if (c.fresh) {
        // initial sub-step from the weighted norms of y0 and f(y0)
        const double sc = c.atol + o.rtol * fabs(c.yr);
        const double ny = sqrt(C::lane_sum(sh + C::oRed, r, (c.yr / sc) * (c.yr / sc)) / N);
        const double nf = sqrt(C::lane_sum(sh + C::oRed + N, r, (f0 / sc) * (f0 / sc)) / N);
        c.h = (nf > 0.0) ? fmin(0.01 * ny / nf, c.dtc) : c.dtc;
        if (!(c.h >= o.h_min)) c.h = o.h_min;
        c.fresh = false;
    }
    const bool last = (c.t + c.h >= c.dtc);
    const double ht = last ? c.dtc - c.t : c.h;
    double winv[N];
    C::invert(sh, r, 1.0 / (Rodas4::g * ht), winv);

    // own components: stage vectors u_s[r]
    double u[6], ysr = c.yr;
    const double ih = 1.0 / ht;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        double fs;
        if (s == 0) {
            fs = f0;
        } else {
            ysr = c.yr;
#pragma unroll
            for (int j = 0; j < s; ++j) ysr = fma(Rodas4::a[s][j], u[j], ysr);
            double ys[N];
            C::gather(sh + C::oVec, r, ysr, ys);
            fs = C::rhs(tb, sh, r, rl, c.p, c.ip, ys, ysr, li, lc);
        }
        double cu = 0.0;
#pragma unroll
        for (int j = 0; j < s; ++j) cu = fma(Rodas4::c[s][j], u[j], cu);
        double rv[N];
        C::gather(sh + C::oVec2, r, fma(cu, ih, fs), rv);
        double us = 0.0;
#pragma unroll
        for (int q = 0; q < N; ++q) us = fma(winv[q], rv[q], us);
        u[s] = us;
    }
    // y_new = (stage-6 state) + u6 ; error = u6
    const double ynr = ysr + u[5];
    const double sc = c.atol + o.rtol * fmax(fabs(c.yr), fabs(ynr));
    const double er = (r < N) ? u[5] / sc : 0.0;
    const double err = sqrt(C::lane_sum(sh + C::oRed + 2 * N, r, er * er) / N);

    const double fmx = c.prev_rej ? 1.0 : 6.0;
    double fac;
    if (!isfinite(err))
        fac = 0.2;
    else if (err == 0.0)
        fac = fmx;
    else
        fac = fmin(fmx, fmax(0.2, 0.9 / sqrt(sqrt(err))));  // 0.9 err^(-1/4)

    if (isfinite(err) && err <= 1.0) {
        if (a.tape && c.acc < a.tape_cap && r < N) {
            // the accepted sub-step for the adjoint: lane r's component of the start state, its
            // row of W^-1 and its components of the stage vectors
            const Tape tp(K, a.n, a.tape_cap);
            const int64_t s = c.acc;
            a.tape[tp.y(s, r) + c.i] = c.yr;
            if (r == 0) a.tape[tp.h(s) + c.i] = ht;
#pragma unroll
            for (int q = 0; q < N; ++q) a.tape[tp.w(s, r * N + q) + c.i] = winv[q];
#pragma unroll
            for (int si = 0; si < 6; ++si) a.tape[tp.u(s, si * N + r) + c.i] = u[si];
        }
        ++c.acc;
        C::gather(sh + C::oVec, r, ynr, c.y);
        c.yr = (r < N) ? ynr : 0.0;
        c.h_final = c.h;
        c.prev_rej = false;
        if (last) {
            group_finish<K>(a, r, c, DF_CELL_OK);
            return true;
        }
        c.t += ht;
        c.h = ht * fac;
    } else {
        ++c.rej;
        c.prev_rej = true;
        c.h = ht * fac;
        if (c.h < o.h_min) {
            group_finish<K>(a, r, c, DF_CELL_H_UNDERFLOW);
            return true;
        }
    }
    return false;
}

// Static schedule: the block's cells are the slots slot0, slot0 + 1, ... (four 16-lane or two
// 32-lane cells per block), and slot s is cell cidx[s] (or s).
template <int K, int RPL, int H>
__device__ __forceinline__ void coop_static_block(const MechDev &mg, const StepArgs &a, const CellQueue &q,
                                                  int64_t slot0, double *lds) {
    using C = Coop<K, RPL, H>;
    const int lane = threadIdx.x;
    const int r = lane & (G - 1);        // row of the cell held by the lane (both halves)
    const int rl = lane & (C::GL - 1);   // lane within the cell
    const int64_t limit = q.dcount ? int64_t(*q.dcount) : a.n;
    if (slot0 >= limit) return;  // whole block idle (e.g. no fallback cells)
    const typename C::Tab tb = stage_tables<K, RPL, H>(mg, lds, lane);
    double *sh = lds + C::tBytes / 8 + (lane / C::GL) * C::kStride;
    const int64_t slot = slot0 + lane / C::GL;
    if (slot >= limit) return;  // the lanes of a cell leave together
    init_cell_region<K, RPL, H>(sh, r);
    int li[kCoopList];
    double lc[kCoopList];
    load_lists(mg, r, li, lc);
    GroupTask<K> c;
    bool have = group_load<K>(a, tb.sp, r, q.cidx ? int64_t(q.cidx[slot]) : slot, c);
    while (have) have = !group_attempt<K, RPL, H>(a, tb, sh, r, rl, li, lc, c);
}

template <int K, int RPL, int H>
__global__ __launch_bounds__(64) void chem_coop_kernel(MechDev mg, StepArgs a, CellQueue q) {
    extern __shared__ double lds[];
    coop_static_block<K, RPL, H>(mg, a, q, int64_t(blockIdx.x) * Coop<K, RPL, H>::CPB, lds);
}

// Static schedule with a 32-lane head: blocks [0, head_blocks) take the first 2 head_blocks slots of
// the cost order as 32-lane cells, the other blocks the rest as 16-lane cells.  The head of the
// order holds the stiffest cells, whose chains of sub-steps set the launch's time; an attempt
// costs less at 32 lanes, while the bulk keeps the layout that needs half as many waves.  The
// two layouts give the same results bit for bit.
template <int K, int RPL>
__global__ __launch_bounds__(64) void chem_coop_head_kernel(MechDev mg, StepArgs a, CellQueue q, int head_blocks) {
    extern __shared__ double lds[];
    constexpr int C2 = Coop<K, RPL, 2>::CPB, C1 = Coop<K, RPL, 1>::CPB;
    const int b = int(blockIdx.x);
    if (b < head_blocks)
        coop_static_block<K, RPL, 2>(mg, a, q, int64_t(b) * C2, lds);
    else
        coop_static_block<K, RPL, 1>(mg, a, q, int64_t(head_blocks) * C2 + int64_t(b - head_blocks) * C1, lds);
}

// Queue schedule: a persistent grid.  Blocks [0, head_blocks) run four 16-lane groups that
// take the most expensive cells from the front of the queue.  The other blocks first run one
// cell per lane on the cold cells at the back, then join the front claims as 16-lane groups.
// A group or lane that finishes a cell claims the next one at once, until the queue is empty.
// LANES = false compiles the 16-lane body alone (every block starts as 16-lane groups), so
// that it keeps the registers of the static kernel.
template <int K, int RPL, bool LANES>
__global__ __launch_bounds__(64) void chem_queue_kernel(MechDev mg, StepArgs a, CellQueue q) {
    using C = Coop<K, RPL>;
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    if (LANES && int(blockIdx.x) >= q.head_blocks) {
        using L = Cell<K>;
        double *sh = lds + lane;  // per-lane arrays, slot-major with a stride of one wave
        L::init_lds(sh);
        LaneTask<K> c;
        auto next = [&]() -> bool {
            for (;;) {
                const int64_t i = queue_claim(q, a.n, false);
                if (i < 0) return false;
                if (lane_load<K>(a, i, c)) return true;
            }
        };
        bool have = next();
        while (have)
            if (lane_attempt<K>(mg, a, sh, c)) have = next();
        __syncthreads();  // the per-lane arrays are dead before the tables overwrite them
    }
    const int r = lane & (G - 1);
    const typename C::Tab tb = stage_tables<K, RPL>(mg, lds, lane);
    double *sh = lds + C::tBytes / 8 + (lane / G) * C::kStride;
    init_cell_region<K, RPL>(sh, r);
    auto *claim = reinterpret_cast<long long *>(sh + C::oClaim);
    int li[kCoopList];
    double lc[kCoopList];
    load_lists(mg, r, li, lc);
    GroupTask<K> c;
    auto next = [&]() -> bool {
        for (;;) {
            if (r == 0) *claim = queue_claim(q, a.n, true);
            wave_sync();
            const int64_t i = *claim;
            wave_sync();
            if (i < 0) return false;
            if (group_load<K>(a, tb.sp, r, i, c)) return true;
        }
    };
    bool have = next();
    while (have)
        if (group_attempt<K, RPL>(a, tb, sh, r, r, li, lc, c)) have = next();
}

}  // namespace

#define DF_COOP_SPECIES_LIST(X) X(2) X(4) X(9)

template <int K, int RPL>
static size_t coop_lds_bytes() {
    return Coop<K, RPL>::lds_bytes();
}

static size_t coop_lds_for(int K, int RPL) {
    switch (K) {
#define DF_CASE(k)                                            \
    case k:                                                   \
        switch (RPL) {                                        \
            case 1: return coop_lds_bytes<k, 1>();            \
            case 2: return coop_lds_bytes<k, 2>();            \
            case 3: return coop_lds_bytes<k, 3>();            \
            case 4: return coop_lds_bytes<k, 4>();            \
            default: return 0;                                \
        }
        DF_COOP_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return 0;
    }
}

constexpr size_t kCoopMaxLds = 64 * 1024;

bool chem_coop_supported(const MechDev &m) {
    if (m.RPL < 1 || m.RPL > kMaxRPL || m.lmax > kCoopList) return false;
    const size_t b = coop_lds_for(m.K, m.RPL);
    return b > 0 && b <= kCoopMaxLds;
}

template <int K, int RPL, int H>
static df_status launch_coop_kh(const MechDev &m, const StepArgs &a, const CellQueue &q, hipStream_t stream) {
    constexpr int cpb = Coop<K, RPL, H>::CPB;
    const int64_t blocks = (a.n + cpb - 1) / cpb;
    if (blocks > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "chem_step: too many cells for one launch");
    const size_t lds = Coop<K, RPL, H>::lds_bytes();
    hipLaunchKernelGGL((chem_coop_kernel<K, RPL, H>), dim3(unsigned(blocks)), dim3(64), lds, stream, m, a, q);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("chem_step launch: ") + hipGetErrorString(e));
    return DF_OK;
}

// cells of the cost order's head that the head variant runs at 32 lanes (the hot-kernel field's
// cells within half of the longest chain of sub-steps are its 538 hottest)
constexpr int64_t kCoopHeadCells = 512;

template <int K, int RPL>
static df_status launch_coop_head(const MechDev &m, const StepArgs &a, const CellQueue &q, hipStream_t stream) {
    using C1 = Coop<K, RPL, 1>;
    using C2 = Coop<K, RPL, 2>;
    const int64_t head = a.n < kCoopHeadCells ? a.n : kCoopHeadCells;
    const int64_t hb = (head + C2::CPB - 1) / C2::CPB;
    const int64_t rest = a.n - hb * C2::CPB;
    const int64_t blocks = hb + (rest > 0 ? (rest + C1::CPB - 1) / C1::CPB : 0);
    if (blocks > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "chem_step: too many cells for one launch");
    const size_t lds = C1::lds_bytes() > C2::lds_bytes() ? C1::lds_bytes() : C2::lds_bytes();
    hipLaunchKernelGGL((chem_coop_head_kernel<K, RPL>), dim3(unsigned(blocks)), dim3(64), lds, stream, m, a, q,
                       int(hb));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("chem_step launch: ") + hipGetErrorString(e));
    return DF_OK;
}

// halves: 1 = 16-lane cells, 2 = 32-lane cells, 3 = 32-lane cells for the head of the cost order
// and 16-lane cells for the rest.  32 lanes only where the reaction slots divide between two
// halves; the taped step keeps the 16-lane layout of the adjoint's tape writer, and the head
// variant needs the cost order (and no fallback list)
template <int K, int RPL>
static df_status launch_coop_k(const MechDev &m, const StepArgs &a, const CellQueue &q, hipStream_t stream,
                               int halves) {
    if constexpr (RPL % 2 == 0) {
        if (halves == 2 && !a.tape) return launch_coop_kh<K, RPL, 2>(m, a, q, stream);
        if (halves == 3 && !a.tape && q.cidx && !q.dcount &&
            Coop<K, RPL, 1>::lds_bytes() <= kCoopMaxLds && Coop<K, RPL, 2>::lds_bytes() <= kCoopMaxLds)
            return launch_coop_head<K, RPL>(m, a, q, stream);
    }
    return launch_coop_kh<K, RPL, 1>(m, a, q, stream);
}

// LDS of the persistent kernel: the larger of the two bodies
template <int K, int RPL>
static size_t queue_lds_bytes() {
    const size_t lane = size_t(Cell<K>::kRows) * 64 * sizeof(double);
    const size_t coop = Coop<K, RPL>::lds_bytes();
    return lane > coop ? lane : coop;
}

// blocks resident at once: the smaller count of the two variants, so that one grid size fits both
template <int K, int RPL>
static int32_t queue_capacity_k() {
    int dev = 0, cus = 0, a = 0, b = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, chem_queue_kernel<K, RPL, true>, 64,
                                                     queue_lds_bytes<K, RPL>()) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, chem_queue_kernel<K, RPL, false>, 64,
                                                     Coop<K, RPL>::lds_bytes()) != hipSuccess)
        return 0;
    return int32_t(cus) * int32_t(a < b ? a : b);
}

template <int K, int RPL>
static df_status launch_queue_k(const MechDev &m, const StepArgs &a, const CellQueue &q, int32_t blocks,
                                hipStream_t stream) {
    if (q.head_blocks >= blocks) {
        const size_t lds = Coop<K, RPL>::lds_bytes();
        hipLaunchKernelGGL((chem_queue_kernel<K, RPL, false>), dim3(unsigned(blocks)), dim3(64), lds, stream, m, a,
                           q);
    } else {
        const size_t lds = queue_lds_bytes<K, RPL>();
        hipLaunchKernelGGL((chem_queue_kernel<K, RPL, true>), dim3(unsigned(blocks)), dim3(64), lds, stream, m, a,
                           q);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("chem_step queue launch: ") + hipGetErrorString(e));
    return DF_OK;
}

#define DF_RPL_SWITCH(k, CALL)                 \
    switch (m.RPL) {                           \
        case 1: return CALL(k, 1);             \
        case 2: return CALL(k, 2);             \
        case 3: return CALL(k, 3);             \
        default: return CALL(k, 4);            \
    }

df_status launch_chem_coop(const MechDev &m, const StepArgs &a, const CellQueue &q, hipStream_t stream,
                           int halves) {
    if (a.n == 0) return DF_OK;
    if (!chem_coop_supported(m))
        return fail(DF_E_UNSUPPORTED, "chem_step: no cooperative kernel for " + std::to_string(m.K) + " species, " +
                                          std::to_string(m.M) + " reactions (needs K in {2, 4, 9}, M <= 64, at most " +
                                          std::to_string(kCoopList) + " reactions per species)");
#define DF_CALL(k, rpl) launch_coop_k<k, rpl>(m, a, q, stream, halves)
    switch (m.K) {
#define DF_CASE(k)              \
    case k:                     \
        DF_RPL_SWITCH(k, DF_CALL)
        DF_COOP_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return fail(DF_E_UNSUPPORTED, "chem_step: no cooperative kernel for " + std::to_string(m.K) + " species");
    }
#undef DF_CALL
}

int32_t chem_queue_capacity(const MechDev &m) {
    if (!chem_coop_supported(m)) return 0;
#define DF_CALL(k, rpl) queue_capacity_k<k, rpl>()
    switch (m.K) {
#define DF_CASE(k)              \
    case k:                     \
        DF_RPL_SWITCH(k, DF_CALL)
        DF_COOP_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return 0;
    }
#undef DF_CALL
}

df_status launch_chem_queue(const MechDev &m, const StepArgs &a, const CellQueue &q, int32_t blocks,
                            hipStream_t stream) {
    if (a.n == 0) return DF_OK;
    if (blocks <= 0 || !chem_coop_supported(m))
        return fail(DF_E_UNSUPPORTED, "chem_step: no persistent kernel for this mechanism");
#define DF_CALL(k, rpl) launch_queue_k<k, rpl>(m, a, q, blocks, stream)
    switch (m.K) {
#define DF_CASE(k)              \
    case k:                     \
        DF_RPL_SWITCH(k, DF_CALL)
        DF_COOP_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return fail(DF_E_UNSUPPORTED, "chem_step: no persistent kernel for " + std::to_string(m.K) + " species");
    }
#undef DF_CALL
}
#undef DF_RPL_SWITCH

}  // namespace df
