// One cell per lane: the per-lane RODAS4 solver shared by the one-cell-per-lane
// launch (df_chem.hip) and the mixed persistent launch (df_chem_coop.hip).
//
// Each lane integrates the constant-pressure adiabatic reactor of its cell,
//   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k h_k dY_k/dt / cp
// (the species source term of the paper's Sec. "Chemistry Integration", with
// the density written out), with the L-stable Rosenbrock method RODAS4
// (Hairer & Wanner, Solving ODEs II, Sec. IV.7, transformed form) and an
// embedded error estimate.  The solver is table-driven: the species and
// reaction tables live in one read-only allocation and are read with
// wave-uniform indices, so they arrive through the scalar cache as SGPR
// operands; per-lane state (y, Jacobian/LU, stage vectors) stays in
// registers.  Per-species arrays are indexed 1..K with index 0 a neutral
// element, so a reaction side with fewer than three molecules needs no
// branch.
#pragma once

#include <cmath>

#include "df_internal.h"
#include "df_kinetics.h"

namespace df {
namespace {

// Per-lane species arrays live in LDS, slot-major with a stride of one wave
// (element k of lane l at sh[k * 64 + l]): a gather with a wave-uniform species
// index is then a single conflict-free ds_read_b64 instead of a select chain
// over registers.  Slot 0 of each array is the neutral element.
constexpr int kWave = 64;

// CV: the constant-volume reactor (the df0DFoam constant-volume case): the density is an input
// (passed where the pressure is otherwise), dT/dt = -sum_k U_k wdot_k / (rho cv) with
// U_k = H_k - R T and cv = cp - R / Wbar, and the concentrations do not depend on T or Wbar.
template <int K, bool CV = false>
struct Cell {
    static constexpr int N = K + 1;
    // LDS slot offsets (in units of one wave-wide row of doubles).  The Jacobian-only
    // arrays (H/RT, dq/dc) overlay the stage vectors u0..u3, which are dead while the
    // Jacobian is formed.
    static constexpr int kC = 0;       // concentrations, mol/cm^3; [0] = 1
    static constexpr int kE = N;       // exp(-G_k/RT); [0] = 1
    static constexpr int kIE = 2 * N;  // exp(+G_k/RT); [0] = 1
    static constexpr int kU = 3 * N;   // stage vectors u0..u3 (N each)
    static constexpr int kH = 3 * N;   // H_k/RT; [0] = 0   (Jacobian phase only)
    static constexpr int kDQ = 4 * N;  // dq/dc scatter target (Jacobian phase only)
    static constexpr int kULds = 4;    // stage vectors kept in LDS; the rest stay in registers
    static constexpr int kRows = 3 * N + kULds * N;

    __device__ __forceinline__ static double &at(double *sh, int slot) { return sh[slot * kWave]; }

    struct Mix {
        double T, iT, lT;
        double rho, Wbar, cp;  // kg/m^3, kg/mol, J/kg/K (cv for the constant-volume reactor)
        double cref, icref;    // p0/(RT) in mol/cm^3 and its inverse
    };

    // thermo of every species and the mixture at (T, Y); fills the LDS arrays c, e, ie
    // (H/RT and cp/R are returned in registers: the H rows overlay stage vector u0)
    __device__ __forceinline__ static void state(const MechDev &m, double p, const double (&y)[N], double *sh,
                                                 Mix &s, double (&cpR)[N], double (&hRT)[N]) {
        const double T = y[0];
        s.T = T;
        s.iT = 1.0 / T;
        s.lT = log(T);
        double sYW = 0.0, cpm = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double *r = m.sp + k * kSpTab;
            const double cp = r[2] + T * (r[3] + T * (r[4] + T * (r[5] + T * r[6])));
            const double h = r[2] + T * (r[9] + T * (r[10] + T * (r[11] + T * r[12]))) + r[7] * s.iT;
            const double sr = r[2] * s.lT + T * (r[3] + T * (r[13] + T * (r[14] + T * r[15]))) + r[8];
            cpR[1 + k] = cp;
            hRT[1 + k] = h;
            const double ek = exp(sr - h);
            at(sh, kE + 1 + k) = ek;
            at(sh, kIE + 1 + k) = 1.0 / ek;
            sYW += y[1 + k] * r[1];
            cpm += y[1 + k] * cp * r[1];
        }
        s.Wbar = 1.0 / sYW;
        s.rho = CV ? p : p * s.Wbar * s.iT * (1.0 / kR);
        s.cp = CV ? (cpm - sYW) * kR : cpm * kR;
        const double cfac = 1e-6 * s.rho;
#pragma unroll
        for (int k = 0; k < K; ++k) at(sh, kC + 1 + k) = cfac * y[1 + k] * m.sp[k * kSpTab + 1];
        cpR[0] = 0.0;
        hRT[0] = 0.0;
        s.cref = 1e-6 * kPref * s.iT * (1.0 / kR);
        s.icref = 1.0 / s.cref;
    }

    // neutral slots, written once per kernel
    __device__ __forceinline__ static void init_lds(double *sh) {
        at(sh, kC) = 1.0;
        at(sh, kE) = 1.0;
        at(sh, kIE) = 1.0;
    }

    template <bool DERIV>
    __device__ __forceinline__ static double kforward(const double *rd, int type, const Mix &s, double Mc,
                                                      double &dlnkf, double &dkfdM) {
        return rate_constant<DERIV>(rd, type, s.T, s.iT, s.lT, Mc, dlnkf, dkfdM);
    }

    __device__ __forceinline__ static double third_body(const MechDev &m, int j, double *sh) {
        const double *ef = m.eff + j * K;
        double Mc = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) Mc = fma(ef[k], at(sh, kC + 1 + k), Mc);
        return Mc;
    }

    // f(y)
    __device__ __forceinline__ static void rhs(const MechDev &m, double p, const double (&y)[N], double *sh,
                                               double (&f)[N]) {
        Mix s;
        double cpR[N], hRT[N];
        state(m, p, y, sh, s, cpR, hRT);
        double wd[N];
#pragma unroll
        for (int k = 0; k < N; ++k) wd[k] = 0.0;
        for (int j = 0; j < m.M; ++j) {
            const int *ri = m.rx + j * kRxInt;
            const double *rd = m.rk + j * kRxDbl;
            const int type = ri[0];
            const int r0 = ri[1], r1 = ri[2], r2 = ri[3], p0 = ri[4], p1 = ri[5], p2 = ri[6], dnu = ri[7];
            const double Mc = (type != 0) ? third_body(m, j, sh) : 0.0;
            double dl, dm;
            const double kf = kforward<false>(rd, type, s, Mc, dl, dm);
            const double iKc = at(sh, kE + r0) * at(sh, kE + r1) * at(sh, kE + r2) * at(sh, kIE + p0) *
                               at(sh, kIE + p1) * at(sh, kIE + p2) * cref_pow(s.cref, s.icref, dnu);
            const double fwd = kf * (at(sh, kC + r0) * at(sh, kC + r1) * at(sh, kC + r2));
            const double rev = kf * iKc * (at(sh, kC + p0) * at(sh, kC + p1) * at(sh, kC + p2));
            double q = fwd - rev;
            if (type == 1) q *= Mc;
            const int *nuj = m.nu + j * K;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int nk = nuj[k];
                if (nk != 0) wd[1 + k] = fma(double(nk), q, wd[1 + k]);
            }
        }
        const double fy = 1e6 / s.rho;
        double hsum = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            f[1 + k] = fy * m.sp[k * kSpTab] * wd[1 + k];
            hsum = fma(CV ? hRT[1 + k] - 1.0 : hRT[1 + k], wd[1 + k], hsum);  // U/RT = H/RT - 1
        }
        f[0] = -hsum * (1e6 * kR) * s.T / (s.rho * s.cp);
    }

    // Analytic Jacobian J = df/dy and f(y).  Reaction derivatives are taken in
    // concentration space (A_kl = sum_j nu_kj dq_j/dc_l, s_k = sum_j nu_kj sum_m c_m dq_j/dc_m,
    // dT_k = sum_j nu_kj dq_j/dT at fixed c), then mapped to (T, Y) with
    //   dc_m/dY_l = 1e-6 rho delta_ml / W_m - c_m Wbar / W_l,   dc_m/dT = -c_m / T.
    // A is accumulated in the species block of J (row/column 1 + k) by rows with
    // compile-time indices and wave-uniform stoichiometric coefficients, so J stays in
    // registers; the T row and column are filled afterwards.
    // With kLnA (the adjoint's products with df/dlnA) it also writes, per reaction j,
    // q_j d ln kf_j / d ln A_j to lna[j * kWave] (for a falloff row the part of q_j that goes
    // through Pr = k0 [M] / k_inf, G_j [M], is taken off), and the two mixture factors of the
    // weights of wd_k in f_k and f_T: mix[0] = fy = 1e6 / rho and mix[1] = fy R T / cp, so that
    // f_k weighs wd_k by fy W_k and f_T by -mix[1] H_k/RT (the H/RT rows stay in sh).
    template <bool kLnA = false>
    __device__ __forceinline__ static void jacobian(const MechDev &m, double p, const double (&y)[N], double *sh,
                                                    double (&J)[N][N], double (&f)[N], double *lna = nullptr,
                                                    double *mix = nullptr) {
        Mix s;
        double cpR[N], hRT[N];
        state(m, p, y, sh, s, cpR, hRT);
#pragma unroll
        for (int k = 0; k < N; ++k) at(sh, kH + k) = hRT[k];  // u0 is dead while J is formed
        double wd[N], sq[N], dt[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            wd[k] = sq[k] = dt[k] = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) J[k][l] = 0.0;
        }
        for (int j = 0; j < m.M; ++j) {
            const int *ri = m.rx + j * kRxInt;
            const double *rd = m.rk + j * kRxDbl;
            const int type = ri[0];
            const int r0 = ri[1], r1 = ri[2], r2 = ri[3], p0 = ri[4], p1 = ri[5], p2 = ri[6], dnu = ri[7];
            const double nr = rd[10], np = rd[11];
            const double Mc = (type != 0) ? third_body(m, j, sh) : 0.0;
            double dlnkf, dkfdM;
            const double kf = kforward<true>(rd, type, s, Mc, dlnkf, dkfdM);
            const double iKc = at(sh, kE + r0) * at(sh, kE + r1) * at(sh, kE + r2) * at(sh, kIE + p0) *
                               at(sh, kIE + p1) * at(sh, kIE + p2) * cref_pow(s.cref, s.icref, dnu);
            const double kr = kf * iKc;
            const double c0 = at(sh, kC + r0), c1 = at(sh, kC + r1), c2 = at(sh, kC + r2);
            const double d0 = at(sh, kC + p0), d1 = at(sh, kC + p1), d2 = at(sh, kC + p2);
            const double Pf = c0 * c1 * c2, Pb = d0 * d1 * d2;
            const double fwd = kf * Pf, rev = kr * Pb, X = fwd - rev;
            const double dlnKc = (at(sh, kH + p0) + at(sh, kH + p1) + at(sh, kH + p2) - at(sh, kH + r0) -
                                  at(sh, kH + r1) - at(sh, kH + r2) - dnu) *
                                 s.iT;
            const double dXdT = fwd * dlnkf - rev * (dlnkf - dlnKc);
            const double Mq = (type == 1) ? Mc : 1.0;
            const double q = Mq * X;
            const double dqdT = Mq * dXdT;
            double S = Mq * (nr * fwd - np * rev);
            double G = 0.0;  // coefficient of the dense third-body term eff_l * G
            if (type == 1) {
                G = X;
                S += Mc * X;
            } else if (type == 2) {
                G = dkfdM * (Pf - Pb * iKc);
                S += G * Mc;
            }
            if constexpr (kLnA) lna[j * kWave] = (type == 2) ? q - G * Mc : q;
            // dq/dc: the slot terms (each slot's derivative is the product of the other slots)
            // are scattered into LDS, the dense third-body term is added on the way out;
            // slot 0 collects the empty slots
            const double *ef = m.eff + j * K;
#pragma unroll
            for (int l = 0; l < N; ++l) at(sh, kDQ + l) = 0.0;
            at(sh, kDQ + r0) += Mq * kf * c1 * c2;
            at(sh, kDQ + r1) += Mq * kf * c0 * c2;
            at(sh, kDQ + r2) += Mq * kf * c0 * c1;
            at(sh, kDQ + p0) -= Mq * kr * d1 * d2;
            at(sh, kDQ + p1) -= Mq * kr * d0 * d2;
            at(sh, kDQ + p2) -= Mq * kr * d0 * d1;
            double dq[K];
#pragma unroll
            for (int l = 0; l < K; ++l) dq[l] = (type != 0) ? fma(G, ef[l], at(sh, kDQ + 1 + l)) : at(sh, kDQ + 1 + l);
            const int *nuj = m.nu + j * K;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int nk = nuj[k];
                if (nk == 0) continue;  // wave-uniform branch
                const double sg = double(nk);
#pragma unroll
                for (int l = 0; l < K; ++l) J[1 + k][1 + l] = fma(sg, dq[l], J[1 + k][1 + l]);
                sq[1 + k] = fma(sg, S, sq[1 + k]);
                dt[1 + k] = fma(sg, dqdT, dt[1 + k]);
                wd[1 + k] = fma(sg, q, wd[1 + k]);
            }
        }
        // species rows
        double hm[N], cpm[N];
        const double fy = 1e6 / s.rho;
        double dcpdT = 0.0, hf = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double *r = m.sp + k * kSpTab;
            const double Wk = r[0];
            const int row = 1 + k;
            const double coef = fy * Wk;
            // at constant pressure c depends on T and Wbar (dc_m/dT = -c_m/T, and the Wbar term);
            // at constant volume it does not
            const double gk = CV ? 0.0 : coef * s.Wbar * (wd[row] - sq[row]);
            J[row][0] = CV ? coef * dt[row] : coef * (dt[row] + (wd[row] - sq[row]) * s.iT);
#pragma unroll
            for (int l = 0; l < K; ++l) {
                const double iWl = m.sp[l * kSpTab + 1];
                J[row][1 + l] = (Wk * J[row][1 + l] + gk) * iWl;
            }
            f[row] = coef * wd[row];
            hm[row] = (CV ? hRT[row] - 1.0 : hRT[row]) * kR * s.T * r[1];  // J/kg: h_k, or u_k
            cpm[row] = (CV ? cpR[row] - 1.0 : cpR[row]) * kR * r[1];       // J/kg/K: cp_k, or cv_k
            dcpdT += y[row] * (r[3] + s.T * (r[16] + s.T * (r[17] + s.T * r[18]))) * kR * r[1];
            hf += hm[row] * f[row];
        }
        const double icp = 1.0 / s.cp;
        f[0] = -hf * icp;
        if constexpr (kLnA) {
            mix[0] = fy;
            mix[1] = fy * kR * s.T * icp;
        }
        // temperature row: f_T = -sum_k h_k f_k / cp (u_k and cv at constant volume)
#pragma unroll
        for (int l = 0; l < N; ++l) {
            double acc = 0.0;
#pragma unroll
            for (int k = 1; k < N; ++k) acc += hm[k] * J[k][l];
            const double dcp = (l == 0) ? dcpdT : cpm[l];
            if (l == 0) {
#pragma unroll
                for (int k = 1; k < N; ++k) acc += cpm[k] * f[k];
            }
            J[0][l] = -(acc + f[0] * dcp) * icp;
        }
    }

    // In-place LU with partial pivoting (largest magnitude, ties to the lowest row);
    // row exchanges are done with selects so the matrix stays in registers.  The
    // diagonal holds 1/U_kk on return.
    __device__ __forceinline__ static void lu(double (&A)[N][N], int (&piv)[N]) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            int pk = k;
            if (k < N - 1) {
                double best = fabs(A[k][k]);
#pragma unroll
                for (int r = k + 1; r < N; ++r) {
                    const double v = fabs(A[r][k]);
                    const bool gt = v > best;
                    best = gt ? v : best;
                    pk = gt ? r : pk;
                }
#pragma unroll
                for (int r = k + 1; r < N; ++r) {
                    const bool sw = (pk == r);
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        const double a = A[k][c], b = A[r][c];
                        A[k][c] = sw ? b : a;
                        A[r][c] = sw ? a : b;
                    }
                }
            }
            piv[k] = pk;
            const double inv = 1.0 / A[k][k];
            A[k][k] = inv;
#pragma unroll
            for (int r = k + 1; r < N; ++r) {
                const double l = A[r][k] * inv;
                A[r][k] = l;
#pragma unroll
                for (int c = k + 1; c < N; ++c) A[r][c] = fma(-l, A[k][c], A[r][c]);
            }
        }
    }

    __device__ __forceinline__ static void solve(const double (&A)[N][N], const int (&piv)[N], double (&b)[N]) {
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
#pragma unroll
            for (int r = k + 1; r < N; ++r) {
                const bool sw = (piv[k] == r);
                const double a = b[k], c = b[r];
                b[k] = sw ? c : a;
                b[r] = sw ? a : c;
            }
        }
#pragma unroll
        for (int i = 1; i < N; ++i)
#pragma unroll
            for (int j = 0; j < i; ++j) b[i] = fma(-A[i][j], b[j], b[i]);
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
#pragma unroll
            for (int j = i + 1; j < N; ++j) b[i] = fma(-A[i][j], b[j], b[i]);
            b[i] *= A[i][i];
        }
    }
};

// State of the cell a lane is integrating.  The solver advances it one RODAS4
// attempt at a time, so that a lane whose cell is done can take another cell
// while the other lanes of its wave continue.
template <int K>
struct LaneTask {
    static constexpr int N = K + 1;
    int64_t i;  // cell index
    double y[N];
    double p, dtc, t, h, h_final;
    int acc, rej;
    bool prev_rej, fresh;
};

// Load cell i.  A cell whose input is unusable (non-finite, p or T not positive, or a
// step length that is not positive and finite) gets status DF_CELL_NONFINITE, zero
// steps and zero rr, and false is returned.
template <int K>
__device__ bool lane_load(const StepArgs &a, int64_t i, LaneTask<K> &c) {
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
        if (a.status) a.status[i] = DF_CELL_NONFINITE;
        if (a.nsteps) {
            a.nsteps[i] = 0;
            a.nsteps[a.n + i] = 0;
        }
        if (a.rr)
            for (int k = 0; k < K; ++k) a.rr[k * a.ld + i] = 0.0;
        return false;
    }
    const double h_in = a.h_io ? a.h_io[i] : 0.0;
    c.fresh = !(h_in > 0.0);
    c.h = c.fresh ? 0.0 : fmin(h_in, c.dtc);
    if (!c.fresh && !(c.h >= a.o.h_min)) c.h = a.o.h_min;
    c.t = 0.0;
    c.h_final = 0.0;
    c.acc = c.rej = 0;
    c.prev_rej = false;
    (void)N;
    return true;
}

// write the results of the lane's cell
template <int K>
__device__ void lane_finish(const MechDev &m, const StepArgs &a, const LaneTask<K> &c, int st) {
    const int64_t i = c.i;
    if (a.rr) {
        // rr = rho0 (Y - Y0) / dt with rho0 the density of the input state, which is
        // still in memory: read it back instead of keeping it live through the loop
        const double T0 = a.T[i];
        double Y0[K], sYW = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            Y0[k] = a.Y[k * a.ld + i];
            sYW += Y0[k] * m.sp[k * kSpTab + 1];
        }
        const double rdt = c.p / (sYW * kR * T0) / c.dtc;
#pragma unroll
        for (int k = 0; k < K; ++k) a.rr[k * a.ld + i] = rdt * (c.y[1 + k] - Y0[k]);
    }
    a.T[i] = c.y[0];
#pragma unroll
    for (int k = 0; k < K; ++k) a.Y[k * a.ld + i] = c.y[1 + k];
    if (a.h_io) a.h_io[i] = (st == DF_CELL_OK) ? c.h_final : c.h;
    if (a.status) a.status[i] = (st == DF_CELL_OK) ? a.status_ok : st;
    if (a.nsteps) {
        a.nsteps[i] = c.acc;
        a.nsteps[a.n + i] = c.rej;
    }
}

// One RODAS4 attempt of the lane's cell (the first attempt of a cell without a step
// hint also picks the initial step from f(y0)).  Returns true when the cell is done and
// its results have been written.
template <int K, bool CV = false>
__device__ bool lane_attempt(const MechDev &m, const StepArgs &a, double *sh, LaneTask<K> &c) {
    using C = Cell<K, CV>;
    constexpr int N = K + 1;
    const Opts &o = a.o;
    if (c.acc + c.rej >= o.max_steps) {
        lane_finish<K>(m, a, c, DF_CELL_MAX_STEPS);
        return true;
    }
    double W[N][N], f0[N];
    int piv[N];
    C::jacobian(m, c.p, c.y, sh, W, f0);
    if (c.fresh) {
        // initial sub-step from the weighted norms of y0 and f(y0)
        double ny = 0.0, nf = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double sc = (k == 0 ? o.atol_T : o.atol_Y) + o.rtol * fabs(c.y[k]);
            ny += (c.y[k] / sc) * (c.y[k] / sc);
            nf += (f0[k] / sc) * (f0[k] / sc);
        }
        ny = sqrt(ny / N);
        nf = sqrt(nf / N);
        c.h = (nf > 0.0) ? fmin(0.01 * ny / nf, c.dtc) : c.dtc;
        if (!(c.h >= o.h_min)) c.h = o.h_min;
        c.fresh = false;
    }
    const bool last = (c.t + c.h >= c.dtc);
    const double ht = last ? c.dtc - c.t : c.h;
    const double ig = 1.0 / (Rodas4::g * ht);
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int q = 0; q < N; ++q) W[r][q] = (r == q ? ig : 0.0) - W[r][q];
    C::lu(W, piv);

    // stages; u0..u3 are kept in LDS, u4 and u5 in registers
    double u4[N], u5[N], ys[N];
    const double ih = 1.0 / ht;
#pragma unroll
    for (int sidx = 0; sidx < 6; ++sidx) {
        double v[N];
        if (sidx == 0) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = f0[k];
        } else {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double w = c.y[k];
#pragma unroll
                for (int jj = 0; jj < sidx; ++jj) {
                    const double uj = (jj < C::kULds) ? C::at(sh, C::kU + jj * N + k) : u4[k];
                    w = fma(Rodas4::a[sidx][jj], uj, w);
                }
                ys[k] = w;
            }
            C::rhs(m, c.p, ys, sh, v);
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double w = 0.0;
#pragma unroll
                for (int jj = 0; jj < sidx; ++jj) {
                    const double uj = (jj < C::kULds) ? C::at(sh, C::kU + jj * N + k) : u4[k];
                    w = fma(Rodas4::c[sidx][jj], uj, w);
                }
                v[k] = fma(w, ih, v[k]);
            }
        }
        C::solve(W, piv, v);
        if (sidx < C::kULds) {
#pragma unroll
            for (int k = 0; k < N; ++k) C::at(sh, C::kU + sidx * N + k) = v[k];
        } else if (sidx == 4) {
#pragma unroll
            for (int k = 0; k < N; ++k) u4[k] = v[k];
        } else {
#pragma unroll
            for (int k = 0; k < N; ++k) u5[k] = v[k];
        }
    }
    // y_new = (stage-6 state) + u5 ; error = u5
    double err = 0.0;
    double yn[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        yn[k] = ys[k] + u5[k];
        const double sc = (k == 0 ? o.atol_T : o.atol_Y) + o.rtol * fmax(fabs(c.y[k]), fabs(yn[k]));
        const double r = u5[k] / sc;
        err += r * r;
    }
    err = sqrt(err / N);

    const double fmx = c.prev_rej ? 1.0 : 6.0;
    double fac;
    if (!isfinite(err))
        fac = 0.2;
    else if (err == 0.0)
        fac = fmx;
    else
        fac = fmin(fmx, fmax(0.2, 0.9 * pow(err, -0.25)));

    if (isfinite(err) && err <= 1.0) {
        ++c.acc;
#pragma unroll
        for (int k = 0; k < N; ++k) c.y[k] = yn[k];
        c.h_final = c.h;
        c.prev_rej = false;
        if (last) {
            lane_finish<K>(m, a, c, DF_CELL_OK);
            return true;
        }
        c.t += ht;
        c.h = ht * fac;
    } else {
        ++c.rej;
        c.prev_rej = true;
        c.h = ht * fac;
        if (c.h < o.h_min) {
            lane_finish<K>(m, a, c, DF_CELL_H_UNDERFLOW);
            return true;
        }
    }
    return false;
}

}  // namespace
}  // namespace df
