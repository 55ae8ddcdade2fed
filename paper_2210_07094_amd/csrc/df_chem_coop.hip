// Detailed-chemistry step on gfx950 with 16 lanes per cell (four cells per wave64).
//
// Same integration as the one-cell-per-lane kernel (constant-pressure reactor,
// RODAS4, identical step-size controller), with the work of one attempt spread
// over the lanes of the cell so that the latency of a sub-step -- which sets
// the time of a stiff cell's hundreds of sequential sub-steps -- shrinks:
//   * thermo: lane r (1..K) evaluates species r-1 and publishes its
//     concentration, exp(-G/RT), exp(+G/RT) and H/RT in LDS;
//   * rates: lane r evaluates reactions r, r+16, ...; the species lanes sum
//     their own production rates over per-species reaction lists;
//   * Jacobian: the reaction lanes write a dense dq/dc record per reaction to
//     LDS, species lane r assembles row r, the T row is a column reduction;
//   * linear algebra: row i of the iteration matrix W = I/(gamma h) - J lives in
//     lane i; a row-distributed Gauss-Jordan elimination with partial pivoting
//     gives W^-1, so each of the six stage solves is one N-term dot product per
//     lane instead of a sequential substitution.
// State vectors are replicated in the lanes of a cell; every scalar that steers
// control flow (error norm, step size, accept/reject) is computed from the same
// LDS data in the same order by all 16 lanes, so a cell's lanes never diverge.
// Cells of a wave communicate only through their own LDS region.
#include <cmath>

#include "df_internal.h"
#include "df_kinetics.h"

namespace df {
namespace {

constexpr int G = 16;               // lanes per cell
constexpr int kCellsPerBlock = 4;   // one wave64 per block

// Order LDS accesses of the lanes of a wave: the wave executes in lockstep and LDS
// requests of one wave are served in order, so only the compiler must not move
// memory operations across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row strides of the LDS copies of the tables and of the per-reaction records: an
// odd number of doubles (or ints), so that the 16 lanes of a cell reading 16
// different rows at the same column hit 16 different banks.
constexpr int kSpS = kSpTab + 1;   // 21 doubles per species row
constexpr int kRkS = kRxDbl + 1;   // 13 doubles per reaction row
constexpr int kRxS = kRxInt + 1;   // 9 ints per reaction row
__host__ __device__ constexpr int odd(int x) { return x | 1; }

// per-cell LDS layout, in doubles
struct Lay {
    int c, e, ie, h, vec, vec2, red, piv, prow, q, rec, rows, stride;
};

__host__ __device__ inline Lay lay(int K, int M) {
    const int N = K + 1;
    Lay L;
    int o = 0;
    L.c = o, o += N;
    L.e = o, o += N;
    L.ie = o, o += N;
    L.h = o, o += N;
    L.vec = o, o += N;
    L.vec2 = o, o += N;
    L.red = o, o += 4 * N;
    L.piv = o, o += N;
    L.prow = o, o += 2 * N;
    L.q = o, o += M + 1;            // slot M stays zero: it pads the species lists
    L.rec = o, o += (M + 1) * odd(K + 3);
    L.rows = o, o += N * N;
    // cells of a wave start 10 doubles (20 banks) apart modulo the 64 banks
    L.stride = o + ((10 - o % 32) + 32) % 32;
    return L;
}

// Mechanism tables staged in LDS once per block (the per-lane table reads of the
// cooperative kernel are data-dependent gathers, which would otherwise be global
// loads on the critical path of every sub-step).  Offsets in bytes.
struct TabLay {
    int sp, rk, eff, rx, spl, bytes;
};

__host__ __device__ inline TabLay tab_lay(int K, int M, int lmax) {
    TabLay t;
    const int Mm = M > 0 ? M : 1;
    int o = 0;
    t.sp = o, o += K * kSpS * 8;
    t.rk = o, o += Mm * kRkS * 8;
    t.eff = o, o += Mm * odd(K) * 8;
    t.rx = o, o += Mm * kRxS * 4;
    t.spl = o, o += K * odd(2 * lmax) * 4;
    t.bytes = (o + 15) & ~15;
    return t;
}

template <int K>
struct Coop {
    static constexpr int N = K + 1;

    // Mixture terms every lane needs; species thermo of the lane's own species
    struct Own {
        double T, iT, lT, rho, Wbar, cref, icref;
        double hRT, cpR, dcpR;  // of the lane's species (lanes 1..K)
    };

    __device__ __forceinline__ static void prologue(const MechDev &m, const Lay &L, double *sh, int r, double p,
                                                    const double (&y)[N], Own &o) {
        const double T = y[0];
        o.T = T;
        o.iT = 1.0 / T;
        o.lT = log(T);
        double sYW = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) sYW = fma(y[1 + k], m.sp[k * kSpS + 1], sYW);
        o.Wbar = 1.0 / sYW;
        o.rho = p * o.Wbar * o.iT * (1.0 / kR);
        o.cref = 1e-6 * kPref * o.iT * (1.0 / kR);
        o.icref = 1.0 / o.cref;
        o.hRT = o.cpR = o.dcpR = 0.0;
        if (r >= 1 && r <= K) {
            const double *s = m.sp + (r - 1) * kSpS;
            o.cpR = s[2] + T * (s[3] + T * (s[4] + T * (s[5] + T * s[6])));
            o.dcpR = s[3] + T * (s[16] + T * (s[17] + T * s[18]));
            o.hRT = s[2] + T * (s[9] + T * (s[10] + T * (s[11] + T * s[12]))) + s[7] * o.iT;
            const double sr = s[2] * o.lT + T * (s[3] + T * (s[13] + T * (s[14] + T * s[15]))) + s[8];
            const double e = exp(sr - o.hRT);
            sh[L.e + r] = e;
            sh[L.ie + r] = 1.0 / e;
            sh[L.h + r] = o.hRT;
            sh[L.c + r] = 1e-6 * o.rho * y[r] * s[1];
        } else if (r == 0) {
            sh[L.c] = 1.0;
            sh[L.e] = 1.0;
            sh[L.ie] = 1.0;
            sh[L.h] = 0.0;
        }
    }

    // component r of f(y) in lane r (r < N)
    __device__ __forceinline__ static double rhs(const MechDev &m, const Lay &L, double *sh, int r, double p,
                                                 const double (&y)[N]) {
        Own o;
        prologue(m, L, sh, r, p, y, o);
        wave_sync();
        for (int j = r; j < m.M; j += G) {
            const int *ri = m.rx + j * kRxS;
            const double *rd = m.rk + j * kRkS;
            const int type = ri[0];
            const int r0 = ri[1], r1 = ri[2], r2 = ri[3], p0 = ri[4], p1 = ri[5], p2 = ri[6], dnu = ri[7];
            double Mc = 0.0;
            if (type != 0) {
                const double *ef = m.eff + j * odd(K);
#pragma unroll
                for (int k = 0; k < K; ++k) Mc = fma(ef[k], sh[L.c + 1 + k], Mc);
            }
            double dl, dm;
            const double kf = rate_constant<false>(rd, type, o.T, o.iT, o.lT, Mc, dl, dm);
            const double iKc = sh[L.e + r0] * sh[L.e + r1] * sh[L.e + r2] * sh[L.ie + p0] * sh[L.ie + p1] *
                               sh[L.ie + p2] * cref_pow(o.cref, o.icref, dnu);
            const double fwd = kf * (sh[L.c + r0] * sh[L.c + r1] * sh[L.c + r2]);
            const double rev = kf * iKc * (sh[L.c + p0] * sh[L.c + p1] * sh[L.c + p2]);
            double q = fwd - rev;
            if (type == 1) q *= Mc;
            sh[L.q + j] = q;
        }
        wave_sync();
        double f = 0.0;
        if (r >= 1 && r <= K) {
            const int k = r - 1;
            const int *lst = m.spl + k * odd(2 * m.lmax);
            // fixed trip count (lists are padded with the zero slot M) so the loads of
            // several entries are in flight at once
            double w = 0.0;
#pragma unroll 4
            for (int e = 0; e < m.lmax; ++e) w = fma(double(lst[2 * e + 1]), sh[L.q + lst[2 * e]], w);
            const double *s = m.sp + k * kSpS;
            f = 1e6 * s[0] * w / o.rho;
            sh[L.red + r] = o.hRT * w;
            sh[L.red + N + r] = y[r] * o.cpR * s[1];
        }
        wave_sync();
        if (r == 0) {
            double hs = 0.0, cpm = 0.0;
#pragma unroll
            for (int k = 1; k <= K; ++k) {
                hs += sh[L.red + k];
                cpm += sh[L.red + N + k];
            }
            f = -hs * 1e6 * o.T / (o.rho * cpm);
        }
        return f;
    }

    // row r of the analytic Jacobian (lanes r < N) and f_r; see the one-lane kernel for the
    // derivation: derivatives in concentration space, mapped to (T, Y), T row from
    // f_T = -sum_k h_k f_k / cp
    __device__ __forceinline__ static double jacobian(const MechDev &m, const Lay &L, double *sh, int r, double p,
                                                      const double (&y)[N], double (&Jr)[N]) {
        Own o;
        prologue(m, L, sh, r, p, y, o);
        wave_sync();
        for (int j = r; j < m.M; j += G) {
            const int *ri = m.rx + j * kRxS;
            const double *rd = m.rk + j * kRkS;
            const int type = ri[0];
            const int r0 = ri[1], r1 = ri[2], r2 = ri[3], p0 = ri[4], p1 = ri[5], p2 = ri[6], dnu = ri[7];
            const double nr = rd[10], np = rd[11];
            const double *ef = m.eff + j * odd(K);
            double Mc = 0.0;
            if (type != 0) {
#pragma unroll
                for (int k = 0; k < K; ++k) Mc = fma(ef[k], sh[L.c + 1 + k], Mc);
            }
            double dlnkf, dkfdM;
            const double kf = rate_constant<true>(rd, type, o.T, o.iT, o.lT, Mc, dlnkf, dkfdM);
            const double iKc = sh[L.e + r0] * sh[L.e + r1] * sh[L.e + r2] * sh[L.ie + p0] * sh[L.ie + p1] *
                               sh[L.ie + p2] * cref_pow(o.cref, o.icref, dnu);
            const double kr = kf * iKc;
            const double c0 = sh[L.c + r0], c1 = sh[L.c + r1], c2 = sh[L.c + r2];
            const double d0 = sh[L.c + p0], d1 = sh[L.c + p1], d2 = sh[L.c + p2];
            const double Pf = c0 * c1 * c2, Pb = d0 * d1 * d2;
            const double fwd = kf * Pf, rev = kr * Pb, X = fwd - rev;
            const double dlnKc =
                (sh[L.h + p0] + sh[L.h + p1] + sh[L.h + p2] - sh[L.h + r0] - sh[L.h + r1] - sh[L.h + r2] - dnu) * o.iT;
            const double dXdT = fwd * dlnkf - rev * (dlnkf - dlnKc);
            const double Mq = (type == 1) ? Mc : 1.0;
            double S = Mq * (nr * fwd - np * rev);
            double Gd = 0.0;
            if (type == 1) {
                Gd = X;
                S += Mc * X;
            } else if (type == 2) {
                Gd = dkfdM * (Pf - Pb * iKc);
                S += Gd * Mc;
            }
            double *rc = sh + L.rec + j * odd(K + 3);
#pragma unroll
            for (int l = 0; l < K; ++l) rc[l] = Gd * ef[l];
            if (r0) rc[r0 - 1] += Mq * kf * c1 * c2;
            if (r1) rc[r1 - 1] += Mq * kf * c0 * c2;
            if (r2) rc[r2 - 1] += Mq * kf * c0 * c1;
            if (p0) rc[p0 - 1] -= Mq * kr * d1 * d2;
            if (p1) rc[p1 - 1] -= Mq * kr * d0 * d2;
            if (p2) rc[p2 - 1] -= Mq * kr * d0 * d1;
            rc[K] = Mq * X;
            rc[K + 1] = Mq * dXdT;
            rc[K + 2] = S;
        }
        wave_sync();
        double f = 0.0, cpm_own = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) Jr[l] = 0.0;
        if (r >= 1 && r <= K) {
            const int k = r - 1;
            const int *lst = m.spl + k * odd(2 * m.lmax);
            double A[K];
#pragma unroll
            for (int l = 0; l < K; ++l) A[l] = 0.0;
            double sq = 0.0, dt = 0.0, wd = 0.0;
#pragma unroll 2
            for (int e = 0; e < m.lmax; ++e) {
                const int j = lst[2 * e];
                const double nu = double(lst[2 * e + 1]);
                const double *rc = sh + L.rec + j * odd(K + 3);
#pragma unroll
                for (int l = 0; l < K; ++l) A[l] = fma(nu, rc[l], A[l]);
                wd = fma(nu, rc[K], wd);
                dt = fma(nu, rc[K + 1], dt);
                sq = fma(nu, rc[K + 2], sq);
            }
            const double *s = m.sp + k * kSpS;
            const double Wk = s[0];
            const double coef = 1e6 * Wk / o.rho;
            const double gk = coef * o.Wbar * (wd - sq);
            Jr[0] = coef * (dt + (wd - sq) * o.iT);
#pragma unroll
            for (int l = 0; l < K; ++l) Jr[1 + l] = (Wk * A[l] + gk) * m.sp[l * kSpS + 1];
            f = coef * wd;
            const double hm = o.hRT * kR * o.T * s[1];  // J/kg
            cpm_own = o.cpR * kR * s[1];                 // J/kg/K
#pragma unroll
            for (int l = 0; l < N; ++l) sh[L.rows + k * N + l] = hm * Jr[l];
            sh[L.red + r] = hm * f;
            sh[L.red + N + r] = cpm_own * f;
            sh[L.red + 2 * N + r] = y[r] * o.dcpR * kR * s[1];
            sh[L.red + 3 * N + r] = y[r] * cpm_own;
        }
        wave_sync();
        double hf = 0.0, cf = 0.0, dcpdT = 0.0, cp = 0.0;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            hf += sh[L.red + k];
            cf += sh[L.red + N + k];
            dcpdT += sh[L.red + 2 * N + k];
            cp += sh[L.red + 3 * N + k];
        }
        const double fT = -hf / cp;
        if (r < N) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) acc += sh[L.rows + k * N + r];
            if (r == 0) acc += cf;
            const double dcp = (r == 0) ? dcpdT : cpm_own;
            sh[L.vec + r] = -(acc + fT * dcp) / cp;
        }
        wave_sync();
        if (r == 0) {
#pragma unroll
            for (int l = 0; l < N; ++l) Jr[l] = sh[L.vec + l];
            f = fT;
        }
        return f;
    }

    // Gauss-Jordan inverse of W = I/(g h) - J, rows distributed over the lanes (lane i holds row i
    // of W on entry and row i of W^-1 on return).  Partial pivoting: largest magnitude among the
    // rows not yet used as pivots, ties to the lowest row.
    __device__ __forceinline__ static void invert(const Lay &L, double *sh, int r, const double (&Jr)[N], double ig,
                                                  double (&winv)[N]) {
        double a[N], b[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            a[c] = (r == c ? ig : 0.0) - Jr[c];
            b[c] = (r == c) ? 1.0 : 0.0;
        }
        bool used = (r >= N);
        int myrow = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (r < N) sh[L.piv + r] = used ? -1.0 : fabs(a[k]);
            wave_sync();
            int pk = 0;
            double best = sh[L.piv];
#pragma unroll
            for (int t = 1; t < N; ++t) {
                const double v = sh[L.piv + t];
                const bool gt = v > best;
                best = gt ? v : best;
                pk = gt ? t : pk;
            }
            if (r == pk) {
                const double inv = 1.0 / a[k];
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    a[c] *= inv;
                    b[c] *= inv;
                    sh[L.prow + c] = a[c];
                    sh[L.prow + N + c] = b[c];
                }
                used = true;
                myrow = k;
            }
            wave_sync();
            if (r < N && r != pk) {
                const double fct = a[k];
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    a[c] = fma(-fct, sh[L.prow + c], a[c]);
                    b[c] = fma(-fct, sh[L.prow + N + c], b[c]);
                }
            }
        }
        // the lane that pivoted column k holds row k of the inverse: put the rows in order
        if (r < N)
#pragma unroll
            for (int c = 0; c < N; ++c) sh[L.rows + myrow * N + c] = b[c];
        wave_sync();
#pragma unroll
        for (int c = 0; c < N; ++c) winv[c] = (r < N) ? sh[L.rows + r * N + c] : 0.0;
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

template <int K>
__global__ __launch_bounds__(64) void chem_coop_kernel(MechDev mg, int64_t n, int64_t ld, double dt,
                                                       const double *__restrict__ pres, double *__restrict__ Tio,
                                                       double *__restrict__ Yio, double *__restrict__ h_io,
                                                       double *__restrict__ rr, int32_t *__restrict__ status,
                                                       int32_t *__restrict__ nsteps, Opts o,
                                                       const int32_t *__restrict__ cidx,
                                                       const int32_t *__restrict__ dcount, int32_t status_ok) {
    using C = Coop<K>;
    constexpr int N = C::N;
    extern __shared__ double lds[];
    const Lay L = lay(K, mg.M);
    const TabLay tl = tab_lay(K, mg.M, mg.lmax);
    const int lane = threadIdx.x;
    const int r = lane & (G - 1);
    const int64_t limit = dcount ? int64_t(*dcount) : n;
    if (int64_t(blockIdx.x) * kCellsPerBlock >= limit) return;  // whole block idle (e.g. no fallback cells)
    // stage the tables: one copy per block, read by all its cells
    {
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
        const int Mm = mg.M > 0 ? mg.M : 1;
        cp8(tl.sp, mg.sp, K, kSpTab, kSpS);
        cp8(tl.rk, mg.rk, Mm, kRxDbl, kRkS);
        cp8(tl.eff, mg.eff, Mm, K, odd(K));
        cp4(tl.rx, mg.rx, Mm, kRxInt, kRxS);
        cp4(tl.spl, mg.spl, K, 2 * mg.lmax, odd(2 * mg.lmax));
    }
    __syncthreads();
    MechDev m = mg;
    {
        auto *base = reinterpret_cast<unsigned char *>(lds);
        m.sp = reinterpret_cast<const double *>(base + tl.sp);
        m.rk = reinterpret_cast<const double *>(base + tl.rk);
        m.eff = reinterpret_cast<const double *>(base + tl.eff);
        m.rx = reinterpret_cast<const int *>(base + tl.rx);
        m.spl = reinterpret_cast<const int *>(base + tl.spl);
    }
    double *sh = lds + tl.bytes / 8 + (lane / G) * L.stride;
    const int64_t cell = int64_t(blockIdx.x) * kCellsPerBlock + lane / G;
    if (cell >= limit) return;  // the 16 lanes of a cell leave together
    const int64_t i = cidx ? int64_t(cidx[cell]) : cell;
    // the zero slot that pads the species lists
    if (r == 0) sh[L.q + m.M] = 0.0;
    for (int c = r; c < K + 3; c += G) sh[L.rec + m.M * odd(K + 3) + c] = 0.0;

    double y[N];
    const double p = pres[i];
    y[0] = Tio[i];
#pragma unroll
    for (int k = 0; k < K; ++k) y[1 + k] = Yio[k * ld + i];
    bool finite = isfinite(p) && p > 0.0 && isfinite(y[0]) && y[0] > 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) finite = finite && isfinite(y[1 + k]);
    if (!finite) {
        if (r == 0) {
            if (status) status[i] = DF_CELL_NONFINITE;
            if (nsteps) {
                nsteps[i] = 0;
                nsteps[n + i] = 0;
            }
        }
        if (rr && r >= 1 && r <= K) rr[(r - 1) * ld + i] = 0.0;
        return;
    }
    // input density and own mass fraction for rr
    double rho0 = 0.0, y0own = 0.0;
    if (rr) {
        double sYW = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) sYW += y[1 + k] * m.sp[k * kSpS + 1];
        rho0 = p / (sYW * kR * y[0]);
        y0own = (r >= 1 && r <= K) ? y[r] : 0.0;
    }
    const double atol = (r == 0) ? o.atol_T : o.atol_Y;

    // initial sub-step
    double h;
    const double h_in = h_io ? h_io[i] : 0.0;
    if (h_in > 0.0) {
        h = fmin(h_in, dt);
    } else {
        const double f = C::rhs(m, L, sh, r, p, y);
        double yr = 0.0;
#pragma unroll
        for (int c = 0; c < N; ++c)
            if (c == r) yr = y[c];
        const double sc = atol + o.rtol * fabs(yr);
        const double ny = sqrt(C::lane_sum(sh + L.red, r, (yr / sc) * (yr / sc)) / N);
        const double nf = sqrt(C::lane_sum(sh + L.red + N, r, (f / sc) * (f / sc)) / N);
        h = (nf > 0.0) ? fmin(0.01 * ny / nf, dt) : dt;
    }
    if (!(h >= o.h_min)) h = o.h_min;

    double t = 0.0, h_final = 0.0;
    int acc = 0, rej = 0, st = DF_CELL_OK;
    bool prev_rej = false;
    for (;;) {
        if (acc + rej >= o.max_steps) {
            st = DF_CELL_MAX_STEPS;
            break;
        }
        const bool last = (t + h >= dt);
        const double ht = last ? dt - t : h;
        double Jr[N], winv[N];
        const double f0 = C::jacobian(m, L, sh, r, p, y, Jr);
        C::invert(L, sh, r, Jr, 1.0 / (Rodas4::g * ht), winv);

        // own components: y_r, stage vectors u_s[r]
        double yr = 0.0;
#pragma unroll
        for (int c = 0; c < N; ++c)
            if (c == r) yr = y[c];
        double u[6], ysr = yr;
        const double ih = 1.0 / ht;
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            double fs;
            if (s == 0) {
                fs = f0;
            } else {
                ysr = yr;
#pragma unroll
                for (int j = 0; j < s; ++j) ysr = fma(Rodas4::a[s][j], u[j], ysr);
                double ys[N];
                C::gather(sh + L.vec, r, ysr, ys);
                fs = C::rhs(m, L, sh, r, p, ys);
            }
            double cu = 0.0;
#pragma unroll
            for (int j = 0; j < s; ++j) cu = fma(Rodas4::c[s][j], u[j], cu);
            double rv[N];
            C::gather(sh + L.vec2, r, fma(cu, ih, fs), rv);
            double us = 0.0;
#pragma unroll
            for (int c = 0; c < N; ++c) us = fma(winv[c], rv[c], us);
            u[s] = us;
        }
        // y_new = (stage-6 state) + u6 ; error = u6
        const double ynr = ysr + u[5];
        const double sc = atol + o.rtol * fmax(fabs(yr), fabs(ynr));
        const double er = (r < N) ? u[5] / sc : 0.0;
        const double err = sqrt(C::lane_sum(sh + L.red + 2 * N, r, er * er) / N);

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
            C::gather(sh + L.vec, r, ynr, y);
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

    if (r == 0) {
        Tio[i] = y[0];
        if (h_io) h_io[i] = (st == DF_CELL_OK) ? h_final : h;
        if (status) status[i] = (st == DF_CELL_OK) ? status_ok : st;
        if (nsteps) {
            nsteps[i] = acc;
            nsteps[n + i] = rej;
        }
    } else if (r <= K) {
        double yk = 0.0;
#pragma unroll
        for (int c = 1; c < N; ++c)
            if (c == r) yk = y[c];
        if (rr) rr[(r - 1) * ld + i] = rho0 * (yk - y0own) / dt;
        Yio[(r - 1) * ld + i] = yk;
    }
}

}  // namespace

#define DF_COOP_SPECIES_LIST(X) X(2) X(4) X(9)

bool chem_coop_supported(int K) {
    switch (K) {
#define DF_CASE(k) \
    case k:        \
        return true;
        DF_COOP_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return false;
    }
}

template <int K>
static df_status launch_coop_k(const MechDev &m, int64_t n, int64_t ld, double dt, const double *p, double *T,
                               double *Y, double *h_inout, double *rr, int32_t *status, int32_t *n_steps,
                               const Opts &o, const int32_t *cidx, const int32_t *dcount, int32_t status_ok,
                               hipStream_t stream) {
    const int64_t blocks = (n + kCellsPerBlock - 1) / kCellsPerBlock;
    if (blocks > 0x7fffffff) return fail(DF_E_UNSUPPORTED, "chem_step: too many cells for one launch");
    const size_t lds = size_t(tab_lay(K, m.M, m.lmax).bytes) +
                       size_t(lay(K, m.M).stride) * kCellsPerBlock * sizeof(double);
    if (lds > 64 * 1024) return fail(DF_E_UNSUPPORTED, "chem_step: mechanism too large for the cooperative kernel");
    hipLaunchKernelGGL(chem_coop_kernel<K>, dim3(unsigned(blocks)), dim3(64), lds, stream, m, n, ld, dt, p, T, Y,
                       h_inout, rr, status, n_steps, o, cidx, dcount, status_ok);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("chem_step launch: ") + hipGetErrorString(e));
    return DF_OK;
}

df_status launch_chem_coop(const MechDev &m, int64_t n, int64_t ld, double dt, const double *p, double *T, double *Y,
                           double *h_inout, double *rr, int32_t *status, int32_t *n_steps, const df_chem_opts &opts,
                           const int32_t *cidx, const int32_t *dcount, int32_t status_ok, hipStream_t stream) {
    if (n == 0) return DF_OK;
    const Opts o{opts.rtol, opts.atol_T, opts.atol_Y, opts.h_min, opts.max_steps};
    switch (m.K) {
#define DF_CASE(k)                                                                                               \
    case k:                                                                                                      \
        return launch_coop_k<k>(m, n, ld, dt, p, T, Y, h_inout, rr, status, n_steps, o, cidx, dcount, status_ok, \
                                stream);
        DF_COOP_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            return fail(DF_E_UNSUPPORTED, "chem_step: no cooperative kernel for " + std::to_string(m.K) + " species");
    }
}

}  // namespace df
