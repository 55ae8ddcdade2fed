/*
 * CPU oracle for the per-cell chemistry step -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 C, one cell at a time, written for readability, not speed.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code with the GPU library.  See oracle.h for
 * the paper passages each part follows.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define R_GAS 8.31446261815324  /* J/mol/K */
#define P_REF 101325.0          /* Pa, standard-state pressure of the NASA-7 fits */
#define LN10 2.302585092994045684

/* ------------------------------------------------------------------------- */
/* mechanism file ("dfmech 1", plain text)                                    */
/* ------------------------------------------------------------------------- */

static int next_token(FILE *f, char *buf, int n) {
    for (;;) {
        if (fscanf(f, "%255s", buf) != 1) return 0;
        if (buf[0] == '#') { /* comment: skip rest of line */
            int ch;
            while ((ch = fgetc(f)) != EOF && ch != '\n') {}
            continue;
        }
        (void)n;
        return 1;
    }
}

static int expect(FILE *f, const char *key) {
    char tok[256];
    if (!next_token(f, tok, 256)) return 0;
    if (strcmp(tok, key) != 0) {
        fprintf(stderr, "oracle: mechanism file: expected '%s', found '%s'\n", key, tok);
        return 0;
    }
    return 1;
}

static int read_int(FILE *f, int *v) {
    char tok[256];
    if (!next_token(f, tok, 256)) return 0;
    *v = atoi(tok);
    return 1;
}

static int read_long(FILE *f, long *v) {
    char tok[256];
    if (!next_token(f, tok, 256)) return 0;
    *v = atol(tok);
    return 1;
}

static int read_dbl(FILE *f, double *v) {
    char tok[256];
    if (!next_token(f, tok, 256)) return 0;
    *v = strtod(tok, NULL);
    return 1;
}

void orc_mech_free(orc_mech *m) {
    if (!m) return;
    free(m->element_mass); free(m->W); free(m->comp); free(m->nasa); free(m->type);
    free(m->nu_r); free(m->nu_p); free(m->arr); free(m->eff); free(m->low); free(m->troe);
    free(m);
}

orc_mech *orc_mech_load(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return NULL;
    orc_mech *m = (orc_mech *)calloc(1, sizeof(orc_mech));
    char tok[256];
    int ver = 0, ok = 1, i;
    ok = ok && expect(f, "dfmech") && read_int(f, &ver) && ver == 1;
    ok = ok && expect(f, "name") && next_token(f, tok, 256);
    if (ok) snprintf(m->name, sizeof(m->name), "%s", tok);
    ok = ok && expect(f, "seed") && read_long(f, &m->seed);
    ok = ok && expect(f, "n_elements") && read_int(f, &m->E);
    ok = ok && expect(f, "n_species") && read_int(f, &m->K);
    ok = ok && expect(f, "n_reactions") && read_int(f, &m->M);
    if (!ok || m->K < 1 || m->K > ORC_MAX_SPECIES || m->M < 0 || m->E < 1) { fclose(f); orc_mech_free(m); return NULL; }
    int E = m->E, K = m->K, M = m->M;
    m->element_mass = calloc(E, sizeof(double));
    m->W = calloc(K, sizeof(double));
    m->comp = calloc((size_t)K * E, sizeof(int));
    m->nasa = calloc((size_t)K * 7, sizeof(double));
    m->type = calloc(M + 1, sizeof(int));
    m->nu_r = calloc((size_t)M * K + 1, sizeof(int));
    m->nu_p = calloc((size_t)M * K + 1, sizeof(int));
    m->arr = calloc((size_t)M * 3 + 1, sizeof(double));
    m->eff = calloc((size_t)M * K + 1, sizeof(double));
    m->low = calloc((size_t)M * 3 + 1, sizeof(double));
    m->troe = calloc((size_t)M * 4 + 1, sizeof(double));
    ok = ok && expect(f, "elements");
    for (i = 0; ok && i < E; ++i) ok = next_token(f, tok, 256);
    ok = ok && expect(f, "element_mass");
    for (i = 0; ok && i < E; ++i) ok = read_dbl(f, &m->element_mass[i]);
    ok = ok && expect(f, "species");
    for (i = 0; ok && i < K; ++i) ok = next_token(f, tok, 256);
    ok = ok && expect(f, "molar_mass");
    for (i = 0; ok && i < K; ++i) { ok = read_dbl(f, &m->W[i]); m->W[i] *= 1e-3; /* g/mol -> kg/mol */ }
    ok = ok && expect(f, "composition");
    for (i = 0; ok && i < K * E; ++i) ok = read_int(f, &m->comp[i]);
    ok = ok && expect(f, "nasa7");
    for (i = 0; ok && i < K * 7; ++i) ok = read_dbl(f, &m->nasa[i]);
    ok = ok && expect(f, "reaction_type");
    for (i = 0; ok && i < M; ++i) ok = read_int(f, &m->type[i]);
    ok = ok && expect(f, "nu_reac");
    for (i = 0; ok && i < M * K; ++i) ok = read_int(f, &m->nu_r[i]);
    ok = ok && expect(f, "nu_prod");
    for (i = 0; ok && i < M * K; ++i) ok = read_int(f, &m->nu_p[i]);
    ok = ok && expect(f, "arrhenius");
    for (i = 0; ok && i < M * 3; ++i) ok = read_dbl(f, &m->arr[i]);
    ok = ok && expect(f, "efficiency");
    for (i = 0; ok && i < M * K; ++i) ok = read_dbl(f, &m->eff[i]);
    ok = ok && expect(f, "falloff_low");
    for (i = 0; ok && i < M * 3; ++i) ok = read_dbl(f, &m->low[i]);
    ok = ok && expect(f, "troe");
    for (i = 0; ok && i < M * 4; ++i) ok = read_dbl(f, &m->troe[i]);
    ok = ok && expect(f, "end");
    fclose(f);
    for (i = 0; ok && i < M; ++i) ok = (m->type[i] >= 0 && m->type[i] <= 2);
    if (!ok) { orc_mech_free(m); return NULL; }
    return m;
}

int orc_mech_dims(const orc_mech *m, int *K, int *M, int *E) {
    *K = m->K; *M = m->M; *E = m->E;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* thermo: NASA-7 polynomials, one range                                      */
/* ------------------------------------------------------------------------- */

void orc_species_thermo(const orc_mech *m, double T, double *cp_R, double *h_RT, double *s_R, double *g_RT) {
    for (int k = 0; k < m->K; ++k) {
        const double *a = &m->nasa[7 * k];
        double cp = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        double h = a[0] + a[1] * T / 2 + a[2] * T * T / 3 + a[3] * T * T * T / 4 + a[4] * T * T * T * T / 5 + a[5] / T;
        double s = a[0] * log(T) + a[1] * T + a[2] * T * T / 2 + a[3] * T * T * T / 3 + a[4] * T * T * T * T / 4 + a[6];
        if (cp_R) cp_R[k] = cp;
        if (h_RT) h_RT[k] = h;
        if (s_R) s_R[k] = s;
        if (g_RT) g_RT[k] = h - s;
    }
}

/* d(cp/R)/dT of species k */
static double dcpR_dT(const orc_mech *m, int k, double T) {
    const double *a = &m->nasa[7 * k];
    return a[1] + 2 * a[2] * T + 3 * a[3] * T * T + 4 * a[4] * T * T * T;
}

void orc_mixture(const orc_mech *m, double T, double p, const double *Y, double *Wbar, double *rho,
                 double *cp_mass, double *h_mass) {
    double cp_R[ORC_MAX_SPECIES], h_RT[ORC_MAX_SPECIES];
    orc_species_thermo(m, T, cp_R, h_RT, NULL, NULL);
    double sum = 0, cp = 0, h = 0;
    for (int k = 0; k < m->K; ++k) {
        sum += Y[k] / m->W[k];
        cp += Y[k] * cp_R[k] * R_GAS / m->W[k];
        h += Y[k] * h_RT[k] * R_GAS * T / m->W[k];
    }
    double wb = 1.0 / sum;
    if (Wbar) *Wbar = wb;
    if (rho) *rho = p * wb / (R_GAS * T);
    if (cp_mass) *cp_mass = cp;
    if (h_mass) *h_mass = h;
}

/* ------------------------------------------------------------------------- */
/* kinetics                                                                   */
/* ------------------------------------------------------------------------- */

static double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/* prod_k c_k^nu_k */
static double mass_action(const double *c, const int *nu, int K) {
    double r = 1.0;
    for (int k = 0; k < K; ++k) r *= ipow(c[k], nu[k]);
    return r;
}

/* d/dc_m of prod_k c_k^nu_k */
static double d_mass_action(const double *c, const int *nu, int K, int m) {
    if (nu[m] == 0) return 0.0;
    double r = nu[m] * ipow(c[m], nu[m] - 1);
    for (int k = 0; k < K; ++k)
        if (k != m) r *= ipow(c[k], nu[k]);
    return r;
}

/*
 * Forward rate constant of reaction j at T with third-body concentration Mc
 * (mol/cm3).  Arrhenius k = A T^b exp(-Ta/T); for Troe reactions the
 * Lindemann form k_inf Pr/(1+Pr) times the Troe broadening factor F with
 * Pr = k_0 [M] / k_inf.  Also returns d ln kf / dT at fixed [M] and
 * d kf / d[M] at fixed T.
 */
static void forward_rate(const orc_mech *m, int j, double T, double Mc, double *kf, double *dlnkf_dT,
                         double *dkf_dM) {
    const double *a = &m->arr[3 * j];
    double kinf = a[0] * pow(T, a[1]) * exp(-a[2] / T);
    double dlnkinf = a[1] / T + a[2] / (T * T);
    if (m->type[j] != 2) {
        *kf = kinf;
        *dlnkf_dT = dlnkinf;
        *dkf_dM = 0.0;
        return;
    }
    const double *lo = &m->low[3 * j];
    const double *tr = &m->troe[4 * j];
    double k0 = lo[0] * pow(T, lo[1]) * exp(-lo[2] / T);
    double dlnk0 = lo[1] / T + lo[2] / (T * T);
    double Pr = k0 * Mc / kinf;
    double alpha = tr[0], T3 = tr[1], T1 = tr[2], T2 = tr[3];
    double e3 = exp(-T / T3), e1 = exp(-T / T1), e2 = exp(-T2 / T);
    double Fcent = (1 - alpha) * e3 + alpha * e1 + e2;
    double dFcent = -(1 - alpha) / T3 * e3 - alpha / T1 * e1 + T2 / (T * T) * e2;
    double lFc = log10(Fcent);
    double dlFc_dT = dFcent / (Fcent * LN10);
    double cc = -0.4 - 0.67 * lFc;
    double nn = 0.75 - 1.27 * lFc;
    double x = log10(Pr) + cc;
    double den = nn - 0.14 * x;
    double f1 = x / den;
    double lF = lFc / (1 + f1 * f1);
    double F = pow(10.0, lF);
    double k = kinf * Pr / (1 + Pr) * F;
    double g = 2 * f1 / ((1 + f1 * f1) * (1 + f1 * f1));
    double dlF_dlPr = -lFc * g * nn / (den * den);
    double dlF_dlFc = 1 / (1 + f1 * f1) - lFc * g * (-0.67 * nn + 1.27 * x) / (den * den);
    *kf = k;
    *dlnkf_dT = dlnkinf + (1 / (1 + Pr) + dlF_dlPr) * (dlnk0 - dlnkinf) + LN10 * dlF_dlFc * dlFc_dT;
    *dkf_dM = k0 * F / ((1 + Pr) * (1 + Pr)) + k0 * F * dlF_dlPr / (1 + Pr);
}

/* concentrations in mol/cm3 */
static void concentrations(const orc_mech *m, double T, double p, const double *Y, double *c, double *rho_out,
                           double *Wbar_out) {
    double Wbar, rho;
    orc_mixture(m, T, p, Y, &Wbar, &rho, NULL, NULL);
    for (int k = 0; k < m->K; ++k) c[k] = 1e-6 * rho * Y[k] / m->W[k];
    if (rho_out) *rho_out = rho;
    if (Wbar_out) *Wbar_out = Wbar;
}

/* equilibrium constant in concentration units (mol/cm3)^(sum nu) and d ln Kc / dT */
static void equilibrium_constant(const orc_mech *m, int j, double T, const double *h_RT, const double *g_RT,
                                 double *Kc, double *dlnKc_dT) {
    const int *nr = &m->nu_r[m->K * j];
    const int *np = &m->nu_p[m->K * j];
    double dG = 0, dH = 0;
    int dnu = 0;
    for (int k = 0; k < m->K; ++k) {
        int nu = np[k] - nr[k];
        dG += nu * g_RT[k];
        dH += nu * h_RT[k];
        dnu += nu;
    }
    double cref = 1e-6 * P_REF / (R_GAS * T); /* mol/cm3 */
    *Kc = exp(-dG) * ipow(dnu >= 0 ? cref : 1.0 / cref, dnu >= 0 ? dnu : -dnu);
    *dlnKc_dT = dH / T - dnu / T;
}

static double third_body(const orc_mech *m, int j, const double *c) {
    double Mc = 0;
    for (int k = 0; k < m->K; ++k) Mc += m->eff[m->K * j + k] * c[k];
    return Mc;
}

void orc_rates(const orc_mech *m, double T, double p, const double *Y, double *kf_out, double *kr_out, double *q_out,
               double *wdot) {
    int K = m->K, M = m->M;
    double c[ORC_MAX_SPECIES], h_RT[ORC_MAX_SPECIES], g_RT[ORC_MAX_SPECIES];
    concentrations(m, T, p, Y, c, NULL, NULL);
    orc_species_thermo(m, T, NULL, h_RT, NULL, g_RT);
    if (wdot) for (int k = 0; k < K; ++k) wdot[k] = 0;
    for (int j = 0; j < M; ++j) {
        double Mc = (m->type[j] != 0) ? third_body(m, j, c) : 0.0;
        double kf, dlnkf, dkfdM, Kc, dlnKc;
        forward_rate(m, j, T, Mc, &kf, &dlnkf, &dkfdM);
        equilibrium_constant(m, j, T, h_RT, g_RT, &Kc, &dlnKc);
        double kr = kf / Kc;
        double q = kf * mass_action(c, &m->nu_r[K * j], K) - kr * mass_action(c, &m->nu_p[K * j], K);
        if (m->type[j] == 1) q *= Mc;
        if (kf_out) kf_out[j] = kf;
        if (kr_out) kr_out[j] = kr;
        if (q_out) q_out[j] = q;
        if (wdot)
            for (int k = 0; k < K; ++k) wdot[k] += 1e6 * (m->nu_p[K * j + k] - m->nu_r[K * j + k]) * q;
    }
}

/*
 * Constant-pressure adiabatic reactor:
 *   dY_k/dt = W_k wdot_k / rho
 *   dT/dt   = -sum_k H_k wdot_k / (rho cp)
 * (the species line is the paper's source-term equation with the density
 * restored; the energy line keeps the mixture enthalpy constant at fixed p).
 */
void orc_rhs(const orc_mech *m, double p, const double *y, double *f) {
    int K = m->K;
    double T = y[0];
    const double *Y = y + 1;
    double wdot[ORC_MAX_SPECIES], h_RT[ORC_MAX_SPECIES];
    double Wbar, rho, cp;
    orc_mixture(m, T, p, Y, &Wbar, &rho, &cp, NULL);
    orc_rates(m, T, p, Y, NULL, NULL, NULL, wdot);
    orc_species_thermo(m, T, NULL, h_RT, NULL, NULL);
    double S = 0;
    for (int k = 0; k < K; ++k) {
        f[1 + k] = m->W[k] * wdot[k] / rho;
        S += h_RT[k] * R_GAS * T * wdot[k];
    }
    f[0] = -S / (rho * cp);
}

/*
 * Analytic Jacobian d f / d y, y = (T, Y).  Built by the chain rule:
 * progress rates q_j(T, c) -> concentrations c(T, Y) -> wdot -> f.
 */
void orc_jacobian(const orc_mech *m, double p, const double *y, double *J) {
    int K = m->K, M = m->M, N = K + 1;
    double T = y[0];
    const double *Y = y + 1;
    double c[ORC_MAX_SPECIES], cp_R[ORC_MAX_SPECIES], h_RT[ORC_MAX_SPECIES], g_RT[ORC_MAX_SPECIES];
    double rho, Wbar, cp;
    concentrations(m, T, p, Y, c, &rho, &Wbar);
    orc_mixture(m, T, p, Y, NULL, NULL, &cp, NULL);
    orc_species_thermo(m, T, cp_R, h_RT, NULL, g_RT);

    /* d c_m / d y */
    double *dc = (double *)calloc((size_t)K * N, sizeof(double)); /* dc[m*N + l] */
    for (int mm = 0; mm < K; ++mm) {
        dc[mm * N + 0] = -c[mm] / T;
        for (int l = 0; l < K; ++l)
            dc[mm * N + 1 + l] = (mm == l ? 1e-6 * rho / m->W[mm] : 0.0) - c[mm] * Wbar / m->W[l];
    }
    /* wdot and d wdot / d y */
    double wdot[ORC_MAX_SPECIES];
    double *dw = (double *)calloc((size_t)K * N, sizeof(double)); /* dw[k*N + l] */
    double dqdc[ORC_MAX_SPECIES];
    for (int k = 0; k < K; ++k) wdot[k] = 0;
    for (int j = 0; j < M; ++j) {
        const int *nr = &m->nu_r[K * j];
        const int *np = &m->nu_p[K * j];
        double Mc = (m->type[j] != 0) ? third_body(m, j, c) : 0.0;
        double kf, dlnkf, dkfdM, Kc, dlnKc;
        forward_rate(m, j, T, Mc, &kf, &dlnkf, &dkfdM);
        equilibrium_constant(m, j, T, h_RT, g_RT, &Kc, &dlnKc);
        double kr = kf / Kc;
        double Pf = mass_action(c, nr, K), Pb = mass_action(c, np, K);
        double fwd = kf * Pf, rev = kr * Pb;
        double X = fwd - rev;
        double dXdT = fwd * dlnkf - rev * (dlnkf - dlnKc); /* at fixed c and [M] */
        double q, dqdT;
        for (int mm = 0; mm < K; ++mm) dqdc[mm] = kf * d_mass_action(c, nr, K, mm) - kr * d_mass_action(c, np, K, mm);
        if (m->type[j] == 0) {
            q = X;
            dqdT = dXdT;
        } else if (m->type[j] == 1) {
            q = Mc * X;
            dqdT = Mc * dXdT;
            for (int mm = 0; mm < K; ++mm) dqdc[mm] = Mc * dqdc[mm] + m->eff[K * j + mm] * X;
        } else {
            q = X;
            dqdT = dXdT;
            /* kf depends on [M]; kr = kf / Kc follows it */
            for (int mm = 0; mm < K; ++mm) dqdc[mm] += dkfdM * m->eff[K * j + mm] * (Pf - Pb / Kc);
        }
        /* chain rule to (T, Y) */
        double dqdy[ORC_MAX_SPECIES + 1];
        dqdy[0] = dqdT;
        for (int l = 0; l < N; ++l) {
            double s = (l == 0) ? dqdT : 0.0;
            for (int mm = 0; mm < K; ++mm) s += dqdc[mm] * dc[mm * N + l];
            dqdy[l] = s;
        }
        for (int k = 0; k < K; ++k) {
            int nu = np[k] - nr[k];
            if (nu == 0) continue;
            wdot[k] += 1e6 * nu * q;
            for (int l = 0; l < N; ++l) dw[k * N + l] += 1e6 * nu * dqdy[l];
        }
    }
    /* density derivatives */
    double drho[ORC_MAX_SPECIES + 1];
    drho[0] = -rho / T;
    for (int l = 0; l < K; ++l) drho[1 + l] = -rho * Wbar / m->W[l];
    /* species rows: f_k = W_k wdot_k / rho */
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < N; ++l)
            J[(1 + k) * N + l] = m->W[k] * (dw[k * N + l] / rho - wdot[k] * drho[l] / (rho * rho));
    /* temperature row: f_T = -S / D, S = sum H_k wdot_k, D = rho cp */
    double S = 0;
    for (int k = 0; k < K; ++k) S += h_RT[k] * R_GAS * T * wdot[k];
    double D = rho * cp;
    double dcp_dT = 0;
    for (int k = 0; k < K; ++k) dcp_dT += Y[k] * R_GAS * dcpR_dT(m, k, T) / m->W[k];
    for (int l = 0; l < N; ++l) {
        double dS = 0;
        for (int k = 0; k < K; ++k) dS += h_RT[k] * R_GAS * T * dw[k * N + l];
        double dD;
        if (l == 0) {
            for (int k = 0; k < K; ++k) dS += cp_R[k] * R_GAS * wdot[k];
            dD = drho[0] * cp + rho * dcp_dT;
        } else {
            dD = drho[l] * cp + rho * cp_R[l - 1] * R_GAS / m->W[l - 1];
        }
        J[l] = -dS / D + S * dD / (D * D);
    }
    free(dc);
    free(dw);
}

/*
 * Constant-volume adiabatic reactor (the df0DFoam constant-volume case): the
 * density is fixed and the pressure follows, p = rho R T / Wbar;
 *   dY_k/dt = W_k wdot_k / rho
 *   dT/dt   = -sum_k U_k wdot_k / (rho cv),  U_k = H_k - R T,  cv = cp - R / Wbar
 * (the species line as at constant pressure; the energy line keeps the mixture
 * internal energy constant at fixed volume).
 */
static double pressure_at(const orc_mech *m, double rho, double T, const double *Y) {
    double s = 0;
    for (int k = 0; k < m->K; ++k) s += Y[k] / m->W[k];
    return rho * R_GAS * T * s;
}

void orc_rhs_v(const orc_mech *m, double rho, const double *y, double *f) {
    int K = m->K;
    double T = y[0];
    const double *Y = y + 1;
    double p = pressure_at(m, rho, T, Y);
    double wdot[ORC_MAX_SPECIES], h_RT[ORC_MAX_SPECIES], cp_R[ORC_MAX_SPECIES];
    orc_rates(m, T, p, Y, NULL, NULL, NULL, wdot);
    orc_species_thermo(m, T, cp_R, h_RT, NULL, NULL);
    double S = 0, cv = 0;
    for (int k = 0; k < K; ++k) {
        f[1 + k] = m->W[k] * wdot[k] / rho;
        S += (h_RT[k] - 1.0) * R_GAS * T * wdot[k];
        cv += Y[k] * (cp_R[k] - 1.0) * R_GAS / m->W[k];
    }
    f[0] = -S / (rho * cv);
}

/* analytic Jacobian of the constant-volume reactor: the chain rule through
 * q_j(T, c) with c_m = 1e-6 rho Y_m / W_m independent of T */
void orc_jacobian_v(const orc_mech *m, double rho, const double *y, double *J) {
    int K = m->K, M = m->M, N = K + 1;
    double T = y[0];
    const double *Y = y + 1;
    double c[ORC_MAX_SPECIES], cp_R[ORC_MAX_SPECIES], h_RT[ORC_MAX_SPECIES], g_RT[ORC_MAX_SPECIES];
    for (int k = 0; k < K; ++k) c[k] = 1e-6 * rho * Y[k] / m->W[k];
    orc_species_thermo(m, T, cp_R, h_RT, NULL, g_RT);
    double wdot[ORC_MAX_SPECIES];
    double *dw = (double *)calloc((size_t)K * N, sizeof(double)); /* dw[k*N + l] */
    double dqdc[ORC_MAX_SPECIES];
    for (int k = 0; k < K; ++k) wdot[k] = 0;
    for (int j = 0; j < M; ++j) {
        const int *nr = &m->nu_r[K * j];
        const int *np = &m->nu_p[K * j];
        double Mc = (m->type[j] != 0) ? third_body(m, j, c) : 0.0;
        double kf, dlnkf, dkfdM, Kc, dlnKc;
        forward_rate(m, j, T, Mc, &kf, &dlnkf, &dkfdM);
        equilibrium_constant(m, j, T, h_RT, g_RT, &Kc, &dlnKc);
        double kr = kf / Kc;
        double Pf = mass_action(c, nr, K), Pb = mass_action(c, np, K);
        double fwd = kf * Pf, rev = kr * Pb;
        double X = fwd - rev;
        double dXdT = fwd * dlnkf - rev * (dlnkf - dlnKc);
        double q, dqdT;
        for (int mm = 0; mm < K; ++mm) dqdc[mm] = kf * d_mass_action(c, nr, K, mm) - kr * d_mass_action(c, np, K, mm);
        if (m->type[j] == 0) {
            q = X;
            dqdT = dXdT;
        } else if (m->type[j] == 1) {
            q = Mc * X;
            dqdT = Mc * dXdT;
            for (int mm = 0; mm < K; ++mm) dqdc[mm] = Mc * dqdc[mm] + m->eff[K * j + mm] * X;
        } else {
            q = X;
            dqdT = dXdT;
            for (int mm = 0; mm < K; ++mm) dqdc[mm] += dkfdM * m->eff[K * j + mm] * (Pf - Pb / Kc);
        }
        for (int k = 0; k < K; ++k) {
            int nu = np[k] - nr[k];
            if (nu == 0) continue;
            wdot[k] += 1e6 * nu * q;
            dw[k * N + 0] += 1e6 * nu * dqdT;
            for (int l = 0; l < K; ++l) dw[k * N + 1 + l] += 1e6 * nu * dqdc[l] * 1e-6 * rho / m->W[l];
        }
    }
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < N; ++l) J[(1 + k) * N + l] = m->W[k] * dw[k * N + l] / rho;
    /* temperature row: f_T = -S / D, S = sum U_k wdot_k, D = rho cv */
    double S = 0, cv = 0, dcv_dT = 0;
    for (int k = 0; k < K; ++k) {
        S += (h_RT[k] - 1.0) * R_GAS * T * wdot[k];
        cv += Y[k] * (cp_R[k] - 1.0) * R_GAS / m->W[k];
        dcv_dT += Y[k] * R_GAS * dcpR_dT(m, k, T) / m->W[k];
    }
    double D = rho * cv;
    for (int l = 0; l < N; ++l) {
        double dS = 0;
        for (int k = 0; k < K; ++k) dS += (h_RT[k] - 1.0) * R_GAS * T * dw[k * N + l];
        double dD;
        if (l == 0) {
            for (int k = 0; k < K; ++k) dS += (cp_R[k] - 1.0) * R_GAS * wdot[k]; /* dU_k/dT = cv_k */
            dD = rho * dcv_dT;
        } else {
            dD = rho * (cp_R[l - 1] - 1.0) * R_GAS / m->W[l - 1];
        }
        J[l] = -dS / D + S * dD / (D * D);
    }
    free(dw);
}

/* ------------------------------------------------------------------------- */
/* dense LU with partial pivoting (ties -> lowest row index)                  */
/* ------------------------------------------------------------------------- */

static int lu_factor(int n, double *A, int *piv) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        piv[k] = p;
        if (!(best > 0.0)) return -1;
        if (p != k)
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}

static void lu_solve(int n, const double *LU, const int *piv, double *b) {
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 1; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
        b[i] /= LU[i * n + i];
    }
}

/* ------------------------------------------------------------------------- */
/* RODAS4 (Hairer & Wanner, Solving ODEs II, Sec. IV.7), transformed form:    */
/*   (I/(gamma h) - J) u_i = f(y + sum_j a_ij u_j) + sum_j (c_ij / h) u_j      */
/*   y_new = y + sum m_i u_i,   error = sum (m_i - mhat_i) u_i                 */
/* Stage 6 sits on the embedded (order 3) solution, so the error is u_6.      */
/* ------------------------------------------------------------------------- */

#define NS 6
static const double ROS_GAMMA = 0.25;
static const double ROS_A[NS][NS] = {
    {0, 0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 0},
};
static const double ROS_C[NS][NS] = {
    {0, 0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136, -6.058818238834054, 0},
};
static const double ROS_M[NS] = {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0,
                                 1.0};
static const double ROS_MHAT[NS] = {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950,
                                    1.0, 0.0};
static const int ROS_ORDER_EMBEDDED = 3;

void orc_rodas4_tableau(double *gamma, double *a, double *c, double *mm, double *mhat) {
    *gamma = ROS_GAMMA;
    for (int i = 0; i < NS; ++i) {
        for (int j = 0; j < NS; ++j) { a[i * NS + j] = ROS_A[i][j]; c[i * NS + j] = ROS_C[i][j]; }
        mm[i] = ROS_M[i];
        mhat[i] = ROS_MHAT[i];
    }
}

typedef void (*rhs_fn)(void *ctx, const double *y, double *f);
typedef void (*jac_fn)(void *ctx, const double *y, double *J);

/*
 * Adaptive RODAS4 integration of y' = f(y) over [0, dt].
 *  - initial step: h_in if > 0 (capped at dt), else 0.01 |y|/|f(y)| in the
 *    weighted RMS norm (dt if f = 0), at least h_min;
 *  - the last step is shortened to land exactly on dt;
 *  - weighted RMS error norm with scale atol_i + rtol max(|y_i|, |ynew_i|);
 *  - accept if err <= 1; new h = h * min(fmax, max(0.2, 0.9 err^(-1/4)))
 *    with fmax = 6, or 1 right after a rejection; a non-finite error is a
 *    rejection with factor 0.2;
 *  - stops with MAX_STEPS after max_steps attempts, H_UNDERFLOW when a
 *    rejection pushes h below h_min.
 * h_next is the controller's step proposal in force when the final step was
 * taken (before it was shortened to land on dt).
 */
/*
 * One RODAS4 attempt of length ht from y, with f0 = f(y): writes the new state
 * yn and the embedded error vector ev, and returns the weighted RMS error
 * norm (scale atol_i + rtol max(|y_i|, |yn_i|)), or +inf when the iteration
 * matrix is singular.  Work arrays: J, Wm (N*N), u (NS*N), ys, fs (N), piv.
 */
static double ros_attempt(int N, const double *y, const double *f0, double ht, const double *atol, double rtol,
                          rhs_fn rhs, jac_fn jac, void *ctx, double *J, double *Wm, double *u, double *ys, double *fs,
                          int *piv, double *yn, double *ev) {
    jac(ctx, y, J);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Wm[i * N + j] = (i == j ? 1.0 / (ROS_GAMMA * ht) : 0.0) - J[i * N + j];
    if (lu_factor(N, Wm, piv) != 0) return INFINITY;
    for (int s = 0; s < NS; ++s) {
        double *us = &u[s * N];
        if (s == 0) {
            for (int i = 0; i < N; ++i) fs[i] = f0[i];
        } else {
            for (int i = 0; i < N; ++i) {
                double v = y[i];
                for (int j = 0; j < s; ++j) v += ROS_A[s][j] * u[j * N + i];
                ys[i] = v;
            }
            rhs(ctx, ys, fs);
        }
        for (int i = 0; i < N; ++i) {
            double v = fs[i];
            for (int j = 0; j < s; ++j) v += (ROS_C[s][j] / ht) * u[j * N + i];
            us[i] = v;
        }
        lu_solve(N, Wm, piv, us);
    }
    for (int i = 0; i < N; ++i) {
        double v = y[i], e = 0.0;
        for (int s = 0; s < NS; ++s) {
            v += ROS_M[s] * u[s * N + i];
            e += (ROS_M[s] - ROS_MHAT[s]) * u[s * N + i];
        }
        yn[i] = v;
        ev[i] = e;
    }
    if (!atol) return 0.0;
    double sum = 0.0;
    for (int i = 0; i < N; ++i) {
        double ay = fabs(y[i]), an = fabs(yn[i]);
        double sc = atol[i] + rtol * (ay > an ? ay : an);
        sum += (ev[i] / sc) * (ev[i] / sc);
    }
    return sqrt(sum / N);
}

/*
 * Adaptive RODAS4 integration of y' = f(y) over [0, dt].
 *  - initial step: h_in if > 0 (capped at dt), else 0.01 |y|/|f(y)| in the
 *    weighted RMS norm (dt if f = 0), at least h_min;
 *  - the last step is shortened to land exactly on dt;
 *  - weighted RMS error norm with scale atol_i + rtol max(|y_i|, |ynew_i|);
 *  - accept if err <= 1; new h = h * min(fmax, max(0.2, 0.9 err^(-1/4)))
 *    with fmax = 6, or 1 right after a rejection; a non-finite error is a
 *    rejection with factor 0.2;
 *  - stops with MAX_STEPS after max_steps attempts, H_UNDERFLOW when a
 *    rejection pushes h below h_min.
 * h_next is the controller's step proposal in force when the final step was
 * taken (before it was shortened to land on dt).  When h_rec is given, the
 * length of accepted step s is stored in h_rec[s] for s < rec_cap.
 */
static int ros_integrate(int N, double *y, double dt, double h_in, const double *atol, double rtol, double h_min,
                         int max_steps, rhs_fn rhs, jac_fn jac, void *ctx, double *h_next, int *n_acc, int *n_rej,
                         double *h_rec, int rec_cap) {
    double *J = (double *)malloc(sizeof(double) * N * N);
    double *Wm = (double *)malloc(sizeof(double) * N * N);
    double *u = (double *)malloc(sizeof(double) * NS * N);
    double *f0 = (double *)malloc(sizeof(double) * N);
    double *ys = (double *)malloc(sizeof(double) * N);
    double *fs = (double *)malloc(sizeof(double) * N);
    double *yn = (double *)malloc(sizeof(double) * N);
    double *ev = (double *)malloc(sizeof(double) * N);
    int *piv = (int *)malloc(sizeof(int) * N);
    int status = ORC_OK, acc = 0, rej = 0, prev_rejected = 0;
    double t = 0.0, h, h_final = 0.0;

    rhs(ctx, y, f0);
    if (h_in > 0.0) {
        h = h_in < dt ? h_in : dt;
    } else {
        double ny = 0, nf = 0;
        for (int i = 0; i < N; ++i) {
            double sc = atol[i] + rtol * fabs(y[i]);
            ny += (y[i] / sc) * (y[i] / sc);
            nf += (f0[i] / sc) * (f0[i] / sc);
        }
        ny = sqrt(ny / N);
        nf = sqrt(nf / N);
        h = (nf > 0.0) ? 0.01 * ny / nf : dt;
        if (h > dt) h = dt;
    }
    if (!(h >= h_min)) h = h_min;

    for (;;) {
        if (acc + rej >= max_steps) { status = ORC_MAX_STEPS; break; }
        int last = (t + h >= dt);
        double ht = last ? dt - t : h;
        double err = ros_attempt(N, y, f0, ht, atol, rtol, rhs, jac, ctx, J, Wm, u, ys, fs, piv, yn, ev);

        double fmax = prev_rejected ? 1.0 : 6.0;
        double fac;
        if (!isfinite(err)) fac = 0.2;
        else if (err == 0.0) fac = fmax;
        else {
            fac = 0.9 * pow(err, -1.0 / (ROS_ORDER_EMBEDDED + 1));
            if (fac > fmax) fac = fmax;
            if (fac < 0.2) fac = 0.2;
        }

        if (isfinite(err) && err <= 1.0) {
            if (h_rec && acc < rec_cap) h_rec[acc] = ht;
            ++acc;
            for (int i = 0; i < N; ++i) y[i] = yn[i];
            h_final = h;
            prev_rejected = 0;
            if (last) { t = dt; break; }
            t += ht;
            h = ht * fac;
            rhs(ctx, y, f0);
        } else {
            ++rej;
            prev_rejected = 1;
            h = ht * fac;
            if (h < h_min) { status = ORC_H_UNDERFLOW; break; }
        }
    }
    if (h_next) *h_next = (status == ORC_OK) ? h_final : h;
    if (n_acc) *n_acc = acc;
    if (n_rej) *n_rej = rej;
    free(J); free(Wm); free(u); free(f0); free(ys); free(fs); free(yn); free(ev); free(piv);
    return status;
}

/* ---- linear test problems: y' = A y ---- */
typedef struct { int n; const double *A; } lin_ctx;

static void lin_rhs(void *ctx, const double *y, double *f) {
    lin_ctx *c = (lin_ctx *)ctx;
    for (int i = 0; i < c->n; ++i) {
        double s = 0;
        for (int j = 0; j < c->n; ++j) s += c->A[i * c->n + j] * y[j];
        f[i] = s;
    }
}

static void lin_jac(void *ctx, const double *y, double *J) {
    (void)y;
    lin_ctx *c = (lin_ctx *)ctx;
    memcpy(J, c->A, sizeof(double) * c->n * c->n);
}

int orc_linear_integrate(int n, const double *A, double *y, double dt, double h_in, const orc_opts *o, double *atol,
                         double *h_next, int32_t *n_acc, int32_t *n_rej) {
    lin_ctx c = {n, A};
    int a = 0, r = 0;
    int st = ros_integrate(n, y, dt, h_in, atol, o->rtol, o->h_min, o->max_steps, lin_rhs, lin_jac, &c, h_next, &a, &r,
                           NULL, 0);
    if (n_acc) *n_acc = a;
    if (n_rej) *n_rej = r;
    return st;
}

void orc_linear_fixed_step(int n, const double *A, double *y, double h, double *err_vec) {
    /* one RODAS4 step without error control, written out on its own */
    lin_ctx c = {n, A};
    double *Wm = (double *)malloc(sizeof(double) * n * n);
    double *u = (double *)malloc(sizeof(double) * NS * n);
    double *ys = (double *)malloc(sizeof(double) * n);
    double *fs = (double *)malloc(sizeof(double) * n);
    int *piv = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Wm[i * n + j] = (i == j ? 1.0 / (ROS_GAMMA * h) : 0.0) - A[i * n + j];
    lu_factor(n, Wm, piv);
    for (int s = 0; s < NS; ++s) {
        for (int i = 0; i < n; ++i) {
            double v = y[i];
            for (int j = 0; j < s; ++j) v += ROS_A[s][j] * u[j * n + i];
            ys[i] = v;
        }
        lin_rhs(&c, ys, fs);
        for (int i = 0; i < n; ++i) {
            double v = fs[i];
            for (int j = 0; j < s; ++j) v += (ROS_C[s][j] / h) * u[j * n + i];
            u[s * n + i] = v;
        }
        lu_solve(n, Wm, piv, &u[s * n]);
    }
    for (int i = 0; i < n; ++i) {
        double e = 0;
        for (int s = 0; s < NS; ++s) {
            y[i] += ROS_M[s] * u[s * n + i];
            e += (ROS_M[s] - ROS_MHAT[s]) * u[s * n + i];
        }
        if (err_vec) err_vec[i] = e;
    }
    free(Wm); free(u); free(ys); free(fs); free(piv);
}

/* ---- chemistry ---- */
/* p is the pressure (constant-pressure reactor) or the density (constant-volume, cv != 0) */
typedef struct { const orc_mech *m; double p; int cv; } chem_ctx;

static void chem_rhs(void *ctx, const double *y, double *f) {
    chem_ctx *c = (chem_ctx *)ctx;
    if (c->cv)
        orc_rhs_v(c->m, c->p, y, f);
    else
        orc_rhs(c->m, c->p, y, f);
}

static void chem_jac(void *ctx, const double *y, double *J) {
    chem_ctx *c = (chem_ctx *)ctx;
    if (c->cv)
        orc_jacobian_v(c->m, c->p, y, J);
    else
        orc_jacobian(c->m, c->p, y, J);
}

static orc_opts default_opts(const orc_opts *o) {
    orc_opts d = {1e-8, 1e-6, 1e-14, 1e-20, 100000};
    return o ? *o : d;
}

/* integrate one cell in place; returns status */
static int chem_cell(const orc_mech *m, double dt, double p, double *y, double *h_io, const orc_opts *o,
                     int *acc, int *rej, int cv) {
    int K = m->K, N = K + 1;
    int finite = isfinite(p) && p > 0 && isfinite(y[0]) && y[0] > 0;
    for (int k = 0; k < K; ++k) finite = finite && isfinite(y[1 + k]);
    *acc = 0;
    *rej = 0;
    if (!finite) return ORC_NONFINITE;
    double atol[ORC_MAX_SPECIES + 1];
    atol[0] = o->atol_T;
    for (int k = 0; k < K; ++k) atol[1 + k] = o->atol_Y;
    chem_ctx c = {m, p, cv};
    double h_in = h_io ? *h_io : 0.0, h_next = 0.0;
    int st = ros_integrate(N, y, dt, h_in, atol, o->rtol, o->h_min, o->max_steps, chem_rhs, chem_jac, &c, &h_next,
                           acc, rej, NULL, 0);
    if (h_io) *h_io = h_next;
    return st;
}

int orc_chem_step(const orc_mech *m, int64_t n, int64_t ld, double dt, const double *p, double *T, double *Y,
                  double *h_inout, double *rr, int32_t *status, int32_t *n_acc, int32_t *n_rej, const orc_opts *opts,
                  int nthreads) {
    return orc_chem_step_dt(m, n, ld, dt, NULL, p, T, Y, h_inout, rr, status, n_acc, n_rej, opts, nthreads);
}

int orc_chem_step_dt(const orc_mech *m, int64_t n, int64_t ld, double dt, const double *dt_cells, const double *p,
                     double *T, double *Y, double *h_inout, double *rr, int32_t *status, int32_t *n_acc,
                     int32_t *n_rej, const orc_opts *opts, int nthreads) {
    if (!m || n < 0 || ld < n || !p || !T || !Y) return -1;
    if (!dt_cells && !(dt > 0)) return -1;
    if (dt_cells)
        for (int64_t i = 0; i < n; ++i)
            if (!(dt_cells[i] > 0)) return -1;
    orc_opts o = default_opts(opts);
    int K = m->K;
    int fails = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : fails)
    for (int64_t i = 0; i < n; ++i) {
        double y[ORC_MAX_SPECIES + 1], Y0[ORC_MAX_SPECIES];
        y[0] = T[i];
        for (int k = 0; k < K; ++k) { y[1 + k] = Y[k * ld + i]; Y0[k] = y[1 + k]; }
        double rho0 = 0.0;
        if (rr) orc_mixture(m, T[i], p[i], Y0, NULL, &rho0, NULL, NULL);
        int acc, rej;
        const double dti = dt_cells ? dt_cells[i] : dt;
        int st = chem_cell(m, dti, p[i], y, h_inout ? &h_inout[i] : NULL, &o, &acc, &rej, 0);
        if (st != ORC_NONFINITE) {
            T[i] = y[0];
            for (int k = 0; k < K; ++k) Y[k * ld + i] = y[1 + k];
        }
        if (rr)
            for (int k = 0; k < K; ++k) rr[k * ld + i] = rho0 * (Y[k * ld + i] - Y0[k]) / dti;
        if (status) status[i] = st;
        if (n_acc) n_acc[i] = acc;
        if (n_rej) n_rej[i] = rej;
        if (st != ORC_OK) fails += 1;
    }
    return fails;
}

/* constant-volume step of n cells: rho [n] fixed, T and Y advanced in place
 * (same controller, tolerances and statuses as orc_chem_step) */
int orc_chem_step_v(const orc_mech *m, int64_t n, int64_t ld, double dt, const double *rho, double *T, double *Y,
                    double *h_inout, int32_t *status, int32_t *n_acc, int32_t *n_rej, const orc_opts *opts,
                    int nthreads) {
    if (!m || n < 0 || ld < n || !rho || !T || !Y || !(dt > 0)) return -1;
    orc_opts o = default_opts(opts);
    int K = m->K;
    int fails = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : fails)
    for (int64_t i = 0; i < n; ++i) {
        double y[ORC_MAX_SPECIES + 1];
        y[0] = T[i];
        for (int k = 0; k < K; ++k) y[1 + k] = Y[k * ld + i];
        int acc, rej;
        int st = chem_cell(m, dt, rho[i], y, h_inout ? &h_inout[i] : NULL, &o, &acc, &rej, 1);
        if (st != ORC_NONFINITE) {
            T[i] = y[0];
            for (int k = 0; k < K; ++k) Y[k * ld + i] = y[1 + k];
        }
        if (status) status[i] = st;
        if (n_acc) n_acc[i] = acc;
        if (n_rej) n_rej[i] = rej;
        if (st != ORC_OK) fails += 1;
    }
    return fails;
}

/*
 * Sensitivities of the step (test support): the integration of one cell from
 * a fresh start (no step hint), recording the length of every accepted
 * sub-step; the replay of such a recorded sequence without error control
 * (the same arithmetic as the accepted attempts, so a replay of a cell's own
 * record reproduces its result exactly); and a scaling of one reaction's
 * pre-exponential factor (for Troe rows the high-pressure limit), for finite
 * differences in ln A.
 */
int orc_chem_cell_record(const orc_mech *m, double dt, double p, double *y, const orc_opts *opts, double *h_rec,
                         int32_t rec_cap, int32_t *n_acc, int32_t *n_rej) {
    orc_opts o = default_opts(opts);
    int K = m->K, N = K + 1;
    double atol[ORC_MAX_SPECIES + 1];
    atol[0] = o.atol_T;
    for (int k = 0; k < K; ++k) atol[1 + k] = o.atol_Y;
    chem_ctx c = {m, p, 0};
    int a = 0, r = 0;
    int st = ros_integrate(N, y, dt, 0.0, atol, o.rtol, o.h_min, o.max_steps, chem_rhs, chem_jac, &c, NULL, &a, &r,
                           h_rec, rec_cap);
    if (n_acc) *n_acc = a;
    if (n_rej) *n_rej = r;
    return st;
}

void orc_chem_replay(const orc_mech *m, double p, double *y, const double *hs, int32_t nh) {
    int N = m->K + 1;
    chem_ctx c = {m, p, 0};
    double J[(ORC_MAX_SPECIES + 1) * (ORC_MAX_SPECIES + 1)], Wm[(ORC_MAX_SPECIES + 1) * (ORC_MAX_SPECIES + 1)];
    double u[NS * (ORC_MAX_SPECIES + 1)], f0[ORC_MAX_SPECIES + 1], ys[ORC_MAX_SPECIES + 1], fs[ORC_MAX_SPECIES + 1];
    double yn[ORC_MAX_SPECIES + 1], ev[ORC_MAX_SPECIES + 1];
    int piv[ORC_MAX_SPECIES + 1];
    for (int s = 0; s < nh; ++s) {
        chem_rhs(&c, y, f0);
        ros_attempt(N, y, f0, hs[s], NULL, 0.0, chem_rhs, chem_jac, &c, J, Wm, u, ys, fs, piv, yn, ev);
        for (int i = 0; i < N; ++i) y[i] = yn[i];
    }
}

void orc_mech_scale_A(orc_mech *m, int32_t j, double factor) {
    if (m && j >= 0 && j < m->M) m->arr[3 * j] *= factor;
}

/* ------------------------------------------------------------------------- */
/* DNN form                                                                   */
/* ------------------------------------------------------------------------- */

struct orc_dnn {
    int L, K, n_in, n_out;
    int dims[8];
    double lambda, dt_train;
    double *mu_in, *sig_in, *mu_out, *sig_out, *lo, *hi;
    double *W[8]; /* [dims[l+1] * dims[l]] row-major, values exactly bf16 */
    double *b[8]; /* [dims[l+1]] */
};

static double bf16_bits_to_double(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

void orc_dnn_free(orc_dnn *d) {
    if (!d) return;
    free(d->mu_in); free(d->sig_in); free(d->mu_out); free(d->sig_out); free(d->lo); free(d->hi);
    for (int l = 0; l < d->L; ++l) { free(d->W[l]); free(d->b[l]); }
    free(d);
}

/*
 * Weights file "DFDNN01": little-endian; int32 L, dims[L+1], K, reserved;
 * f64 lambda, dt_train; f64 mu_in[n_in], sig_in[n_in], mu_out[n_out],
 * sig_out[n_out], box_lo[n_in], box_hi[n_in]; then per layer bf16 W[out][in]
 * and f32 b[out].  Inputs are (T, p, BCT(Y_1..Y_K)); outputs are the
 * normalised increments of BCT(Y) over dt_train.
 */
orc_dnn *orc_dnn_load(const char *path) {
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    char magic[8];
    orc_dnn *d = (orc_dnn *)calloc(1, sizeof(orc_dnn));
    int ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "DFDNN01", 7) == 0;
    int32_t L = 0, K = 0, reserved = 0;
    ok = ok && fread(&L, 4, 1, f) == 1 && L >= 1 && L <= 7;
    if (!ok) { fclose(f); free(d); return NULL; }
    d->L = L;
    int32_t dims[8];
    ok = fread(dims, 4, L + 1, f) == (size_t)(L + 1);
    ok = ok && fread(&K, 4, 1, f) == 1 && fread(&reserved, 4, 1, f) == 1;
    ok = ok && fread(&d->lambda, 8, 1, f) == 1 && fread(&d->dt_train, 8, 1, f) == 1;
    if (!ok) { fclose(f); free(d); return NULL; }
    for (int l = 0; l <= L; ++l) d->dims[l] = dims[l];
    d->K = K;
    d->n_in = dims[0];
    d->n_out = dims[L];
    d->mu_in = malloc(8 * d->n_in); d->sig_in = malloc(8 * d->n_in);
    d->mu_out = malloc(8 * d->n_out); d->sig_out = malloc(8 * d->n_out);
    d->lo = malloc(8 * d->n_in); d->hi = malloc(8 * d->n_in);
    ok = fread(d->mu_in, 8, d->n_in, f) == (size_t)d->n_in && fread(d->sig_in, 8, d->n_in, f) == (size_t)d->n_in &&
         fread(d->mu_out, 8, d->n_out, f) == (size_t)d->n_out && fread(d->sig_out, 8, d->n_out, f) == (size_t)d->n_out &&
         fread(d->lo, 8, d->n_in, f) == (size_t)d->n_in && fread(d->hi, 8, d->n_in, f) == (size_t)d->n_in;
    for (int l = 0; ok && l < L; ++l) {
        size_t nw = (size_t)dims[l + 1] * dims[l];
        uint16_t *tmp = malloc(2 * nw);
        float *bt = malloc(4 * dims[l + 1]);
        ok = fread(tmp, 2, nw, f) == nw && fread(bt, 4, dims[l + 1], f) == (size_t)dims[l + 1];
        d->W[l] = malloc(8 * nw);
        d->b[l] = malloc(8 * dims[l + 1]);
        for (size_t i = 0; ok && i < nw; ++i) d->W[l][i] = bf16_bits_to_double(tmp[i]);
        for (int i = 0; ok && i < dims[l + 1]; ++i) d->b[l][i] = bt[i];
        free(tmp);
        free(bt);
    }
    fclose(f);
    if (!ok || d->n_in != K + 2 || d->n_out != K) { orc_dnn_free(d); return NULL; }
    return d;
}

int orc_dnn_dims(const orc_dnn *d, int *n_layers, int *dims, int *K, double *lambda, double *dt_train) {
    *n_layers = d->L;
    for (int l = 0; l <= d->L; ++l) dims[l] = d->dims[l];
    *K = d->K;
    *lambda = d->lambda;
    *dt_train = d->dt_train;
    return 0;
}

/* Box-Cox: z = (Y^lambda - 1) / lambda, with Y clamped at 0 from below */
double orc_bct(double Y, double lambda) {
    if (Y < 0) Y = 0;
    return (pow(Y, lambda) - 1.0) / lambda;
}

/* inverse Box-Cox: Y = (1 + lambda z)^(1/lambda), base clamped at 0 */
double orc_bct_inv(double z, double lambda) {
    double base = 1.0 + lambda * z;
    if (base < 0) base = 0;
    return pow(base, 1.0 / lambda);
}

float orc_bf16_round(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) { /* inf or nan: keep, quiet nans */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, 4);
    return r;
}

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }

void orc_mlp_forward(const orc_dnn *d, const double *x_norm, double *u, int mode) {
    int maxw = 0;
    for (int l = 0; l <= d->L; ++l) if (d->dims[l] > maxw) maxw = d->dims[l];
    double *a = malloc(8 * maxw), *z = malloc(8 * maxw);
    for (int i = 0; i < d->n_in; ++i) a[i] = (mode == 1) ? (double)orc_bf16_round((float)x_norm[i]) : x_norm[i];
    for (int l = 0; l < d->L; ++l) {
        int ni = d->dims[l], no = d->dims[l + 1];
        for (int o = 0; o < no; ++o) {
            const double *w = &d->W[l][(size_t)o * ni];
            if (mode == 1) {
                float acc = 0.0f;
                for (int i = 0; i < ni; ++i) acc = acc + (float)w[i] * (float)a[i];
                acc = acc + (float)d->b[l][o];
                z[o] = acc;
            } else {
                double acc = 0.0;
                for (int i = 0; i < ni; ++i) acc += w[i] * a[i];
                z[o] = acc + d->b[l][o];
            }
        }
        if (l < d->L - 1) {
            for (int o = 0; o < no; ++o) {
                double g = gelu(z[o]);
                a[o] = (mode == 1) ? (double)orc_bf16_round((float)g) : g;
            }
        } else {
            for (int o = 0; o < no; ++o) u[o] = z[o];
        }
    }
    free(a);
    free(z);
}

/* ---- FP8 inference (OCP 8-bit floating point, E4M3FN variant) ----------------
 * E4M3FN: 1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits, no infinities;
 * the largest finite magnitude is 1.75 * 2^8 = 448, normal numbers start at 2^-6
 * and the subnormal spacing is 2^-9.  Rounding is to nearest, ties to even. */
double orc_fp8_e4m3_round(double x) {
    if (!isfinite(x)) return NAN;
    double a = fabs(x);
    if (a == 0.0) return x;
    int e2;
    frexp(a, &e2);             /* a = f * 2^e2, f in [0.5, 1): floor(log2 a) = e2 - 1 */
    int E = e2 - 1;
    if (E < -6) E = -6;        /* below the normal range the spacing stays 2^-9 */
    double q = ldexp(1.0, E - 3);
    double r = nearbyint(a / q) * q; /* a / q is exact; nearbyint rounds ties to even */
    if (r > 448.0) return NAN; /* rounds beyond the format (not reached for scaled values) */
    return copysign(r, x);
}

/* smallest e with amax <= 448 * 2^e, so that amax * 2^-e lies in the E4M3FN range; 0 for amax 0;
 * at least -127, the smallest power of two an E8M0 block scale holds (a block whose largest
 * magnitude is below 448 * 2^-127 keeps the scale 2^-127 and its values round at the FP8 grid) */
int orc_fp8_scale_exp(double amax) {
    if (!(amax > 0.0) || !isfinite(amax)) return 0; /* no finite scale covers it: the values decide */
    int e = 0;
    while (amax > ldexp(448.0, e)) ++e;
    while (amax <= ldexp(448.0, e - 1)) --e;
    return e < -127 ? -127 : e;
}

/* Batched forward with the hidden-to-hidden layers in FP8: layer l (1 <= l <= L-2) quantises each
 * row of its input activations in blocks of 32 consecutive values, block q of row i with its own
 * power-of-two scale 2^e_iq (from the block's largest magnitude; a last block shorter than 32
 * takes the values there are), and each weight row with its own power-of-two scale; it sums the
 * exact products of the quantised values over each block, undoes the block's scale, sums the
 * blocks, and undoes the weight row's scale before the bias and GELU.  The first layer and the
 * output layer are those of mode 1 (bf16 values, fp32 sums); every hidden activation is rounded
 * to bf16.  xn: n x n_in (a zero row for a cell the network does not predict); u: n x n_out. */
void orc_mlp_forward_fp8(const orc_dnn *d, int64_t n, const double *xn, double *u) {
    int maxw = 0;
    for (int l = 0; l <= d->L; ++l) if (d->dims[l] > maxw) maxw = d->dims[l];
    double *A = malloc(sizeof(double) * (size_t)n * maxw), *B = malloc(sizeof(double) * (size_t)n * maxw);
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < d->n_in; ++c) A[i * d->n_in + c] = (double)orc_bf16_round((float)xn[i * d->n_in + c]);
    for (int l = 0; l < d->L; ++l) {
        const int ni = d->dims[l], no = d->dims[l + 1];
        const int fp8 = (l >= 1 && l <= d->L - 2);
        const int nb = (ni + 31) / 32;
        int *ea = NULL;
        double *wq = NULL;
        int *ew = NULL;
        if (fp8) {
            ea = malloc(sizeof(int) * (size_t)n * nb);
            for (int64_t i = 0; i < n; ++i)
                for (int q = 0; q < nb; ++q) {
                    double *a = &A[i * ni];
                    const int c1 = (32 * q + 32 < ni) ? 32 * q + 32 : ni;
                    double amax = 0.0;
                    for (int c = 32 * q; c < c1; ++c) amax = fmax(amax, fabs(a[c]));
                    const int e = orc_fp8_scale_exp(amax);
                    ea[i * nb + q] = e;
                    for (int c = 32 * q; c < c1; ++c) a[c] = orc_fp8_e4m3_round(ldexp(a[c], -e));
                }
            wq = malloc(sizeof(double) * (size_t)no * ni);
            ew = malloc(sizeof(int) * no);
            for (int o = 0; o < no; ++o) {
                const double *w = &d->W[l][(size_t)o * ni];
                double wmax = 0.0;
                for (int c = 0; c < ni; ++c) wmax = fmax(wmax, fabs(w[c]));
                ew[o] = orc_fp8_scale_exp(wmax);
                for (int c = 0; c < ni; ++c) wq[(size_t)o * ni + c] = orc_fp8_e4m3_round(ldexp(w[c], -ew[o]));
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double *a = &A[i * ni];
            for (int o = 0; o < no; ++o) {
                double z;
                if (fp8) {
                    double acc = 0.0;
                    for (int q = 0; q < nb; ++q) {
                        const int c1 = (32 * q + 32 < ni) ? 32 * q + 32 : ni;
                        double s = 0.0;
                        for (int c = 32 * q; c < c1; ++c) s += a[c] * wq[(size_t)o * ni + c];
                        acc += ldexp(s, ea[i * nb + q]);
                    }
                    z = ldexp(acc, ew[o]) + d->b[l][o];
                } else {
                    const double *w = &d->W[l][(size_t)o * ni];
                    float acc = 0.0f;
                    for (int c = 0; c < ni; ++c) acc = acc + (float)w[c] * (float)a[c];
                    acc = acc + (float)d->b[l][o];
                    z = acc;
                }
                if (l < d->L - 1)
                    B[i * no + o] = (double)orc_bf16_round((float)gelu(z));
                else
                    u[i * no + o] = z;
            }
        }
        free(wq);
        free(ew);
        free(ea);
        double *t = A;
        A = B;
        B = t;
    }
    free(A);
    free(B);
}

/* Newton on T -> h(T, Y) - h_target with dh/dT = cp */
int orc_T_from_h(const orc_mech *m, double h_target, const double *Y, double T_guess, double *T_out) {
    double T = T_guess;
    for (int it = 1; it <= 20; ++it) {
        double cp, h;
        orc_mixture(m, T, P_REF, Y, NULL, NULL, &cp, &h);
        double dT = (h - h_target) / cp;
        T -= dT;
        if (!isfinite(T)) break;
        if (fabs(dT) <= 1e-9) { *T_out = T; return it; }
    }
    *T_out = T;
    return -1;
}

int orc_dnn_step(const orc_dnn *d, const orc_mech *m, int64_t n, int64_t ld, double dt, const double *p, double *T,
                 double *Y, double *rr, int32_t *status, int renormalise, int mode, int fallback, const orc_opts *opts,
                 int nthreads) {
    if (!d || !m || d->K != m->K || n < 0 || ld < n || !p || !T || !Y) return -1;
    orc_opts o = default_opts(opts);
    int K = m->K;
    int fails = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* mode 2: the network runs on the whole batch first (its activation scales are batch-wide) */
    double *U = NULL;
    if (mode == 2) {
        double *X = calloc((size_t)n * d->n_in, sizeof(double));
        U = calloc((size_t)n * d->n_out, sizeof(double));
        for (int64_t i = 0; i < n; ++i) {
            double x[ORC_MAX_SPECIES + 2];
            int ok = isfinite(T[i]) && T[i] > 0 && isfinite(p[i]) && p[i] > 0;
            x[0] = T[i];
            x[1] = p[i];
            for (int k = 0; k < K; ++k) {
                ok = ok && isfinite(Y[k * ld + i]);
                x[2 + k] = orc_bct(Y[k * ld + i], d->lambda);
            }
            for (int j = 0; ok && j < d->n_in; ++j) ok = (x[j] >= d->lo[j]) && (x[j] <= d->hi[j]);
            if (ok)
                for (int j = 0; j < d->n_in; ++j) X[i * d->n_in + j] = (x[j] - d->mu_in[j]) / d->sig_in[j];
        }
        orc_mlp_forward_fp8(d, n, X, U);
        free(X);
    }
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : fails)
    for (int64_t i = 0; i < n; ++i) {
        double Y0[ORC_MAX_SPECIES], x[ORC_MAX_SPECIES + 2], xn[ORC_MAX_SPECIES + 2], u[ORC_MAX_SPECIES];
        double Yn[ORC_MAX_SPECIES];
        for (int k = 0; k < K; ++k) Y0[k] = Y[k * ld + i];
        double T0 = T[i];
        double rho0 = 0.0, h0 = 0.0;
        int st = ORC_OK;
        int finite = isfinite(T0) && T0 > 0 && isfinite(p[i]) && p[i] > 0;
        for (int k = 0; k < K; ++k) finite = finite && isfinite(Y0[k]);
        if (!finite) {
            if (status) status[i] = ORC_NONFINITE;
            if (rr) for (int k = 0; k < K; ++k) rr[k * ld + i] = 0.0;
            fails += 1;
            continue;
        }
        orc_mixture(m, T0, p[i], Y0, NULL, &rho0, NULL, &h0);
        /* stage 1: Box-Cox transform and normalisation, with the training-range test */
        x[0] = T0;
        x[1] = p[i];
        for (int k = 0; k < K; ++k) x[2 + k] = orc_bct(Y0[k], d->lambda);
        int in_box = 1;
        for (int j = 0; j < d->n_in; ++j) in_box = in_box && (x[j] >= d->lo[j]) && (x[j] <= d->hi[j]);
        if (!in_box) {
            if (fallback) {
                double y[ORC_MAX_SPECIES + 1];
                y[0] = T0;
                for (int k = 0; k < K; ++k) y[1 + k] = Y0[k];
                int acc, rej;
                st = chem_cell(m, dt, p[i], y, NULL, &o, &acc, &rej, 0);
                T[i] = y[0];
                for (int k = 0; k < K; ++k) Y[k * ld + i] = y[1 + k];
                st = (st == ORC_OK) ? ORC_DNN_FALLBACK : st;
            } else {
                st = ORC_DNN_FALLBACK;
            }
        } else {
            for (int j = 0; j < d->n_in; ++j) xn[j] = (x[j] - d->mu_in[j]) / d->sig_in[j];
            /* stage 2: the network */
            if (mode == 2)
                memcpy(u, &U[i * d->n_out], sizeof(double) * d->n_out);
            else
                orc_mlp_forward(d, xn, u, mode);
            /* stage 3: undo the normalisation and the transform, recover T from h */
            double sum = 0.0;
            for (int k = 0; k < K; ++k) {
                double z1 = x[2 + k] + (u[k] * d->sig_out[k] + d->mu_out[k]);
                Yn[k] = orc_bct_inv(z1, d->lambda);
                sum += Yn[k];
            }
            if (renormalise && sum > 0)
                for (int k = 0; k < K; ++k) Yn[k] /= sum;
            double T1;
            int it = orc_T_from_h(m, h0, Yn, T0, &T1);
            if (it < 0) st = ORC_NONFINITE;
            T[i] = T1;
            for (int k = 0; k < K; ++k) Y[k * ld + i] = Yn[k];
        }
        if (rr)
            for (int k = 0; k < K; ++k) rr[k * ld + i] = rho0 * (Y[k * ld + i] - Y0[k]) / dt;
        if (status) status[i] = st;
        if (st != ORC_OK && st != ORC_DNN_FALLBACK) fails += 1;
    }
    free(U);
    return fails;
}
