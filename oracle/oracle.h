/*
 * CPU oracle for the per-cell chemistry step (test infrastructure only).
 *
 * A plain, slow, FP64 implementation of what the GPU library computes, used
 * by the tests, the smoke check and the CPU baseline of the benchmark to
 * decide whether the GPU results are right.  It shares no code, header,
 * table or helper with the GPU library: only the input files (mechanism,
 * DNN weights, fields) are common.  Nothing in the product may link it.
 *
 * Paper passages followed (DeepFlame, arXiv 2210.07094):
 *   - species source term: Sec. "Chemistry Integration", the equation for
 *     dY/dt as a sum over reactions of forward minus reverse mass-action
 *     terms with Arrhenius rate constants;
 *   - constant-pressure 0-D reactor: Sec. "DeepFlame Solvers" (df0DFoam);
 *   - enthalpy-based thermo update: Sec. "Description of the new classes"
 *     (correctThermo rebuilds the state from h, p, Y);
 *   - DNN integrator: Sec. "Chemistry Integration" (input T, P, Box-Cox(Y);
 *     three hidden layers; output = change over a 1 us step) and the three
 *     stages of DNNInferencer::inference.
 * Where the paper is silent (rate forms beyond Arrhenius, thermo fits, the
 * integration scheme) the textbook definitions are used: NASA-7 polynomials,
 * Lindemann/Troe falloff, equilibrium constants from Gibbs energies, and the
 * 6-stage Rosenbrock method RODAS4 of Hairer & Wanner (Solving ODEs II,
 * Sec. IV.7) in its transformed form.
 */
#ifndef DF_ORACLE_H
#define DF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_SPECIES 128

typedef struct {
    char name[256];
    long seed;
    int E, K, M;
    double *element_mass; /* [E] g/mol */
    double *W;            /* [K] kg/mol */
    int *comp;            /* [K*E] */
    double *nasa;         /* [K*7] */
    int *type;            /* [M] 0 elementary, 1 third body, 2 Troe */
    int *nu_r, *nu_p;     /* [M*K] */
    double *arr;          /* [M*3] A, b, Ta (CGS) */
    double *eff;          /* [M*K] */
    double *low;          /* [M*3] */
    double *troe;         /* [M*4] alpha, T3, T1, T2 */
} orc_mech;

typedef struct {
    double rtol, atol_T, atol_Y, h_min;
    int32_t max_steps;
} orc_opts;

/* per-cell status codes */
enum { ORC_OK = 0, ORC_MAX_STEPS = 1, ORC_H_UNDERFLOW = 2, ORC_NONFINITE = 3, ORC_DNN_FALLBACK = 4 };

orc_mech *orc_mech_load(const char *path);
void orc_mech_free(orc_mech *m);
int orc_mech_dims(const orc_mech *m, int *K, int *M, int *E);

/* thermo of every species at T: cp/R, H/(RT), S/R, G/(RT) */
void orc_species_thermo(const orc_mech *m, double T, double *cp_R, double *h_RT, double *s_R, double *g_RT);
/* mixture: mean molar mass [kg/mol], density [kg/m3], cp [J/kg/K], h [J/kg] */
void orc_mixture(const orc_mech *m, double T, double p, const double *Y, double *Wbar, double *rho,
                 double *cp_mass, double *h_mass);
/* per-reaction kf, kr (CGS), net progress rate q (mol/cm3/s) and wdot (mol/m3/s) */
void orc_rates(const orc_mech *m, double T, double p, const double *Y, double *kf, double *kr, double *q,
               double *wdot);
/* ODE right-hand side f(y), y = (T, Y_1..Y_K), constant p */
void orc_rhs(const orc_mech *m, double p, const double *y, double *f);
/* analytic Jacobian J[i*N + j] = d f_i / d y_j, N = K + 1 */
void orc_jacobian(const orc_mech *m, double p, const double *y, double *J);

/* constant-volume reactor (rho fixed, p = rho R T / Wbar): right-hand side, analytic Jacobian,
 * and the step of n cells with density rho [n] (arguments otherwise as orc_chem_step) */
void orc_rhs_v(const orc_mech *m, double rho, const double *y, double *f);
void orc_jacobian_v(const orc_mech *m, double rho, const double *y, double *J);
int orc_chem_step_v(const orc_mech *m, int64_t n, int64_t ld, double dt, const double *rho, double *T, double *Y,
                    double *h_inout, int32_t *status, int32_t *n_acc, int32_t *n_rej, const orc_opts *opts,
                    int nthreads);

/* RODAS4 coefficients in transformed form: gamma, a[6*6], c[6*6], m[6], mhat[6] */
void orc_rodas4_tableau(double *gamma, double *a, double *c, double *mm, double *mhat);

/* sensitivities of the step (test support): integrate one cell y = (T, Y) in
 * place from a fresh start, recording accepted sub-step lengths in
 * h_rec[0 .. min(n_acc, rec_cap)); replay nh fixed RODAS4 sub-steps of
 * lengths hs from y (no error control); scale A of reaction j (k_inf for
 * Troe rows) by factor */
int orc_chem_cell_record(const orc_mech *m, double dt, double p, double *y, const orc_opts *opts, double *h_rec,
                         int32_t rec_cap, int32_t *n_acc, int32_t *n_rej);
void orc_chem_replay(const orc_mech *m, double p, double *y, const double *hs, int32_t nh);
void orc_mech_scale_A(orc_mech *m, int32_t j, double factor);

/* Adaptive integration of y' = A y over dt (tests of the integrator core). */
int orc_linear_integrate(int n, const double *A, double *y, double dt, double h_in, const orc_opts *o,
                         double *atol, double *h_next, int32_t *n_acc, int32_t *n_rej);
/* One fixed RODAS4 step of size h of y' = A y (no error control). */
void orc_linear_fixed_step(int n, const double *A, double *y, double h, double *err_vec);

/* Chemistry step over n cells: SoA Y[k*ld + i]; T, Y in/out. Optional arrays may be NULL. */
int orc_chem_step(const orc_mech *m, int64_t n, int64_t ld, double dt, const double *p, double *T, double *Y,
                  double *h_inout, double *rr, int32_t *status, int32_t *n_acc, int32_t *n_rej,
                  const orc_opts *o, int nthreads);
/* The same with a step length per cell: dt_cells[n] (each > 0), or NULL to use dt for all. */
int orc_chem_step_dt(const orc_mech *m, int64_t n, int64_t ld, double dt, const double *dt_cells, const double *p,
                     double *T, double *Y, double *h_inout, double *rr, int32_t *status, int32_t *n_acc,
                     int32_t *n_rej, const orc_opts *o, int nthreads);

/* ---- DNN form ---- */
typedef struct orc_dnn orc_dnn;
orc_dnn *orc_dnn_load(const char *path);
void orc_dnn_free(orc_dnn *d);
int orc_dnn_dims(const orc_dnn *d, int *n_layers, int *dims /* n_layers+1 */, int *K, double *lambda,
                 double *dt_train);
/* Box-Cox transform of one mass fraction and its inverse (clamps per the reading of the paper) */
double orc_bct(double Y, double lambda);
double orc_bct_inv(double z, double lambda);
/* bf16 round-to-nearest-even of an fp32 value, returned as fp32 */
float orc_bf16_round(float x);
/* MLP forward on one normalised input vector; mode 0 = FP64, 1 = BF16-emulated (fp32 accumulate) */
void orc_mlp_forward(const orc_dnn *d, const double *x_norm, double *u, int mode);
/* nearest OCP E4M3FN value of x (ties to even); NaN where the rounded magnitude exceeds 448 or x is not finite */
double orc_fp8_e4m3_round(double x);
/* smallest e with amax <= 448 * 2^e (0 for amax 0 or not finite, at least -127): the power-of-two
   scale of an FP8 block */
int orc_fp8_scale_exp(double amax);
/* batched forward with the hidden-to-hidden layers in FP8 (a power-of-two activation scale per
   row and block of 32 inputs, per-row power-of-two weight scales, exact sums); first and output
   layers as mode 1.
   xn: n x n_in normalised inputs (zero rows for cells the network does not predict); u: n x n_out */
void orc_mlp_forward_fp8(const orc_dnn *d, int64_t n, const double *xn, double *u);
/* T from enthalpy at fixed p and composition: Newton from T_guess; returns iterations or -1 */
int orc_T_from_h(const orc_mech *m, double h_target, const double *Y, double T_guess, double *T_out);
/* DNN chemistry step over n cells; cells outside the training box fall back to orc_chem_step.
   renormalise: 1 = rescale sum Y to 1; mode as orc_mlp_forward, or 2 = orc_mlp_forward_fp8 over the
   batch; fallback: 1 = integrate, 0 = leave. */
int orc_dnn_step(const orc_dnn *d, const orc_mech *m, int64_t n, int64_t ld, double dt, const double *p,
                 double *T, double *Y, double *rr, int32_t *status, int renormalise, int mode, int fallback,
                 const orc_opts *o, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
