/*
 * df.h -- C ABI of the MI355X (gfx950) per-cell chemistry step library.
 *
 * The library advances the thermochemical state of N independent cells over
 * one chemistry sub-step of an operator-split reacting-flow solver, in the
 * two forms of DeepFlame (arXiv 2210.07094):
 *   (a) detailed chemistry integrated by a stiff solver (the paper integrates
 *       the species source-term equation of Sec. "Chemistry Integration" with
 *       CVODE; this library uses the L-stable Rosenbrock method RODAS4 with
 *       error control, Hairer & Wanner, Solving ODEs II, Sec. IV.7), and
 *   (b) the paper's DNN integrator (same section: input T, P and the Box-Cox
 *       transform of Y; three hidden layers; output = change of the input
 *       over a 1 us step), in the three stages of DNNInferencer::inference
 *       (Sec. "Description of the new classes").
 * The flow solver hands over (p, T, Y) per cell and receives the new state and
 * the reaction rates (the OpenFOAM <-> chemistry coupling of Sec. "DeepFlame
 * Code Structure"; dfChemistryModel::solve() and RR()).
 *
 * Conventions shared by every call
 *  - All state arrays are caller-owned DEVICE memory on the handle's device.
 *    The library never frees them and keeps no reference after the call.
 *  - Layout is structure-of-arrays: per-cell scalars are [n] arrays; species
 *    arrays are species-major, element (k, i) at Y[k * ld + i], ld >= n.
 *  - Units are SI: p [Pa], T [K], dt [s], rr [kg/m^3/s]; Y are mass fractions.
 *  - Calls that take a hip_stream (a hipStream_t, NULL = default stream) are
 *    asynchronous on it.  Argument errors are detected on the host and
 *    returned before anything is launched; outputs are valid once the stream
 *    has completed.
 *  - Return value: DF_OK (0) on success, a negative DF_E_* code on error (no
 *    output has been written).  df_last_error() then describes the error.
 *  - Per-cell outcomes go to cell_status[i] (DF_CELL_*), when given.
 *  - Handles are immutable after load and may be shared by threads.
 */
#ifndef DF_H
#define DF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t df_status;

/* return codes */
#define DF_OK 0
#define DF_E_INVALID (-1)     /* bad argument (null pointer, n < 0, ld < n, dt <= 0, ...) */
#define DF_E_UNSUPPORTED (-2) /* valid but not supported (too many species, dt != DNN training dt, ...) */
#define DF_E_HIP (-3)         /* HIP runtime error (allocation, copy, launch) */
#define DF_E_IO (-4)          /* file cannot be opened or read */
#define DF_E_FORMAT (-5)      /* file content malformed */
#define DF_CELL_FAILURES 1    /* df_step_stats only: the step ran, and at least one cell failed
                                 (status MAX_STEPS, H_UNDERFLOW, NONFINITE or TAPE_FULL) */

/* per-cell status codes */
#define DF_CELL_OK 0
#define DF_CELL_MAX_STEPS 1    /* integrator stopped after max_steps attempts; state as reached */
#define DF_CELL_H_UNDERFLOW 2  /* a rejected step pushed h below h_min; state as reached */
#define DF_CELL_NONFINITE 3    /* input not finite / T <= 0 / p <= 0 (state untouched), or the DNN
                                  temperature recovery did not converge */
#define DF_CELL_DNN_FALLBACK 4 /* DNN form: cell outside the network's training range, advanced by
                                  the integrator instead (success) */
#define DF_CELL_TAPE_FULL 5    /* taped step: more accepted sub-steps than the tape holds; state as
                                  integrated, no tape (the adjoint gives zero gradients) */

typedef struct df_mech df_mech;       /* opaque mechanism handle */
typedef struct df_dnn df_dnn;         /* opaque DNN handle */
typedef struct df_trainer df_trainer; /* opaque DNN training state */

/* Integrator options (see df_chem_default_opts for the defaults). */
typedef struct {
    double rtol;       /* relative tolerance, default 1e-8 */
    double atol_T;     /* absolute tolerance on T [K], default 1e-6 */
    double atol_Y;     /* absolute tolerance on Y, default 1e-14 */
    double h_min;      /* smallest sub-step [s], default 1e-20 */
    int32_t max_steps; /* attempted sub-steps per cell and call, default 100000 */
    int32_t mapping;   /* work mapping of the static schedule: 0 (default) automatic, 1 one cell
                          per lane, 2 sixteen lanes per cell (species count <= 15), 3 one
                          wavefront (64 lanes) per cell (species count <= 63), 4 thirty-two
                          lanes per cell (as 2, the second 16 lanes taking half of the rate
                          constants: a shorter sub-step for stiff cells, half the cells per wave;
                          16 lanes where the reaction slots do not divide in two), 5 thirty-two
                          lanes for the 512 cells at the head of the cost order (the stiffest,
                          whose sub-step chains set the launch's time) and sixteen for the rest
                          (needs the workspace, which holds the order; as 2 without it);
                          automatic takes 5 where the reaction slots divide in two, else 16 lanes,
                          where compiled, else one cell per lane, else a wavefront.  Mappings 2, 4
                          and 5 give the same bits */
    int32_t schedule;  /* 0 (default) or 1: static, one launch that gives each lane (or group of
                          16 lanes) one cell; 2: persistent work queue (needs the workspace):
                          cells sorted by estimated cost (temperature, then step length) are
                          claimed from a device queue as lanes become free, by 16-lane groups
                          from the stiff end; optionally some waves first take the cold cells
                          (about 500 K and below) from the other end one cell per lane */
    int32_t coop_blocks; /* queue schedule: waves that start as 16-lane groups; the others start
                            one cell per lane on the cold cells and then join the groups.
                            0 (default) all resident waves, -1 none, k > 0 k waves (capped at
                            the resident count); df_chem_autotune picks it */
} df_chem_opts;

/* DNN options. */
typedef struct {
    int32_t renormalise; /* 1 (default): rescale the predicted Y to sum 1 */
    int32_t fallback;    /* 1 (default): integrate cells outside the training range;
                            0: leave them unchanged and flag DF_CELL_DNN_FALLBACK */
    int32_t precision;   /* 0 (default): every hidden layer in bf16 (fp32 sums);
                            1: the layers between two hidden layers in FP8 (OCP E4M3FN on the
                            block-scaled matrix cores, fp32 sums), an inference variant the
                            paper's BF16 network does not fix: each row of a layer's input
                            activations takes one power-of-two scale per block of 32 values
                            (from the block's largest |value|, at least 2^-127), weights one
                            power-of-two scale per row, quantised at load; round to nearest
                            even.  The first hidden layer and the output layer stay as with 0;
                            a first layer with more than 64 padded inputs is refused
                            (DF_E_UNSUPPORTED) */
    int32_t reserved1;   /* must be 0 */
} df_dnn_opts;

/* Message describing the last error of this thread; valid until the next df_* call. */
const char *df_last_error(void);

/* Library version string. */
const char *df_version(void);

void df_chem_default_opts(df_chem_opts *opts);
void df_dnn_default_opts(df_dnn_opts *opts);

/*
 * Load a mechanism file ("dfmech 1" text format: elements, species molar
 * masses and compositions, single-range NASA-7 thermo, reactions with
 * reactant/product stoichiometry, Arrhenius parameters in cm-mol-s units,
 * third-body efficiencies, Troe falloff parameters) and upload its tables to
 * `device`.  The species source term follows the paper's equation in Sec.
 * "Chemistry Integration"; the rate-constant forms (Arrhenius, third body,
 * Troe falloff, reverse rate from the equilibrium constant) are the standard
 * forms the paper leaves to Cantera.  At most 3 molecules per reaction side.
 * Errors: DF_E_INVALID (null path/out), DF_E_IO, DF_E_FORMAT, DF_E_HIP.
 * On success *out owns host and device tables; release with df_mech_free.
 */
df_status df_mech_load(const char *path, int32_t device, df_mech **out);
void df_mech_free(df_mech *mech);
df_status df_mech_info(const df_mech *mech, int32_t *n_species, int32_t *n_reactions, int32_t *n_elements);

/*
 * Summary of a finished step (the outcome of dfChemistryModel::solve() over the whole mesh,
 * Sec. "Description of the new classes"), reduced on the device from the per-cell outputs that
 * df_chem_step, df_chem_step_cells, df_chem_step_const_volume or df_dnn_step wrote.
 */
typedef struct {
    int64_t n_cells;
    int64_t count[8];     /* cells per status code DF_CELL_OK .. 7 (needs cell_status, else 0) */
    int64_t failed;       /* cells with MAX_STEPS, H_UNDERFLOW, NONFINITE or TAPE_FULL */
    int64_t accepted;     /* accepted sub-steps summed over the cells (needs n_steps, else 0) */
    int64_t rejected;     /* rejected sub-steps summed over the cells */
    int32_t max_attempts; /* largest accepted + rejected of one cell (0 without n_steps) */
    int32_t max_cell;     /* the lowest-index cell with that count (-1 without n_steps or cells) */
    double min_Y;         /* smallest mass fraction over the cells, NaN ignored (+inf without Y);
                             the integrator never clips negative mass fractions */
} df_stats;

/*
 * Reduce the outputs of a step into *stats_dev, asynchronously on hip_stream, ordered after the
 * step when launched on its stream.
 *   cell_status [n], n_steps [2n] (accepted at [i], rejected at [n + i]), Y [n_species * ld]:
 *               device arrays as the step wrote them, each nullable (its fields stay 0)
 *   stats_dev   device memory for one df_stats, 8-byte aligned, caller-owned, written
 *   stats_host  host memory for one df_stats, or NULL.  When given, the call waits for
 *               hip_stream, copies the summary there and returns DF_CELL_FAILURES (> 0) if any
 *               cell failed, DF_OK otherwise.  When NULL, nothing waits and DF_OK is returned.
 * Runs on the current device.  Errors: DF_E_INVALID (null or misaligned stats_dev, n_cells < 0
 * or >= 2^31, Y without n_species >= 1 and ld >= n_cells), DF_E_HIP.
 */
df_status df_step_stats(int64_t n_cells, int64_t ld, int32_t n_species, const int32_t *cell_status,
                        const int32_t *n_steps, const double *Y, df_stats *stats_dev, df_stats *stats_host,
                        void *hip_stream);

/* Bytes of device workspace df_chem_step / df_chem_step_cells can use for n_cells (see their
   `workspace`). */
df_status df_chem_workspace_size(const df_mech *mech, int64_t n_cells, size_t *bytes);

/*
 * Advance n_cells constant-pressure adiabatic reactors by dt (detailed
 * chemistry, the paper's dfChemistryModel::solve() with its stiff solver;
 * the species line is the source-term equation of Sec. "Chemistry
 * Integration" with the density written out, and T follows from constant
 * enthalpy at fixed p).
 *   p           [n]      in      pressure per cell
 *   T           [n]      in/out  temperature
 *   Y           [K*ld]   in/out  mass fractions
 *   h_inout     [n]      in/out  sub-step hint carried across calls (<= 0 or NULL: estimate)
 *   rr          [K*ld]   out     rho0 (Y - Y0) / dt, rho0 the density at the start (nullable)
 *   cell_status [n]      out     DF_CELL_* (nullable)
 *   n_steps     [2*n]    out     accepted sub-steps at [i], rejected at [n + i] (nullable)
 *   workspace   device memory of df_chem_workspace_size bytes, 256-byte aligned (nullable;
 *               required by the queue schedule).  With it, cells are integrated hottest first
 *               (a counting sort on temperature), so that the stiffest cells, whose sub-steps
 *               set the time of the call, start first; without it they are taken in index
 *               order.  Results do not depend on it beyond rounding of the first sub-step.
 *   opts        nullable = defaults
 * Cells with non-finite input are left untouched with DF_CELL_NONFINITE.
 * Errors: DF_E_INVALID (null handle/array, n < 0, ld < n, dt not > 0 and
 * finite, bad opts, workspace given but too small or misaligned, queue schedule without
 * workspace), DF_E_UNSUPPORTED (species count beyond the compiled kernels), DF_E_HIP.
 */
df_status df_chem_step(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *p, double *T,
                       double *Y, double *h_inout, double *rr, int32_t *cell_status, int32_t *n_steps,
                       void *workspace, size_t workspace_bytes, const df_chem_opts *opts, void *hip_stream);

/*
 * df_chem_step with a step length per cell (a chemistry step of a solver with local time
 * steps, or cells of different sub-systems in one call):
 *   dt          [n]      in      step length per cell [s], device memory, not NULL for n > 0
 * A cell whose dt is not positive and finite is left untouched with DF_CELL_NONFINITE; rr is
 * divided by the cell's own dt.  With the workspace, cells are ordered hottest first and,
 * within a temperature bucket, longest step first.  Other arguments and errors as
 * df_chem_step.
 */
df_status df_chem_step_cells(const df_mech *mech, int64_t n_cells, int64_t ld, const double *dt, const double *p,
                             double *T, double *Y, double *h_inout, double *rr, int32_t *cell_status,
                             int32_t *n_steps, void *workspace, size_t workspace_bytes, const df_chem_opts *opts,
                             void *hip_stream);

/*
 * df_chem_step for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the cost-ordering and queue workspace
 * is the library's own static device array instead of a caller workspace, so the call allocates
 * nothing.  Arguments, schedules, results and errors as df_chem_step with a workspace, for at most
 * 1,048,576 cells per call (more: DF_E_UNSUPPORTED before anything is launched).  The array
 * (about 4.2 MB on each device the library runs on) is held until the process ends and is shared
 * by every call on that device: calls that overlap on one device (several streams or host
 * threads at once) race on it and must not be issued.  Each call clears what it needs itself.
 */
df_status df_chem_step_noalloc(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *p, double *T,
                               double *Y, double *h_inout, double *rr, int32_t *cell_status, int32_t *n_steps,
                               const df_chem_opts *opts, void *hip_stream);

/*
 * The constant-volume reactor (df0DFoam's constant-volume case): density fixed per cell,
 * pressure following from the state (p = rho R T / Wbar),
 *   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k U_k wdot_k / (rho cv),
 * U_k = H_k - R T, cv = cp - R / Wbar; the mixture internal energy is conserved.
 *   rho         [n]      in      density per cell [kg/m^3]
 *   T, Y, h_inout, cell_status, n_steps, opts: as df_chem_step (one cell per lane for the
 *               species counts with that kernel, else one wavefront per cell for up to 63
 *               species; opts.mapping and opts.schedule are ignored)
 * A cell whose rho or T is not positive and finite, or whose Y is not finite, is left untouched
 * with DF_CELL_NONFINITE.  Errors: DF_E_INVALID, DF_E_UNSUPPORTED, DF_E_HIP.
 */
df_status df_chem_step_const_volume(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *rho,
                                    double *T, double *Y, double *h_inout, int32_t *cell_status, int32_t *n_steps,
                                    const df_chem_opts *opts, void *hip_stream);

/* reactors of df_rollout */
#define DF_REACTOR_CONST_P 0
#define DF_REACTOR_CONST_V 1

/*
 * 0-D rollouts (the paper's 0-D autoignition cases and ignition-delay curves, Sec. "df0DFoam-
 * solver"; the delay is taken at the largest dT/dt): n_steps consecutive chemistry steps of
 * length dt of the DNN form (dnn != NULL, df_dnn_step with its fallback) or of the integrator
 * (dnn == NULL: df_chem_step, or df_chem_step_const_volume for DF_REACTOR_CONST_V, carrying each
 * cell's sub-step hint), on (T, Y) in place, tracking each cell's ignition delay: the time of the
 * largest temperature rate, r_k = (T_{k+1} - T_k)/dt at t_k = (k + 1/2) dt, refined by the vertex
 * of the parabola through the rates of the steps around it.
 *   reactor                in      DF_REACTOR_CONST_P, or DF_REACTOR_CONST_V (integrator only)
 *   p [n]                  in      pressure [Pa]; the density [kg/m^3] for DF_REACTOR_CONST_V
 *   T [n], Y [K*ld]        in/out  state (after n_steps steps on return)
 *   idt [n]                out     ignition delay [s]; NaN when the largest rate falls on the
 *                                  first or last step
 *   T_traj [(n_steps+1)*n] out     temperature after each step, row 0 the initial one (nullable)
 *   workspace             device memory of df_rollout_workspace_size bytes (enough for either
 *                         reactor), 256-byte aligned
 *   opts                  integrator options (also the DNN's fallback), nullable
 * Errors: DF_E_INVALID (also a DNN with DF_REACTOR_CONST_V), those of df_chem_step /
 * df_chem_step_const_volume / df_dnn_step, DF_E_HIP.
 */
df_status df_rollout_workspace_size(const df_mech *mech, const df_dnn *dnn, int64_t n_cells, size_t *bytes);
df_status df_rollout(const df_mech *mech, const df_dnn *dnn, int64_t n_cells, int64_t ld, double dt, int32_t n_steps,
                     int32_t reactor, const double *p, double *T, double *Y, double *idt, double *T_traj, void *workspace,
                     size_t workspace_bytes, const df_chem_opts *opts, void *hip_stream);

/* Bytes of device workspace df_chem_autotune needs for n_cells. */
df_status df_chem_autotune_workspace_size(const df_mech *mech, int64_t n_cells, size_t *bytes);

/*
 * Pick the schedule of df_chem_step / df_chem_step_cells for a workload (the cells-per-wave
 * choice of uneven stiffness: one cell per 16 or 32 lanes, or one cell per lane for all cells or
 * for the cold cells first): time one step of each candidate -- static schedule with the cost
 * order, with the given mapping (the automatic one runs the 32-lane head of mapping 5 there) and
 * (for the automatic or 16-lane mapping) with 32 lanes per cell and with one cell per lane (where that kernel is compiled for the species count); queue
 * schedule with every wave as 16-lane groups; queue schedule with a half or a quarter of the
 * waves as 16-lane groups from the start -- on copies of the input, and write the fastest into
 * opts->schedule, opts->coop_blocks and opts->mapping (the other fields are kept and used for
 * the trials).
 *   dt, dt_cells  step length of every cell, or per cell (dt_cells [n] device, nullable)
 *   p, T, Y       the workload, device memory, layouts as df_chem_step; not modified
 *   workspace     device memory of df_chem_autotune_workspace_size bytes, 256-byte aligned
 * Synchronous: returns after the trials have run on hip_stream.
 * Errors: DF_E_INVALID (null handle/opts/array, n < 0, ld < n, dt, bad opts, workspace missing,
 * too small or misaligned), DF_E_UNSUPPORTED, DF_E_HIP.
 */
df_status df_chem_autotune(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *dt_cells,
                           const double *p, const double *T, const double *Y, void *workspace, size_t workspace_bytes,
                           df_chem_opts *opts, void *hip_stream);

/*
 * ---- Discrete adjoint of the chemistry step ----
 * Gradients of the state after one chemistry step with respect to the state before it and to
 * the log pre-exponential factors (the integration of the source-term equation of Sec.
 * "Chemistry Integration" as df_chem_step does it, differentiated).  The step is the sequence
 * of accepted RODAS4 sub-steps that df_chem_step_taped took, with their lengths held fixed
 * (the step-size controller's choices are not differentiated), so the gradient is the exact
 * derivative of the computed result, up to rounding.
 *
 * Bytes of tape (the adjoint's checkpoints: for each accepted sub-step its start state, its
 * length, the inverse of its iteration matrix and its six stage vectors) for n_cells and at
 * most max_substeps accepted sub-steps per cell: 8 max_substeps (N^2 + 7N + 1) n_cells +
 * 4 n_cells with N = K + 1.
 */
df_status df_chem_tape_size(const df_mech *mech, int64_t n_cells, int32_t max_substeps, size_t *bytes);

/*
 * df_chem_step (16 lanes per cell, each cell from a fresh start: no sub-step hint, no rr)
 * that also records the tape for df_chem_adjoint.
 *   p, T, Y, cell_status, n_steps, opts: as df_chem_step
 *   tape          device memory of df_chem_tape_size(mech, n_cells, max_substeps) bytes,
 *                 256-byte aligned, written; keep it (and p) unchanged until the adjoint ran.
 *                 Layout, with N = K + 1, S = max_substeps and every array cell-minor (stride
 *                 n_cells): f64 [S][N] start states, f64 [S] sub-step lengths, f64 [S][N*N]
 *                 inverses of W = I/(gamma h) - J (row-major), f64 [S][6*N] stage vectors
 *                 (stage-major), then int32 [n_cells] sub-step counts (-1: the cell has no tape).
 * A cell with more accepted sub-steps than max_substeps keeps its integrated state and gets
 * DF_CELL_TAPE_FULL (no tape); cells that fail as in df_chem_step get no tape either.
 * Errors: DF_E_INVALID (as df_chem_step; max_substeps < 1; tape null, too small or misaligned),
 * DF_E_UNSUPPORTED (no 16-lane integrator or adjoint kernel for the mechanism), DF_E_HIP.
 */
df_status df_chem_step_taped(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *p,
                             double *T, double *Y, int32_t *cell_status, int32_t *n_steps, void *tape,
                             size_t tape_bytes, int32_t max_substeps, const df_chem_opts *opts, void *hip_stream);

/* Bytes of device workspace df_chem_adjoint needs for n_cells: 8 M n_cells. */
df_status df_chem_adjoint_workspace_size(const df_mech *mech, int64_t n_cells, size_t *bytes);

/*
 * Reverse sweep: given the adjoint (T_bar, Y_bar) of the state after the taped step (for a
 * scalar loss L, dL/dT and dL/dY), return the adjoint of the state before it and of ln A:
 *   (T0_bar, Y0_bar) = (dy/dy0)^T (T_bar, Y_bar) and lnA_bar = (dy/dlnA)^T (T_bar, Y_bar) per cell.
 *   p              [n]           in    the pressures the taped step used
 *   tape, max_substeps                 as written by df_chem_step_taped for the same n_cells
 *   T_bar [n], Y_bar [K*ld]      in    seeds
 *   T0_bar [n], Y0_bar [K*ld]    out   adjoint of (T0, Y0)
 *   lnA_bar_cells [M*ld]         out   per cell, d L / d ln A_j (row j in the mechanism file's
 *                                      reaction order; k_inf's A for falloff rows) (nullable)
 *   lnA_bar [M]                  out   the same summed over cells, in a fixed order (nullable)
 *   workspace     device memory of df_chem_adjoint_workspace_size bytes, 256-byte aligned
 * Cells without a tape get zero gradients.  Inputs are not modified.  The tape, the seeds and
 * the outputs are caller-owned device memory; nothing is kept after the call.
 * Errors: DF_E_INVALID (null handle/array, n < 0, ld < n, max_substeps < 1, tape or workspace
 * too small or misaligned), DF_E_UNSUPPORTED, DF_E_HIP.
 */
df_status df_chem_adjoint(const df_mech *mech, int64_t n_cells, int64_t ld, const double *p, const void *tape,
                          size_t tape_bytes, int32_t max_substeps, const double *T_bar, const double *Y_bar,
                          double *T0_bar, double *Y0_bar, double *lnA_bar_cells, double *lnA_bar, void *workspace,
                          size_t workspace_bytes, void *hip_stream);

/*
 * Load a DNN weights file ("DFDNN01", little-endian: int32 L, dims[L+1], K,
 * reserved; f64 lambda, dt_train; f64 mu_in[K+2], sig_in[K+2], mu_out[K],
 * sig_out[K], box_lo[K+2], box_hi[K+2]; per layer bf16 W[out][in], f32
 * b[out]).  Inputs are (T, p, BoxCox(Y_1..Y_K)) and outputs the normalised
 * increments of BoxCox(Y) over dt_train, the structure of Sec. "Chemistry
 * Integration" (three hidden layers, GELU).  `mech` must have the same K.
 * Errors: DF_E_INVALID, DF_E_IO, DF_E_FORMAT, DF_E_UNSUPPORTED (layer count
 * or widths the kernels do not take), DF_E_HIP.
 */
df_status df_dnn_load(const char *path, const df_mech *mech, int32_t device, df_dnn **out);
void df_dnn_free(df_dnn *dnn);
df_status df_dnn_info(const df_dnn *dnn, int32_t *n_layers, int32_t *dims /* [n_layers+1] */, double *lambda,
                      double *dt_train);

/* Bytes of device workspace df_dnn_step needs for n_cells. */
df_status df_dnn_workspace_size(const df_dnn *dnn, int64_t n_cells, size_t *bytes);

/*
 * DNN chemistry step (DNNInferencer::inference): (1) Box-Cox transform and
 * normalisation of (T, p, Y) with the training-range test, (2) the MLP in
 * BF16 with FP32 accumulation, (3) inverse transform, optional
 * renormalisation of Y, T from enthalpy conservation at fixed p, and rr.
 * Cells outside the training range are advanced by df_chem_step instead
 * (fallback_opts) and flagged DF_CELL_DNN_FALLBACK.  Arguments as in
 * df_chem_step; `workspace` is caller-owned device memory of at least
 * df_dnn_workspace_size bytes, 256-byte aligned.
 * Errors: DF_E_INVALID, DF_E_UNSUPPORTED (dt != the network's dt_train,
 * relative difference above 1e-12, or a species count without compiled
 * pre- and post-processing kernels: 2, 4, 9 and 53 are compiled), DF_E_HIP.
 */
df_status df_dnn_step(const df_dnn *dnn, const df_mech *mech, int64_t n_cells, int64_t ld, double dt,
                      const double *p, double *T, double *Y, double *rr, int32_t *cell_status, void *workspace,
                      size_t workspace_bytes, const df_dnn_opts *opts, const df_chem_opts *fallback_opts,
                      void *hip_stream);

/*
 * ---- Training the DNN on the device ----
 * The network of the DNN form (Sec. "Chemistry Integration") fitted to pairs the integrator
 * produces, with hand-written backward kernels: mean squared error of the z-scored outputs,
 * L = 1/(B O) sum_b sum_o (u_bo - t_bo)^2, bf16 forward and backward products on the matrix
 * cores with fp32 accumulation, fp32 gradients, Adam on fp32 master weights.  Training
 * rewrites the DNN handle's weights, so df_dnn_step runs the trained network.
 */
typedef struct {
    float lr, beta1, beta2, eps; /* defaults 1e-4, 0.9, 0.999, 1e-8 */
} df_adam_opts;
void df_adam_default_opts(df_adam_opts *opts);

/* Training state for batches of up to max_batch rows: fp32 master copies of the weights, Adam
   moments, transposed bf16 weights and activation buffers (device memory owned by the trainer;
   about 2.2 kB per batch row plus 50 bytes per parameter for the 11-1600-800-400-9 network).
   Errors: DF_E_INVALID, DF_E_UNSUPPORTED (output width other than 9), DF_E_HIP. */
df_status df_dnn_trainer_create(df_dnn *dnn, int64_t max_batch, df_trainer **out);
void df_dnn_trainer_free(df_trainer *trainer);

/*
 * Training rows from states before and after one integrator step of the network's dt_train:
 *   p, T [n], Y0 [K*ld]   in   state before the step;  Y1 [K*ld] in  mass fractions after it
 *   x [n][K+2] fp32       out  z-scored (T, p, Box-Cox(Y0)), the network's input
 *   target [n][K] fp32    out  z-scored Box-Cox(Y1) - Box-Cox(Y0), the network's output
 *   valid [n] int32       out  1 inside the network's training box, else 0 (nullable)
 * Errors: DF_E_INVALID, DF_E_UNSUPPORTED (species count other than 9), DF_E_HIP.
 */
df_status df_dnn_make_batch(const df_dnn *dnn, int64_t n_cells, int64_t ld, const double *p, const double *T,
                            const double *Y0, const double *Y1, float *x, float *target, int32_t *valid,
                            void *hip_stream);

/*
 * One training step on `batch` rows (1 <= batch <= max_batch): forward, loss, gradients, and,
 * when update != 0, one Adam step (opts nullable = defaults).  x [batch][K+2], target
 * [batch][K] fp32 device arrays as df_dnn_make_batch writes them; loss (nullable) receives L,
 * the loss before the update, as one fp32 on the device.  Asynchronous on hip_stream; the
 * trainer's buffers are reused by the next call on it.
 * Errors: DF_E_INVALID (null trainer/array, batch out of range, bad Adam options), DF_E_HIP.
 */
df_status df_dnn_train_step(df_trainer *trainer, int64_t batch, const float *x, const float *target,
                            const df_adam_opts *opts, int32_t update, float *loss, void *hip_stream);

/* Copy a trainer array of layer `layer` (0 .. n_layers-1) into dst (device, fp32):
   what = 0 master weights [n_out][n_in], 1 master biases [n_out], 2 weight gradients of the
   last step [n_out][n_in], 3 bias gradients [n_out].  Errors: DF_E_INVALID, DF_E_HIP. */
df_status df_dnn_trainer_get(const df_trainer *trainer, int32_t layer, int32_t what, float *dst, void *hip_stream);

/* Set the weights (what = 0, src [n_out][n_in]) or biases (what = 1, src [n_out]) of layer
   `layer` from fp32 device memory: the trainer's master copy and the handle's weights (bf16)
   both take them; the Adam moments are left as they are.  Errors: DF_E_INVALID, DF_E_HIP. */
df_status df_dnn_trainer_set(df_trainer *trainer, int32_t layer, int32_t what, const float *src, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* DF_H */
