// Internal declarations of the chemistry-step library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "df.h"

namespace df {

constexpr double kR = 8.31446261815324;  // J/mol/K
constexpr double kPref = 101325.0;       // Pa, standard state of the NASA-7 fits
constexpr int kSlots = 3;                // molecules per reaction side
constexpr int kSpTab = 20;               // doubles per species row
constexpr int kRxInt = 8;                // ints per reaction row
constexpr int kRxDbl = 12;               // doubles per reaction row

// Species row (doubles): W, 1/W, a1..a7, a2/2, a3/3, a4/4, a5/5, a3/2, a4/3, a5/4, 2a3, 3a4, 4a5, pad.
// Reaction row (ints): type, r0, r1, r2, p0, p1, p2, dnu.  Slots hold 1 + species index, 0 = empty;
//   the kernels keep index 0 of every per-species array as a neutral element (concentration 1,
//   enthalpy 0, dummy accumulator) so that empty slots need no branch.
// Reaction row (doubles): ln A, b, Ta, ln A0, b0, Ta0, alpha, 1/T***, 1/T*, T**, n_reac, n_prod.
//
// Tables of the cooperative kernel (16 lanes per cell; stored reaction j is evaluated by lane
// j % 16 as its slot j / 16).  Reaction rows are padded to MP = 16 * RPL with inert rows whose
// rate of progress is exactly zero.
constexpr int kCoopLanes = 16;
constexpr int kCoopList = 16;  // entries of the per-lane production-rate list
constexpr int kCoopEnt = 6;    // Jacobian entries per reaction (distinct species)
// coop reaction row (doubles):
//   [0..2]   ln k_f (ln k_inf for falloff rows) over (1, ln T, 1/T)
//   [3..9]   ln k_f - ln K_c (concentration units) over (1, ln T, 1/T, T, T^2, T^3, T^4)
//   [10..15] reaction enthalpy sum_k nu_k H_k/(R T) over (1, T, T^2, T^3, T^4, 1/T)
//   [16..18] ln(k_0 / k_inf) over (1, ln T, 1/T)
//   [19] alpha, [20] -1/T***, [21] -1/T*, [22] -T**, [23] n_reac, [24] n_prod
constexpr int kCrDbl = 25;
// coop reaction row (ints): type, r0, r1, r2, p0, p1, p2, then kCoopEnt pairs (column, mask):
//   column = species index of a distinct species of the reaction (K + 3 = scratch column for
//   unused entries); mask bits 0..2 = reactant slots holding it, bits 3..5 = product slots.
constexpr int kCiInt = 7 + 2 * kCoopEnt;
struct MechDev {
    int K, M;
    const double *sp;   // [K][kSpTab]
    const int *rx;      // [M][kRxInt]
    const double *rk;   // [M][kRxDbl]
    const double *eff;  // [M][K]
    const int *nu;      // [M][K] net stoichiometric coefficients nu'' - nu'
    int RPL;            // reaction slots per lane of the cooperative kernel (MP = 16 * RPL rows)
    int lmax;           // longest per-species reaction list
    const double *cr;    // [MP][kCrDbl]
    const int *ci;       // [MP][kCiInt]
    const double *ceff;  // [MP][K + 4] third-body efficiencies (zero beyond K)
    const double *ceffw; // [MP][K] efficiencies divided by W_k
    const int *cli;      // [16][kCoopList] per-lane list: index into the per-cell rate array
    const double *clc;   // [16][kCoopList] per-lane list: coefficient
    const int *src;      // [M] mechanism-file index of stored reaction j
    // column-major copies for the one-wave-per-cell kernel (field f of stored reaction j at f M + j)
    const double *wcr;   // [kCrDbl][M]
    const int *wci;      // [7][M] type, slots
    const double *weff;  // [K][M] third-body efficiencies (zero for plain rows)
    // its Jacobian's sparse entries: target t (LDS offset wtk[t] = (1 + k)(K + 2) + 1 + l) is the
    // sum over its entries of nu D[idx], D[r M + j] the derivative of q_j with respect to the
    // concentration in the slot of D row r; targets go in rounds of 64, one per lane, and entry e of the lane
    // of target 64 r + l is well[wrb[r] + 64 e + l], e < wrc[r] (padding has nu = 0).  Entries
    // are packed idx | (nu + 8) << 20.
    int wnt, wnr;
    // slots in use: reactant slots 0..wsr-1 and product slots 3..3+wsp-1 (the slot derivatives
    // D hold wsr + wsp rows: slot s < 3 in row s, slot 3 + s in row wsr + s)
    int wsr, wsp;
    const int *wtk;      // [wnt]
    const int *well;
    const int *wrb;      // [wnr]
    const int *wrc;      // [wnr]
    // the per-species reaction lists packed (j, nu), species k at wlo[k] <= e < wlo[k + 1]
    const int *wlo;     // [K + 1]
    const int *wlp;
    // the dense third-body terms: row k gains sum over wdo[k] <= e < wdo[k + 1] of
    // nu G_j eff_jl, (j, nu) packed in wdp[e]
    const int *wdo;      // [K + 1]
    const int *wdp;
};

struct HostMech {
    std::string name;
    long seed = 0;
    int E = 0, K = 0, M = 0;
    std::vector<double> W;        // kg/mol
    std::vector<int> comp;        // [K][E]
    std::vector<double> nasa;     // [K][7]
    std::vector<int> type;        // [M]
    std::vector<int> nu_r, nu_p;  // [M][K]
    std::vector<double> arr;      // [M][3]
    std::vector<double> eff;      // [M][K]
    std::vector<double> low;      // [M][3]
    std::vector<double> troe;     // [M][4]
};

// error reporting (thread-local message)
df_status fail(df_status code, const std::string &msg);
void clear_error();

// parse a "dfmech 1" file; returns DF_OK or an error code (message set)
df_status parse_mech_file(const char *path, HostMech &out);

struct Opts {
    double rtol, atol_T, atol_Y, h_min;
    int max_steps;
};

// Arguments of one chemistry-step launch (device pointers, layouts as in df_chem_step).
struct StepArgs {
    int64_t n, ld;
    double dt;          // step length of every cell, unless dts is given
    const double *dts;  // [n] step length per cell, or nullptr
    const double *p;
    double *T, *Y, *h_io, *rr;
    int32_t *status, *nsteps;
    Opts o;
    int32_t status_ok;  // status written for cells that succeed (DF_CELL_OK or DF_CELL_DNN_FALLBACK)
    // tape of the accepted sub-steps for the adjoint (16-lane launch only; nullptr = none),
    // layout in Tape below
    double *tape = nullptr;
    int32_t tape_cap = 0;
};

// Tape of a taped step: for each accepted sub-step s < cap of each of n cells, its start
// state y (N = K + 1), its length h, the inverse of its iteration matrix W = I/(g h) - J(y)
// (entry (r, c) at r N + c) and its six stage vectors (entry (i, k) at i N + k); then the
// sub-step count of each cell (int32, -1 for a cell without a tape).  Every array is
// cell-minor (stride n), so the lanes of a wave read and write it coalesced.
struct Tape {
    int N;
    int64_t n, cap;
    __host__ __device__ Tape(int K, int64_t n_, int64_t cap_) : N(K + 1), n(n_), cap(cap_) {}
    __host__ __device__ int64_t y(int64_t s, int k) const { return (s * N + k) * n; }
    __host__ __device__ int64_t h(int64_t s) const { return cap * N * n + s * n; }
    __host__ __device__ int64_t w(int64_t s, int e) const { return cap * (N + 1) * n + (s * N * N + e) * n; }
    __host__ __device__ int64_t u(int64_t s, int e) const {
        return cap * (N + 1 + N * N) * n + (s * 6 * N + e) * n;
    }
    __host__ __device__ int64_t doubles() const { return cap * (7 * N + 1 + N * N) * n; }
    __host__ __device__ int32_t *count(double *t) const { return reinterpret_cast<int32_t *>(t + doubles()); }
    __host__ __device__ const int32_t *count(const double *t) const {
        return reinterpret_cast<const int32_t *>(t + doubles());
    }
    size_t bytes() const { return size_t(8) * size_t(doubles()) + size_t(4) * size_t(n); }
};

inline size_t tape_bytes(int K, int64_t n, int32_t cap) { return Tape(K, n, cap).bytes(); }

// Where the lanes (or 16-lane groups) of a launch get their cells.
//   static: slot s (global lane or group index) takes cell cidx[s] (or s), for s < *dcount (or n);
//   queue:  ctr != nullptr; cells are taken from order[] (most expensive first).  Blocks
//           [0, head_blocks) run 16-lane groups that claim from the front.  The other blocks
//           first run one cell per lane on cells claimed from the back, at most *tail_max of
//           them (the cells of the cold buckets), then join the front claims as 16-lane
//           groups.  The low 32 bits of *ctr count front claims, the high 32 bits back
//           claims (queue_claim tells the valid ones), so every cell is taken exactly once.
struct CellQueue {
    const int32_t *cidx;
    const int32_t *dcount;
    const int32_t *order;
    unsigned long long *ctr;
    const int32_t *tail_max;
    int32_t head_blocks;
};

// species counts with a compiled one-cell-per-lane kernel
#define DF_CHEM_SPECIES_LIST(X) X(2) X(4) X(9)

inline Opts kernel_opts(const df_chem_opts &o) { return Opts{o.rtol, o.atol_T, o.atol_Y, o.h_min, o.max_steps}; }

// integrator launch with the static schedule (df_chem.hip); arrays already validated.
// cidx/dcount (both nullable): slot s < *dcount works on cell cidx[s] (compacted subset).
df_status launch_chem_step(const MechDev &m, const StepArgs &a, int mapping, const int32_t *cidx,
                           const int32_t *dcount, hipStream_t stream);

df_status validate_chem_opts(const df_chem_opts &o);

// one-wave-per-cell integrator (df_chem_wave.hip): mechanisms of up to 63 species with a
// compiled instantiation; cidx/dcount as launch_chem_step
bool chem_wave_supported(const MechDev &m);
df_status launch_chem_wave(const MechDev &m, const StepArgs &a, const int32_t *cidx, const int32_t *dcount,
                           hipStream_t stream);

// cooperative integrator (df_chem_coop.hip): 16 lanes per cell (halves = 1), or 32 (halves = 2, where
// the reaction slots divide between two halves and no tape is written), for the species counts
// and table sizes it is instantiated for
bool chem_coop_supported(const MechDev &m);
df_status launch_chem_coop(const MechDev &m, const StepArgs &a, const CellQueue &q, hipStream_t stream,
                           int halves = 1);
// persistent work-queue launch mixing the 16-lane and the one-cell-per-lane bodies
// (df_chem_coop.hip): blocks resident at once on the current device, and the launch
int32_t chem_queue_capacity(const MechDev &m);
df_status launch_chem_queue(const MechDev &m, const StepArgs &a, const CellQueue &q, int32_t blocks,
                            hipStream_t stream);

}  // namespace df

struct df_mech {
    int device;
    df::HostMech host;
    void *dev_blob;   // one device allocation holding all tables
    df::MechDev dev;  // pointers into dev_blob
};

namespace df {

// ---- DNN form ----
typedef unsigned short bf16_t;  // raw bfloat16 bits

constexpr int kGemmBM = 128;  // cells per GEMM tile
constexpr int kGemmBN = 160;  // outputs per GEMM tile
constexpr int kGemmBK = 32;   // reduction depth per stage
constexpr int kInPad = 32;    // padded width of the network input

struct DnnLayer {
    int n_in, n_out;    // true widths
    int k_pad, n_pad;   // padded widths on the device (k_pad = previous n_pad, or kInPad)
    bf16_t *W;          // [n_pad][k_pad] device, zero padded
    float *b;           // [n_pad] device, zero padded
};

struct DnnDevParams {   // kernel argument for the pre/post kernels
    int K, n_in;
    double lambda, inv_lambda;
    const double *mu_in, *sig_in, *mu_out, *sig_out, *lo, *hi;  // device arrays
};

// C[M][N] = act(A[M][K] B[N][K]^T + bias) in bf16 with fp32 accumulation; M % kGemmBM == 0,
// N % kGemmBN == 0, K % kGemmBK == 0, row strides in elements.
df_status launch_gemm_bf16(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C, int ldc,
                           int64_t M, int N, int K, bool gelu, hipStream_t stream);
// the same GEMM with the training epilogues: gelu_save also stores the pre-activation
// (A B^T + bias) to P with C's layout; gelu_grad writes (A B^T) * GELU'(P) (no bias)
enum class GemmEpi { gelu, linear, gelu_save, gelu_grad };
df_status launch_gemm_bf16_epi(const bf16_t *A, int lda, const bf16_t *B, int ldb, const float *bias, bf16_t *C,
                               int ldc, int64_t M, int N, int K, GemmEpi epi, bf16_t *P, hipStream_t stream);

}  // namespace df

struct df_dnn {
    int device;
    int K;
    int L;
    std::vector<int> dims;
    double lambda, dt_train;
    std::vector<df::DnnLayer> layers;  // hidden layers (MFMA path) and the output layer
    void *dev_blob;                    // all device memory of the handle
    df::DnnDevParams prm;
};
