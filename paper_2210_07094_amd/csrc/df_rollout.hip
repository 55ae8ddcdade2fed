// Multi-step 0-D rollouts: n consecutive chemistry steps of the DNN form or of the integrator
// from the same initial states, with each cell's ignition delay tracked on the device (the
// validation style of the paper's 0-D tests: DNN and integrator ignition curves side by side).
//
// Ignition delay: the time of the largest temperature rate on the sampled trajectory.  With
// r_k = (T_{k+1} - T_k) / dt the mean rate over step k, centred at t_k = (k + 1/2) dt, and k*
// the step of the largest r_k, the delay is the vertex of the parabola through
// (t_{k*-1}, r_{k*-1}), (t_{k*}, r_{k*}), (t_{k*+1}, r_{k*+1}).  A cell whose largest rate falls
// on the first or the last step has no maximum inside the run: NaN.
//
// The integrator rolls out either reactor of the paper's 0-D cases: constant pressure, or constant
// volume (the density fixed, the pressure following the state).  The DNN maps a constant-pressure
// step, so its rollouts are constant-pressure ones.
#include <cmath>

#include "df_internal.h"

extern "C" df_status df_chem_step(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *p,
                                  double *T, double *Y, double *h_inout, double *rr, int32_t *cell_status,
                                  int32_t *n_steps, void *workspace, size_t ws_bytes, const df_chem_opts *opts,
                                  void *hip_stream);
extern "C" df_status df_dnn_step(const df_dnn *dnn, const df_mech *mech, int64_t n, int64_t ld, double dt,
                                 const double *p, double *T, double *Y, double *rr, int32_t *cell_status,
                                 void *workspace, size_t ws_bytes, const df_dnn_opts *opts,
                                 const df_chem_opts *fallback_opts, void *hip_stream);
extern "C" df_status df_chem_step_const_volume(const df_mech *mech, int64_t n_cells, int64_t ld, double dt,
                                               const double *rho, double *T, double *Y, double *h_inout,
                                               int32_t *cell_status, int32_t *n_steps, const df_chem_opts *opts,
                                               void *hip_stream);
extern "C" df_status df_chem_workspace_size(const df_mech *mech, int64_t n_cells, size_t *bytes);
extern "C" df_status df_dnn_workspace_size(const df_dnn *dnn, int64_t n_cells, size_t *bytes);

namespace df {
namespace {

constexpr int kT = 256;

// per cell: initial and previous temperature, largest rate so far, the rates of the steps
// before (rm) and after (rp) it, the last step's rate, the integrator's sub-step hint, the step
// of the largest rate
struct Track {
    double *T0, *Tprev, *best, *rm, *rp, *rlast, *h;
    int32_t *kbest;
};

__global__ __launch_bounds__(kT) void track_init_kernel(int64_t n, const double *__restrict__ T, Track t) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    t.T0[i] = T[i];
    t.Tprev[i] = T[i];
    t.best[i] = -INFINITY;
    t.rm[i] = NAN;
    t.rp[i] = NAN;
    t.rlast[i] = NAN;
    t.h[i] = 0.0;
    t.kbest[i] = -1;
}

// after step k: the rate of step k; a new largest rate keeps the previous step's rate as its
// left neighbour, the step right after the largest rate gives the right neighbour
__global__ __launch_bounds__(kT) void track_step_kernel(int64_t n, int32_t k, double dt, const double *__restrict__ T,
                                                        Track t) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    const double Tn = T[i];
    const double r = (Tn - t.Tprev[i]) / dt;
    if (r > t.best[i]) {
        t.rm[i] = t.rlast[i];
        t.best[i] = r;
        t.kbest[i] = k;
        t.rp[i] = NAN;
    } else if (k == t.kbest[i] + 1) {
        t.rp[i] = r;
    }
    t.rlast[i] = r;
    t.Tprev[i] = Tn;
}

__global__ __launch_bounds__(kT) void track_finish_kernel(int64_t n, int32_t steps, double dt, Track t,
                                                          double *__restrict__ idt) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    const int32_t kb = t.kbest[i];
    if (kb <= 0 || kb + 1 >= steps) {
        idt[i] = NAN;
        return;
    }
    double tk = (kb + 0.5) * dt;
    const double a = t.rm[i], b = t.best[i], c = t.rp[i];
    const double den = a - 2.0 * b + c;
    if (isfinite(a) && isfinite(c) && den < 0.0) tk += 0.5 * (a - c) / den * dt;
    idt[i] = tk;
}

}  // namespace
}  // namespace df

using namespace df;

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

static size_t rollout_track_bytes(int64_t n) { return 7 * al256(size_t(n) * 8) + al256(size_t(n) * 4); }

extern "C" df_status df_rollout_workspace_size(const df_mech *mech, const df_dnn *dnn, int64_t n_cells,
                                               size_t *bytes) {
    clear_error();
    if (!mech || !bytes || n_cells < 0) return fail(DF_E_INVALID, "df_rollout_workspace_size: bad arguments");
    size_t inner = 0;
    const df_status st = dnn ? df_dnn_workspace_size(dnn, n_cells, &inner) : df_chem_workspace_size(mech, n_cells, &inner);
    if (st != DF_OK) return st;
    *bytes = rollout_track_bytes(n_cells) + al256(inner);
    return DF_OK;
}

extern "C" df_status df_rollout(const df_mech *mech, const df_dnn *dnn, int64_t n_cells, int64_t ld, double dt,
                                int32_t n_steps, int32_t reactor, const double *p, double *T, double *Y, double *idt, double *T_traj,
                                void *workspace, size_t ws_bytes, const df_chem_opts *opts, void *hip_stream) {
    clear_error();
    const char *who = "df_rollout";
    if (!mech) return fail(DF_E_INVALID, std::string(who) + ": null mechanism handle");
    if (n_cells < 0 || ld < n_cells || n_steps < 1 || !(dt > 0.0) || !std::isfinite(dt))
        return fail(DF_E_INVALID, std::string(who) + ": need 0 <= n_cells <= ld, n_steps >= 1, dt > 0");
    if (reactor != DF_REACTOR_CONST_P && reactor != DF_REACTOR_CONST_V)
        return fail(DF_E_INVALID, std::string(who) + ": reactor must be DF_REACTOR_CONST_P or DF_REACTOR_CONST_V");
    if (dnn && reactor != DF_REACTOR_CONST_P)
        return fail(DF_E_INVALID, std::string(who) + ": the DNN form is a constant-pressure step");
    if (n_cells > 0 && (!p || !T || !Y || !idt || !workspace))
        return fail(DF_E_INVALID, std::string(who) + ": null p, T, Y, idt or workspace");
    size_t need = 0;
    df_status st = df_rollout_workspace_size(mech, dnn, n_cells, &need);
    if (st != DF_OK) return st;
    if (n_cells > 0 && (ws_bytes < need || reinterpret_cast<uintptr_t>(workspace) % 256 != 0))
        return fail(DF_E_INVALID, std::string(who) + ": workspace smaller than df_rollout_workspace_size or misaligned");
    clear_error();
    if (n_cells == 0) return DF_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": hipGetDevice failed");
    if (prev != mech->device && hipSetDevice(mech->device) != hipSuccess)
        return fail(DF_E_HIP, std::string(who) + ": cannot select the mechanism's device");
    auto s = static_cast<hipStream_t>(hip_stream);
    auto *base = static_cast<unsigned char *>(workspace);
    const size_t a8 = al256(size_t(n_cells) * 8);
    Track t;
    t.T0 = reinterpret_cast<double *>(base);
    t.Tprev = reinterpret_cast<double *>(base + a8);
    t.best = reinterpret_cast<double *>(base + 2 * a8);
    t.rm = reinterpret_cast<double *>(base + 3 * a8);
    t.rp = reinterpret_cast<double *>(base + 4 * a8);
    t.rlast = reinterpret_cast<double *>(base + 5 * a8);
    t.h = reinterpret_cast<double *>(base + 6 * a8);
    t.kbest = reinterpret_cast<int32_t *>(base + 7 * a8);
    void *inner = base + rollout_track_bytes(n_cells);
    const size_t inner_bytes = ws_bytes - rollout_track_bytes(n_cells);
    const dim3 g = dim3(unsigned((n_cells + kT - 1) / kT)), b = dim3(kT);
    hipLaunchKernelGGL(track_init_kernel, g, b, 0, s, n_cells, T, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) st = fail(DF_E_HIP, std::string(who) + ": " + hipGetErrorString(e));
    if (st == DF_OK && T_traj)
        if (hipMemcpyAsync(T_traj, T, size_t(n_cells) * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            st = fail(DF_E_HIP, std::string(who) + ": trajectory copy failed");
    for (int32_t k = 0; k < n_steps && st == DF_OK; ++k) {
        if (dnn)
            st = df_dnn_step(dnn, mech, n_cells, ld, dt, p, T, Y, nullptr, nullptr, inner, inner_bytes, nullptr, opts,
                             hip_stream);
        else if (reactor == DF_REACTOR_CONST_V)
            st = df_chem_step_const_volume(mech, n_cells, ld, dt, p, T, Y, t.h, nullptr, nullptr, opts, hip_stream);
        else
            st = df_chem_step(mech, n_cells, ld, dt, p, T, Y, t.h, nullptr, nullptr, nullptr, inner, inner_bytes, opts,
                              hip_stream);
        if (st != DF_OK) break;
        hipLaunchKernelGGL(track_step_kernel, g, b, 0, s, n_cells, k, dt, T, t);
        e = hipGetLastError();
        if (e != hipSuccess) st = fail(DF_E_HIP, std::string(who) + ": " + hipGetErrorString(e));
        if (st == DF_OK && T_traj &&
            hipMemcpyAsync(T_traj + size_t(k + 1) * size_t(n_cells), T, size_t(n_cells) * 8, hipMemcpyDeviceToDevice,
                           s) != hipSuccess)
            st = fail(DF_E_HIP, std::string(who) + ": trajectory copy failed");
    }
    if (st == DF_OK) {
        hipLaunchKernelGGL(track_finish_kernel, g, b, 0, s, n_cells, n_steps, dt, t, idt);
        e = hipGetLastError();
        if (e != hipSuccess) st = fail(DF_E_HIP, std::string(who) + ": " + hipGetErrorString(e));
    }
    if (prev != mech->device) (void)hipSetDevice(prev);
    return st;
}
