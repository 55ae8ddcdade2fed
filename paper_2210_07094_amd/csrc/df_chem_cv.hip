// Constant-volume chemistry step on gfx950: one cell per lane, FP64 throughout.
//
// The closed homogeneous reactor of the paper's 0-D ignition tests at fixed density:
//   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k U_k wdot_k / (rho cv),
// with U_k = H_k - R T the molar internal energy and cv = cp - R / Wbar; the pressure follows
// the state (p = rho R T / Wbar).  The per-lane RODAS4 solver is the constant-pressure one with
// its constant-volume thermodynamics (Cell<K, true>); species counts without a per-lane kernel
// go to the one-wavefront-per-cell kernel's constant-volume instantiation (df_chem_wave.hip).
//
// This file is compiled on its own, with the machine instruction scheduler off: optimised
// builds of this instantiation with the scheduler on produced wrong sub-steps on gfx950
// (every attempt after the first rejected, the step length driven to 1e-17 s) while the same
// source built without optimisation, built with FP contraction off, or run on the CPU under
// sanitizers (tests/test_cpu_emu.py) gave the oracle's sub-step sequence; the constant-pressure
// instantiation of the same solver is correct with the scheduler on, and the optimised IR of
// this file carries no undefined value into the arithmetic.  The parity tests of the
// constant-volume step check this build.
#include <cmath>

#include "df_internal.h"
#include "df_kinetics.h"
#include "df_lane.h"

namespace df {
// the constant-volume reactor on one wavefront per cell (df_chem_wave.hip), for species counts
// without a one-cell-per-lane kernel; a.p holds the density
bool chem_wave_supported(const MechDev &m);
df_status launch_chem_wave_cv(const MechDev &m, const StepArgs &a, hipStream_t stream);

namespace {

template <int K>
__global__ __launch_bounds__(kWave) void chem_step_cv_kernel(MechDev m, StepArgs a) {
    using C = Cell<K, true>;
    __shared__ double lds[C::kRows * kWave];
    double *sh = lds + threadIdx.x;
    C::init_lds(sh);
    const int64_t slot = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (slot >= a.n) return;
    LaneTask<K> c;
    bool have = lane_load<K>(a, slot, c);
    while (have) have = !lane_attempt<K, true>(m, a, sh, c);
}

template <int K>
df_status launch_cv(const MechDev &m, const StepArgs &a, hipStream_t stream) {
    const int64_t blocks = (a.n + kWave - 1) / kWave;
    hipLaunchKernelGGL(chem_step_cv_kernel<K>, dim3(unsigned(blocks)), dim3(kWave), 0, stream, m, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("df_chem_step_const_volume launch: ") + hipGetErrorString(e));
    return DF_OK;
}

}  // namespace
}  // namespace df

extern "C" df_status df_chem_step_const_volume(const df_mech *mech, int64_t n_cells, int64_t ld, double dt,
                                               const double *rho, double *T, double *Y, double *h_inout,
                                               int32_t *cell_status, int32_t *n_steps, const df_chem_opts *opts,
                                               void *hip_stream) {
    using namespace df;
    clear_error();
    const char *who = "df_chem_step_const_volume";
    if (!mech) return fail(DF_E_INVALID, std::string(who) + ": null mechanism handle");
    if (n_cells < 0 || ld < n_cells) return fail(DF_E_INVALID, std::string(who) + ": need 0 <= n_cells <= ld");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DF_E_INVALID, std::string(who) + ": dt must be finite and > 0");
    if (n_cells > 0 && (!rho || !T || !Y)) return fail(DF_E_INVALID, std::string(who) + ": null rho, T or Y");
    if (n_cells > int64_t(kWave) * 0x7fffffff) return fail(DF_E_UNSUPPORTED, std::string(who) + ": too many cells");
    df_chem_opts o;
    df_chem_default_opts(&o);
    if (opts) o = *opts;
    df_status st = validate_chem_opts(o);
    if (st != DF_OK) return st;
    if (n_cells == 0) return DF_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": hipGetDevice failed");
    if (prev != mech->device && hipSetDevice(mech->device) != hipSuccess)
        return fail(DF_E_HIP, std::string(who) + ": cannot select the mechanism's device");
    // the density goes where the constant-pressure step takes the pressure
    const StepArgs a{n_cells, ld, dt, nullptr, rho, T, Y, h_inout, nullptr, cell_status, n_steps, kernel_opts(o),
                     DF_CELL_OK};
    auto s = static_cast<hipStream_t>(hip_stream);
    switch (mech->dev.K) {
#define DF_CASE(k)                             \
    case k:                                    \
        st = launch_cv<k>(mech->dev, a, s);    \
        break;
        DF_CHEM_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            if (chem_wave_supported(mech->dev))
                st = launch_chem_wave_cv(mech->dev, a, s);
            else
                st = fail(DF_E_UNSUPPORTED,
                          std::string(who) + ": no compiled kernel for " + std::to_string(mech->dev.K) + " species");
    }
    if (prev != mech->device) (void)hipSetDevice(prev);
    return st;
}
