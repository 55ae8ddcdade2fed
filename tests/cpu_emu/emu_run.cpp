// CPU run of the integrator kernels through the host stand-in for the HIP runtime
// (hip/hip_runtime.h beside this file), for the sanitizer test.  Test infrastructure.
//
//   emu_run <mechanism file> <kernel> <input> <output>
//     kernel: "wave"  the one-wavefront-per-cell kernel, constant pressure
//             "cv"    the constant-volume step (one cell per lane where compiled, else a wavefront)
//     input:  int64 n; double dt; double p[n] (the density for "cv"), T[n], Y[K][n]
//     output: double T[n], Y[K][n]; int32 status[n], n_steps[2n]
#include <cstdio>
#include <vector>

#include "df_internal.h"

int main(int argc, char **argv) {
    if (argc != 5) {
        std::fprintf(stderr, "usage: emu_run <mech> <wave|cv> <input> <output>\n");
        return 2;
    }
    df_mech *m = nullptr;
    if (df_mech_load(argv[1], 0, &m) != DF_OK) {
        std::fprintf(stderr, "df_mech_load: %s\n", df_last_error());
        return 1;
    }
    const int K = m->host.K;
    FILE *f = std::fopen(argv[3], "rb");
    if (!f) return 1;
    int64_t n = 0;
    double dt = 0.0;
    bool ok = std::fread(&n, 8, 1, f) == 1 && std::fread(&dt, 8, 1, f) == 1 && n > 0;
    std::vector<double> p(n), T(n), Y(size_t(K) * n);
    ok = ok && std::fread(p.data(), 8, n, f) == size_t(n) && std::fread(T.data(), 8, n, f) == size_t(n) &&
         std::fread(Y.data(), 8, Y.size(), f) == Y.size();
    std::fclose(f);
    if (!ok) {
        std::fprintf(stderr, "bad input file\n");
        return 1;
    }
    std::vector<int32_t> st(n, -7), ns(2 * n, -7);
    df_chem_opts o;
    df_chem_default_opts(&o);
    df_status r;
    const std::string kernel(argv[2]);
    if (kernel == "wave") {
        const df::StepArgs a{n, n, dt, nullptr, p.data(), T.data(), Y.data(), nullptr, nullptr, st.data(),
                             ns.data(), df::kernel_opts(o), DF_CELL_OK};
        r = df::launch_chem_wave(m->dev, a, nullptr, nullptr, nullptr);
    } else if (kernel == "cv") {
        r = df_chem_step_const_volume(m, n, n, dt, p.data(), T.data(), Y.data(), nullptr, st.data(), ns.data(), &o,
                                      nullptr);
    } else {
        std::fprintf(stderr, "unknown kernel %s\n", argv[2]);
        return 2;
    }
    if (r != DF_OK) {
        std::fprintf(stderr, "step: %s\n", df_last_error());
        return 1;
    }
    f = std::fopen(argv[4], "wb");
    if (!f) return 1;
    std::fwrite(T.data(), 8, n, f);
    std::fwrite(Y.data(), 8, Y.size(), f);
    std::fwrite(st.data(), 4, n, f);
    std::fwrite(ns.data(), 4, 2 * n, f);
    std::fclose(f);
    df_mech_free(m);
    return 0;
}
