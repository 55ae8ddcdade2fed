"""The integrator kernel sources run on the CPU under sanitizers, against the oracle.

The one-wavefront-per-cell kernel (df_chem_wave.hip) and the constant-volume step
(df_chem_cv.hip, one cell per lane at 9 species and the wavefront kernel at 53) are compiled as
plain C++ with a host stand-in for the HIP runtime (tests/cpu_emu/hip/hip_runtime.h: the threads
of a block are fibers, every cross-lane operation and barrier a meeting of all of them), three
times:
  * with AddressSanitizer and UndefinedBehaviorSanitizer (g++, -fno-sanitize-recover: any finding
    ends the run with an error), and
  * twice with clang's -ftrivial-auto-var-init, once filling every automatic variable with a
    pattern and once with zeros: a variable read before it is written makes the two differ.
Each run must end cleanly; the two initialisations must give the same bits; and the results must
match the oracle to the integrator's parity bar (1e-8 relative in T and in Y > 1e-10) with the
oracle's accepted and rejected sub-step counts, so that the sub-step sequences are the same.

The only change to the kernel source is textual: the dynamic LDS declaration of the wavefront
kernel becomes a pointer to the emulated block's dynamic area.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import fields

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2210_07094_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "cpu_emu")
H2 = os.path.join(ROOT, "synth", "data", "h2_synth_9sp_24r.mech")
HC = os.path.join(ROOT, "synth", "data", "hc_synth_53sp_325r.mech")
CLANG = "/opt/rocm/llvm/bin/clang++"

BUILDS = {
    "sanitized": ["g++", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-omit-frame-pointer"],
    "init_pattern": [CLANG, "-O2", "-ftrivial-auto-var-init=pattern"],
    "init_zero": [CLANG, "-O2", "-ftrivial-auto-var-init=zero"],
}


@pytest.fixture(scope="module")
def exes(tmp_path_factory):
    d = tmp_path_factory.mktemp("emu")
    src = open(os.path.join(CSRC, "df_chem_wave.hip")).read()
    decl = "extern __shared__ double lds[];"
    assert src.count(decl) == 1
    wave = d / "df_chem_wave.cpp"
    wave.write_text(src.replace(decl, "double *lds = ::emu::dyn_lds<double>();"))
    common = ["-std=c++17", "-Wno-unknown-pragmas", "-I", EMU, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-x", "c++", os.path.join(CSRC, "df_mech.cpp"), "-x", "c++", os.path.join(CSRC, "df_chem_cv.hip"),
              "-x", "c++", str(wave), "-x", "c++", os.path.join(EMU, "emu_run.cpp")]
    procs, out = {}, {}
    for name, flags in BUILDS.items():
        if flags[0] == CLANG and not os.path.exists(CLANG):
            pytest.skip("clang++ of the ROCm toolchain not found")
        out[name] = str(d / f"emu_{name}")
        procs[name] = subprocess.Popen([*flags, *common, "-o", out[name]], stdout=subprocess.PIPE,
                                       stderr=subprocess.STDOUT, text=True)
    for name, p in procs.items():
        log, _ = p.communicate(timeout=600)
        assert p.returncode == 0, f"{name} build failed:\n{log[-4000:]}"
    return out


def _run_all(exes, tmp, mech_path, kernel, K, p, T, Y, dt):
    """Run every build on the same input at once; {build: (arrays, raw bytes)}."""
    n = T.size
    fin = tmp / f"in_{kernel}.bin"
    with open(fin, "wb") as f:
        f.write(np.int64(n).tobytes())
        f.write(np.float64(dt).tobytes())
        for a in (p, T, Y):
            f.write(np.ascontiguousarray(a, np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    procs = {}
    for name, exe in exes.items():
        fout = tmp / f"out_{kernel}_{name}.bin"
        procs[name] = (subprocess.Popen([exe, mech_path, kernel, str(fin), str(fout)], stdout=subprocess.PIPE,
                                        stderr=subprocess.PIPE, text=True, env=env), fout)
    res = {}
    for name, (pr, fout) in procs.items():
        _, err = pr.communicate(timeout=600)
        assert pr.returncode == 0, f"{name} {kernel}: exit {pr.returncode}\n{err[-6000:]}"
        b = open(fout, "rb").read()
        res[name] = ({"T": np.frombuffer(b, np.float64, n, 0),
                      "Y": np.frombuffer(b, np.float64, K * n, 8 * n).reshape(K, n),
                      "status": np.frombuffer(b, np.int32, n, 8 * n * (K + 1)),
                      "n_steps": np.frombuffer(b, np.int32, 2 * n, 8 * n * (K + 1) + 4 * n)}, b)
    return res


def _parity(g, o):
    assert np.all(g["status"] == 0) and np.all(o["status"] == 0)
    n = g["T"].size
    np.testing.assert_array_equal(g["n_steps"][:n], o["n_acc"])
    np.testing.assert_array_equal(g["n_steps"][n:], o["n_rej"])
    relT = np.abs(g["T"] - o["T"]) / o["T"]
    m = o["Y"] > 1e-10
    relY = np.where(m, np.abs(g["Y"] - o["Y"]) / np.where(m, o["Y"], 1.0), 0.0)
    assert max(relT.max(), relY.max()) <= 1e-8


def _cheapest_hc_cells(k, dt):
    mech = synth.read_mech(HC)
    om = oracle.Mech(HC)
    f = fields.hydrocarbon_field(mech, n=256, seed=11)
    o = om.chem_step(f["T"], f["p"], f["Y"], dt)
    idx = np.sort(np.argsort(o["n_acc"] + o["n_rej"], kind="stable")[:k])
    return mech, om, {"T": f["T"][idx].copy(), "p": f["p"][idx].copy(), "Y": np.ascontiguousarray(f["Y"][:, idx])}


CASES = ["wave53", "wave9", "cv9", "cv53"]


@pytest.mark.parametrize("case", CASES)
def test_kernels_on_cpu_under_sanitizers(exes, tmp_path, case):
    if case == "wave53":
        # the two 53-species cells with the fewest sub-steps at 10 ns
        mech, om, f = _cheapest_hc_cells(2, 1e-8)
        dt, kernel, path, p = 1e-8, "wave", HC, f["p"]
        o = om.chem_step(f["T"], f["p"], f["Y"], dt)
    elif case == "wave9":
        mech, om = synth.read_mech(H2), oracle.Mech(H2)
        f = fields.ignition_cells(mech, n=2, seed=5)
        dt, kernel, path, p = 2e-8, "wave", H2, f["p"]
        o = om.chem_step(f["T"], f["p"], f["Y"], dt)
    elif case == "cv9":
        mech, om = synth.read_mech(H2), oracle.Mech(H2)
        f = fields.ignition_cells(mech, n=70, seed=6)
        p = np.array([om.mixture(f["T"][i], f["p"][i], f["Y"][:, i])[1] for i in range(70)])
        dt, kernel, path = 1e-6, "cv", H2
        o = om.chem_step_v(f["T"], p, f["Y"], dt)
    else:
        mech, om, f = _cheapest_hc_cells(1, 1e-8)
        p = np.array([om.mixture(f["T"][i], f["p"][i], f["Y"][:, i])[1] for i in range(f["T"].size)])
        dt, kernel, path = 1e-8, "cv", HC
        o = om.chem_step_v(f["T"], p, f["Y"], dt)
    K = mech.n_species
    print(f"case {case}: {f['T'].size} cells, oracle sub-steps {o['n_acc'] + o['n_rej']}", flush=True)
    res = _run_all(exes, tmp_path, path, kernel, K, p, f["T"], f["Y"], dt)
    assert res["init_pattern"][1] == res["init_zero"][1], "results depend on uninitialised automatic variables"
    for name, (g, _) in res.items():
        _parity(g, o)
