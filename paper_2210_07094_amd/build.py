"""Build libdf.so (HIP for gfx950) in-tree.

    python -m paper_2210_07094_amd.build

Each source is compiled to an object in parallel, then linked into
``paper_2210_07094_amd/libdf.so``.  Always rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdf.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         # packed FP32 instructions stay off in all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]

SOURCES = ["df_mech.cpp", "df_chem.hip", "df_chem_cv.hip", "df_chem_wave.hip", "df_chem_coop.hip", "df_dnn.hip", "df_mlp.hip", "df_adjoint.hip", "df_train.hip", "df_rollout.hip", "df_stats.hip"]

# per-source additions: the constant-volume kernel is built with the machine instruction
# scheduler off and the one-wavefront-per-cell kernel with the scheduler's max-memory-clause
# strategy.  -O2 and -O3 builds with the default scheduling gave wrong results on gfx950, while
# these builds, -O1 and the CPU build of the same sources under sanitizers (tests/test_cpu_emu.py)
# agree with the oracle; the optimised IR of both files carries no undefined value into the
# arithmetic, so the difference arises in code generation.  Their parity tests check these builds.
EXTRA = {"df_chem_cv.hip": ["-mllvm", "-enable-misched=0"],
         "df_chem_wave.hip": ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"]}


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
