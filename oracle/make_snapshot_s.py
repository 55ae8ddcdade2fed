"""Snapshot S of the 256 x 256 hot-kernel field: the field advanced by the oracle integrator.

The benchmark field as generated (snapshot 0) holds premixed H2/air with no radicals: its hot
kernels have not ignited, so most of a chemistry step happens nowhere.  Snapshot S is the same
field after repeated chemistry steps of the oracle integrator (each cell carrying
its sub-step hint, as a flow solver's chemistry calls would; advanced in calls of 10 us, since
the synthetic mechanism takes milliseconds to ignite at 1800 K) until the hottest cell has risen by
more than 500 K over the hottest initial cell: the kernels are then igniting, with radicals,
in-flame temperatures and the steep fronts between them, the states the chemistry step sees
inside the paper's jet flame (Sec. "Two-Dimensional Jet Flame").  There is no transport: each
cell evolves as a closed reactor, which is what the chemistry step of an operator-split solver
sees within one flow step.

This script calls only the oracle; the stored file is an input of the benchmark and of the GPU
parity tests (test infrastructure writes it, the GPU path never does).

    python -m oracle.make_snapshot_s      # writes synth/data/h2_field_snapshot_s.npz
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import fields  # noqa: E402

MECH = os.path.join(ROOT, "synth", "data", "h2_synth_9sp_24r.mech")
OUT = os.path.join(ROOT, "synth", "data", "h2_field_snapshot_s.npz")
DT = 1e-5     # length of one advancing call
RISE = 500.0
MAX_STEPS = 2000


def make(out=OUT, verbose=True):
    mech = synth.read_mech(MECH)
    om = oracle.Mech(MECH)
    f = fields.hot_kernel_field_2d(mech)
    T, p, Y = f["T"].copy(), f["p"].copy(), f["Y"].copy()
    h = np.zeros_like(T)
    T0max = T.max()
    t0 = time.time()
    for step in range(1, MAX_STEPS + 1):
        r = om.chem_step(T, p, Y, DT, h_inout=h)
        assert np.all(r["status"] == 0), "an oracle step failed"
        T, Y, h = r["T"], r["Y"], r["h"]
        if verbose and step % 10 == 0:
            print(f"step {step}: max T {T.max():.1f} K ({time.time() - t0:.0f} s)", flush=True)
        if T.max() - T0max > RISE:
            break
    else:
        raise RuntimeError("the field did not rise by 500 K")
    np.savez_compressed(out, T=T, p=p, Y=Y, h=h, steps=np.int64(step), dt=np.float64(DT),
                        shape=np.array(f["shape"], dtype=np.int64))
    if verbose:
        print(f"snapshot S after {step} steps of {DT} s: max T {T.max():.1f} K (initially {T0max:.1f} K), "
              f"cells above 1500 K: {(T > 1500).sum()}; written to {out}")
    return step


if __name__ == "__main__":
    make()
