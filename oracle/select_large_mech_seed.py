"""Pick the seed of the synthetic 53-species mechanism (run once; prints the seed).

Test infrastructure: it runs the CPU oracle.  Starting from a base seed it tries seeds
in order and accepts the first mechanism that
  1. has at least 55 one <-> two reactions to draw from (else the generator refuses);
  2. ignites stoichiometric CH4/air at 1 atm from 1500 K (T rise > 400 K) within 0.1 s
     and ends above 1800 K;
  3. integrates 128 cells of the hydrocarbon field over dt = 1e-6 s at rtol 1e-8 with
     every cell OK.

    python oracle/select_large_mech_seed.py [base_seed] [max_tries]
"""
from __future__ import annotations

import os
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import fields  # noqa: E402
from synth.mechgen_large import generate_large_mechanism  # noqa: E402


def ignition(om, mech, T0, t_end=0.1):
    Y = fields.premixed_ch4_air(mech, 1.0)
    T = np.array([T0])
    p = np.array([fields.P_ATM])
    h = np.array([0.0])
    t, dt = 0.0, 1e-9
    o = oracle.default_opts(rtol=1e-6, atol_Y=1e-12, max_steps=200000)
    while t < t_end:
        r = om.chem_step(T, p, Y, dt, h_inout=h, opts=o)
        if r["status"][0] != 0:
            return None, None
        T, Y, h = r["T"], r["Y"], r["h"]
        t += dt
        if T[0] - T0 > 400.0:
            return t, T[0]
        dt = min(dt * 1.2, 1e-3)
    return None, T[0]


def check(seed, verbose=True):
    try:
        mech = generate_large_mechanism(seed)
    except ValueError as e:
        if verbose:
            print(e, flush=True)
        return False
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.mech")
        synth.write_mech(path, mech)
        om = oracle.Mech(path)
        tau, _ = ignition(om, mech, 1500.0)
        if tau is None:
            if verbose:
                print(f"seed {seed}: no ignition within 0.1 s at 1500 K", flush=True)
            return False
        f = fields.hydrocarbon_field(mech, n=128)
        r = om.chem_step(f["T"], f["p"], f["Y"], 1e-6, nthreads=8)
        if np.any(r["status"] != 0):
            if verbose:
                print(f"seed {seed}: {np.count_nonzero(r['status'])} failed cells in the field", flush=True)
            return False
        # end state of the ignition: a long step from the ignited state
        Y = fields.premixed_ch4_air(mech, 1.0)
        o = oracle.default_opts(rtol=1e-6, atol_Y=1e-12, max_steps=400000)
        e = om.chem_step(np.array([1500.0]), np.array([fields.P_ATM]), Y, 0.05, opts=o)
        if e["status"][0] != 0 or e["T"][0] < 1800.0:
            if verbose:
                print(f"seed {seed}: end state {e['status'][0]} T {e['T'][0]:.0f}", flush=True)
            return False
        if verbose:
            print(f"seed {seed}: ACCEPT ignition at 1500 K after {tau:.3e} s, T(50 ms) = {e['T'][0]:.0f} K, "
                  f"field sub-steps mean {r['n_acc'].mean():.0f} max {r['n_acc'].max()}", flush=True)
        return True


if __name__ == "__main__":
    base = int(sys.argv[1]) if len(sys.argv) > 1 else 20221101
    tries = int(sys.argv[2]) if len(sys.argv) > 2 else 50
    for s in range(base, base + tries):
        if check(s):
            print(s)
            break
