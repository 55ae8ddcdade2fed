"""Pick the seed of the synthetic H2/air mechanism (run once; prints the seed).

Test infrastructure: it runs the CPU oracle.  Starting from a base seed it
tries seeds in order and accepts the first mechanism that
  1. ignites (T rise > 400 K) within 1 s from 1000 K, phi = 1, 1 atm;
  2. has an ignition delay that decreases from 1000 K to 1600 K;
  3. reaches an equilibrium temperature in [2000, 3000] K from 1600 K
     (a hot start that ignites quickly; the enthalpy-pressure equilibrium
     from 300 K is checked by the tests with an independent Gibbs
     minimisation);
  4. integrates the 1024-cell ignition set and the 65,536-cell hot-kernel
     field over dt = 1e-6 s at rtol 1e-8 with every cell OK.
The ignition delay is the time of the largest dT/dt on the sampled trajectory.

    python oracle/select_mech_seed.py [base_seed] [max_tries]
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


def ignition(om, mech, T0, phi=1.0, t_end=1.0, rtol=1e-6):
    Y = fields.premixed_h2_air(mech, phi)
    T = np.array([T0])
    p = np.array([fields.P_ATM])
    h = np.array([0.0])
    t, dt = 0.0, 1e-9
    ts, Ts = [0.0], [T0]
    t_rise = None
    o = oracle.default_opts(rtol=rtol, atol_Y=1e-12, max_steps=20000)
    while t < t_end:
        r = om.chem_step(T, p, Y, dt, h_inout=h, opts=o)
        if r["status"][0] != 0:
            return None, None
        T, Y, h = r["T"], r["Y"], r["h"]
        t += dt
        ts.append(t)
        Ts.append(T[0])
        if T[0] - T0 > 400 and t_rise is None:
            t_rise = t
        if t_rise is not None and t > 3 * t_rise:
            break
        dt = min(dt * 1.1, 2e-3)
    Ts, ts = np.array(Ts), np.array(ts)
    if Ts.max() - T0 <= 400:
        return None, Ts[-1]
    i = int(np.argmax(np.diff(Ts) / np.diff(ts)))
    return 0.5 * (ts[i] + ts[i + 1]), Ts[-1]


def equilibrium_T(om, mech, T0=1600.0):
    Y = fields.premixed_h2_air(mech, 1.0)
    T = np.array([T0])
    p = np.array([fields.P_ATM])
    o = oracle.default_opts(rtol=1e-6, atol_Y=1e-12, max_steps=200000)
    r = om.chem_step(T, p, Y, 1.0, opts=o)
    return r["T"][0] if r["status"][0] == 0 else None


def check(seed, verbose=True):
    mech = synth.generate_h2_mechanism(seed)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.mech")
        synth.write_mech(path, mech)
        om = oracle.Mech(path)
        idt = []
        for T0 in (1000.0, 1200.0, 1400.0, 1600.0):
            tau, _ = ignition(om, mech, T0)
            idt.append(tau)
            if tau is None:
                if verbose:
                    print(f"seed {seed}: no ignition within 1 s at {T0} K")
                return False
        if not all(a > b for a, b in zip(idt[:-1], idt[1:])):
            if verbose:
                print(f"seed {seed}: ignition delay not decreasing {idt}")
            return False
        Teq = equilibrium_T(om, mech)
        if Teq is None or not (2000.0 <= Teq <= 3000.0):
            if verbose:
                print(f"seed {seed}: equilibrium T {Teq}")
            return False
        for f in (fields.ignition_cells(mech), fields.hot_kernel_field_2d(mech)):
            r = om.chem_step(f["T"], f["p"], f["Y"], 1e-6)
            if np.any(r["status"] != 0):
                if verbose:
                    print(f"seed {seed}: {np.count_nonzero(r['status'])} failed cells in a field")
                return False
        if verbose:
            print(f"seed {seed}: ACCEPT idt={['%.3e' % x for x in idt]} Teq(1600K start)={Teq:.1f}")
        return True


if __name__ == "__main__":
    base = int(sys.argv[1]) if len(sys.argv) > 1 else 20221014
    tries = int(sys.argv[2]) if len(sys.argv) > 2 else 200
    for s in range(base, base + tries):
        if check(s):
            print(s)
            break
