"""0-D rollouts -- test infrastructure only.

n consecutive chemistry steps of length dt with the oracle's integrator (carrying each cell's
sub-step hint, as a solver does from one flow step to the next) or the oracle's DNN step, and
the ignition delay of each cell: the time of the largest temperature rate on the sampled
trajectory, r_k = (T_{k+1} - T_k)/dt at t_k = (k + 1/2) dt, refined by the vertex of the parabola
through the rates of the steps before, at and after the maximum; NaN when the maximum falls on
the first or the last step.
"""
from __future__ import annotations

import numpy as np


def ignition_delay(T_traj, dt):
    """T_traj [n_steps + 1, n] -> ignition delay [n]."""
    r = np.diff(np.asarray(T_traj, dtype=np.float64), axis=0) / dt
    steps = r.shape[0]
    k = np.argmax(r, axis=0)
    out = np.full(r.shape[1], np.nan)
    for i, kb in enumerate(k):
        if kb <= 0 or kb + 1 >= steps:
            continue
        a, b, c = r[kb - 1, i], r[kb, i], r[kb + 1, i]
        den = a - 2.0 * b + c
        off = 0.5 * (a - c) / den if den < 0.0 else 0.0
        out[i] = (kb + 0.5 + off) * dt
    return out


def integrator_rollout(om, T, p, Y, dt, n_steps, nthreads=0, constant_volume=False):
    """Constant pressure p, or with constant_volume the constant-volume reactor at density p."""
    T = np.array(T, dtype=np.float64, copy=True)
    Y = np.array(Y, dtype=np.float64, copy=True)
    h = np.zeros(T.size)
    traj = [T.copy()]
    step = om.chem_step_v if constant_volume else om.chem_step
    for _ in range(n_steps):
        r = step(T, p, Y, dt, h_inout=h, nthreads=nthreads)
        T, Y, h = r["T"], r["Y"], r["h"]
        traj.append(T.copy())
    traj = np.array(traj)
    return traj, Y, ignition_delay(traj, dt)


def dnn_rollout(od, om, T, p, Y, dt, n_steps, nthreads=0):
    T = np.array(T, dtype=np.float64, copy=True)
    Y = np.array(Y, dtype=np.float64, copy=True)
    traj = [T.copy()]
    for _ in range(n_steps):
        r = od.step(om, T, p, Y, dt, mode=1, nthreads=nthreads)
        T, Y = r["T"], r["Y"]
        traj.append(T.copy())
    traj = np.array(traj)
    return traj, Y, ignition_delay(traj, dt)
