"""Pins of the oracle's rollout and ignition-delay definition (oracle/rollout.py)."""
import numpy as np

from oracle import rollout as ro
from synth import fields


def test_ignition_delay_of_a_logistic_trajectory():
    """T(t) = T0 + A / (1 + exp(-(t - t0)/w)) has its largest rate at t0 exactly; the sampled and
    refined delay recovers it to O(dt^2)."""
    w, t0, dt = 2e-5, 3.37e-4, 1e-6
    t = np.arange(0, 801) * dt
    T = 1000.0 + 800.0 / (1.0 + np.exp(-(t - t0) / w))
    idt = ro.ignition_delay(T[:, None], dt)[0]
    assert abs(idt - t0) < 0.05 * dt
    # the maximum on an end step is not a delay
    assert np.isnan(ro.ignition_delay(np.linspace(0, 1, 10)[:, None] ** 2, dt)[0])


def test_integrator_rollout_delays(h2_mech, h2_oracle):
    """Stoichiometric H2/air: a finite delay that shortens as T0 rises."""
    Y0 = fields.premixed_h2_air(h2_mech, 1.0).reshape(-1)
    Y = np.repeat(Y0[:, None], 2, axis=1)
    T = np.array([1000.0, 1050.0])
    p = np.full(2, 101325.0)
    traj, _, idt = ro.integrator_rollout(h2_oracle, T, p, Y, 1e-6, 800)
    assert traj.shape == (801, 2)
    assert np.all(np.isfinite(idt)) and idt[1] < idt[0]
    assert 1e-4 < idt[0] < 8e-4


def test_constant_volume_rollout_conserves_internal_energy(h2_mech, h2_oracle, npchem):
    """The paper's constant-volume case (phi = 1, 1000 K, 0.5 atm): along the whole trajectory the
    mixture internal energy stays at its initial value, the mass fractions keep their sum, and the
    pressure rho R T / Wbar rises through ignition; the delay is finite."""
    R = 8.31446261815324
    Y0 = fields.premixed_h2_air(h2_mech, 1.0).reshape(-1)
    T0, p0 = 1000.0, 0.5 * 101325.0
    rho = p0 / (R * T0 * np.sum(Y0 / npchem.W))
    u0 = npchem.u_mass(T0, Y0)
    T, Y = np.array([T0]), Y0[:, None].copy()
    h = np.zeros(1)
    traj = [T0]
    pmax = p0
    for _ in range(2500):
        r = h2_oracle.chem_step_v(T, np.array([rho]), Y, 1e-6, h_inout=h)
        T, Y, h = r["T"], r["Y"], r["h"]
        assert r["status"][0] == 0
        traj.append(T[0])
        cv = np.sum(Y[:, 0] * (npchem.cp_R(T[0]) - 1.0) * R / npchem.W)
        assert abs(npchem.u_mass(T[0], Y[:, 0]) - u0) <= 20 * 1e-8 * cv * T[0]
        pmax = max(pmax, rho * R * T[0] * np.sum(Y[:, 0] / npchem.W))
    assert abs(Y.sum() - Y0.sum()) < 1e-12
    assert traj[-1] - T0 > 150.0 and pmax > 1.1 * p0
    traj2, _, idt = ro.integrator_rollout(h2_oracle, np.array([T0]), np.array([rho]), Y0[:, None], 1e-6, 2500,
                                          constant_volume=True)
    assert np.array_equal(traj2[:, 0], np.array(traj))
    assert np.isfinite(idt[0]) and 1e-4 < idt[0] < 2.5e-3
