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
