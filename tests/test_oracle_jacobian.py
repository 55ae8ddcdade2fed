"""P4: the oracle's analytic Jacobian against derivatives taken independently:
complex-step derivatives of the independent NumPy right-hand side, and
high-order central differences of the oracle's own right-hand side."""
import numpy as np
import pytest

from conftest import random_states


def _check(J, Jref, rtol):
    scale = np.abs(Jref).max(axis=1, keepdims=True) + 1e-300
    err = np.abs(J - Jref) / scale
    assert err.max() < rtol, (err.max(), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_P4_jacobian_vs_complex_step(h2_oracle, npchem, h2_mech, seed):
    for T, Y in random_states(h2_mech, 4, seed=seed, T_range=(500.0, 2800.0)):
        y = np.concatenate([[T], Y])
        for p in (101325.0, 10 * 101325.0):
            J = h2_oracle.jacobian(p, y)
            Jc = npchem.jac_complex_step(p, y)
            _check(J, Jc, 1e-9)


def test_P4_jacobian_on_config_states(h2_oracle, npchem, cfg1):
    # radical-free inputs: many zero concentrations (mass-action derivatives at c = 0)
    for i in (0, 100, 500):
        y = np.concatenate([[cfg1["T"][i]], cfg1["Y"][:, i]])
        J = h2_oracle.jacobian(101325.0, y)
        Jc = npchem.jac_complex_step(101325.0, y)
        _check(J, Jc, 1e-9)


def test_P4_jacobian_vs_central_differences(h2_oracle, h2_mech):
    T, Y = random_states(h2_mech, 1, seed=11, T_range=(1500.0, 1600.0))[0]
    y = np.concatenate([[T], Y])
    p = 101325.0
    J = h2_oracle.jacobian(p, y)
    N = y.size
    Jfd = np.zeros((N, N))
    for l in range(N):
        h = 1e-3 * (abs(y[l]) if l else 1.0) if l == 0 else 1e-4 * y[l]
        def f(s):
            yy = y.copy()
            yy[l] += s
            return h2_oracle.rhs(p, yy)
        Jfd[:, l] = (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)
    _check(J, Jfd, 1e-5)
