"""P5, P6: the Rosenbrock core of the oracle.

P5 converts the oracle's transformed coefficients back to the standard form
(alpha, gamma, b) and checks the Rosenbrock order conditions up to order 4
(order 3 for the embedded weights), and L-stability.  P6 checks linear
problems against the matrix exponential and the stability function, and the
observed order under step refinement.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle


def _standard_form():
    g, a, c, m, mh = oracle.rodas4_tableau()
    Gi = np.eye(6) / g - c
    G = np.linalg.inv(Gi)
    alpha = a @ G
    b = m @ G
    bh = mh @ G
    beta = alpha + G
    np.fill_diagonal(beta, 0.0)
    return g, alpha, beta, G, b, bh


def _conditions(b, alpha, beta, g):
    ai = alpha.sum(1)
    bi = beta.sum(1)
    return np.array([
        b.sum() - 1,
        b @ bi - (0.5 - g),
        b @ ai ** 2 - 1 / 3,
        b @ (beta @ bi) - (1 / 6 - g + g * g),
        b @ ai ** 3 - 1 / 4,
        b @ (ai * (alpha @ bi)) - (1 / 8 - g / 3),
        b @ (beta @ ai ** 2) - (1 / 12 - g / 3),
        b @ (beta @ (beta @ bi)) - (1 / 24 - g / 2 + 1.5 * g * g - g ** 3),
    ])


def test_P5_order_conditions():
    g, alpha, beta, G, b, bh = _standard_form()
    assert np.allclose(np.diag(G), g, rtol=0, atol=1e-14)
    assert np.max(np.abs(_conditions(b, alpha, beta, g))) < 1e-13
    ch = _conditions(bh, alpha, beta, g)
    assert np.max(np.abs(ch[:4])) < 1e-13
    assert np.max(np.abs(ch[4:])) > 1e-3          # the embedded method is of order exactly 3


def test_P5_L_stability():
    g, alpha, beta, G, b, bh = _standard_form()
    B = alpha + G

    def R(z, w):
        return 1 + z * w @ np.linalg.solve(np.eye(6) - z * B, np.ones(6))

    for z in (-1e6, -1e9, -1e12):
        assert abs(R(z, b)) < 1e3 / abs(z)
        assert abs(R(z, bh)) < 1e3 / abs(z)
    # A-stability on a sample of the left half plane
    for x in np.linspace(-50, 0, 11):
        for yv in np.linspace(-50, 50, 11):
            assert abs(R(complex(x, yv), b)) <= 1 + 1e-12


def test_P6_fixed_step_is_stability_function():
    """One step on y' = Ay equals R(hA) y0 with R from the standard form."""
    rng = np.random.default_rng(0)
    A = rng.normal(size=(4, 4)) - 3 * np.eye(4)
    y0 = rng.normal(size=4)
    h = 0.3
    g, alpha, beta, G, b, bh = _standard_form()
    B = alpha + G
    # R(Z) = I + sum_i b_i k_i / y-form for matrices: stages k = (I (x) I - B (x) hA)^{-1} (1 (x) hA y0)
    n = 4
    big = np.eye(6 * n) - np.kron(B, h * A)
    k = np.linalg.solve(big, np.kron(np.ones(6), h * A @ y0))
    y_ref = y0 + np.kron(b, np.eye(n)) @ k
    y1, _ = oracle.linear_fixed_step(A, y0, h)
    np.testing.assert_allclose(y1, y_ref, rtol=1e-13, atol=1e-13)


def test_P6_linear_adaptive_matches_expm():
    rng = np.random.default_rng(1)
    # stiff linear system with eigenvalues spread over 6 decades
    Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    lam = -np.logspace(0, 6, 6)
    A = Q @ np.diag(lam) @ Q.T
    y0 = rng.normal(size=6)
    dt = 2.0
    y, st, hn, na, nr = oracle.linear_integrate(A, y0, dt, rtol=1e-10, atol=np.full(6, 1e-14))
    assert st == 0
    np.testing.assert_allclose(y, expm(A * dt) @ y0, rtol=0, atol=1e-9 * np.abs(y0).max())


def test_P6_observed_order_four():
    """Global error of fixed steps on a linear oscillator decays as h^4."""
    A = np.array([[0.0, 1.0], [-1.0, -0.1]])
    y0 = np.array([1.0, 0.0])
    T = 2.0
    exact = expm(A * T) @ y0
    errs = []
    for n in (8, 16, 32, 64):
        y = y0.copy()
        for _ in range(n):
            y, _ = oracle.linear_fixed_step(A, y, T / n)
        errs.append(np.linalg.norm(y - exact))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 4.0) < 0.25), slopes


def test_controller_counts_and_hnext():
    """h_next carries over: a second call started with it takes no more steps."""
    A = np.array([[-1e3, 0.0], [1e3, -1.0]])
    y0 = np.array([1.0, 0.0])
    y1, st, hn, na, nr = oracle.linear_integrate(A, y0, 1e-2, rtol=1e-8, atol=np.full(2, 1e-12))
    assert st == 0 and na > 1 and hn > 0
    y2, st2, hn2, na2, nr2 = oracle.linear_integrate(A, y1, 1e-2, h_in=hn, rtol=1e-8, atol=np.full(2, 1e-12))
    assert st2 == 0 and na2 <= na


def test_max_steps_and_underflow_status():
    A = np.array([[-1e3, 0.0], [1e3, -1.0]])
    y0 = np.array([1.0, 0.0])
    _, st, _, na, nr = oracle.linear_integrate(A, y0, 1.0, rtol=1e-10, atol=np.full(2, 1e-14), max_steps=3)
    assert st == 1 and na + nr == 3
    _, st, _, _, _ = oracle.linear_integrate(A, y0, 1.0, h_in=1e-3, rtol=1e-10, atol=np.full(2, 1e-14), h_min=1e-3)
    assert st == 2
