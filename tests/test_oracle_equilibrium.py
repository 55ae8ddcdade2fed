"""Long-time pin (P8): the oracle's reactor converges to the enthalpy-pressure
equilibrium found by an independent Gibbs minimisation (element potentials)."""
import numpy as np
import pytest
from scipy.optimize import brentq, root

R = 8.31446261815324
P0 = 101325.0


def gibbs_equilibrium_TP(npc, mech, T, p, Y0):
    """Composition minimising the Gibbs energy at fixed T, p and element totals.

    Element-potential form: at the minimum mu_k = g_k/RT + ln(p/p0) +
    ln(n_k/N) = sum_e lambda_e a_ek for every species, so
    n_k = N exp(sum_e lambda_e a_ek - g_k/RT - ln(p/p0)); the unknowns
    (lambda, ln N) are fixed by the element totals and sum n_k = N.
    """
    A = mech.composition.astype(float)             # [K, E]
    W = mech.molar_mass * 1e-3
    n0 = Y0 / W                                    # mol per kg of mixture
    b = A.T @ n0
    mu0 = (npc.h_RT(T) - npc.s_R(T)) + np.log(p / P0)

    def species(x):
        lam, lnN = x[:-1], x[-1]
        return np.exp(np.clip(lnN + A @ lam - mu0, -700, 700))

    def resid(x):
        n = species(x)
        return np.concatenate([np.log(A.T @ n) - np.log(b), [np.log(n.sum()) - x[-1]]])

    # start: potentials fitted to the major species of complete combustion
    lnN0 = np.log(n0.sum())
    major = [mech.index(s) for s in ("H2O", "O2", "N2", "H2")]
    lam0, *_ = np.linalg.lstsq(A[major], mu0[major] + np.log(0.2), rcond=None)
    sol = root(resid, np.concatenate([lam0, [lnN0]]), method="hybr", tol=1e-14)
    if not sol.success:
        sol = root(resid, sol.x, method="lm", tol=1e-15)
    n = species(sol.x)
    assert np.max(np.abs(resid(sol.x))) < 1e-11, sol
    Y = n * W
    return Y / Y.sum()


def hp_equilibrium(npc, mech, T0, p, Y0):
    h0 = npc.h_mass(T0, Y0)

    def g(T):
        return npc.h_mass(T, gibbs_equilibrium_TP(npc, mech, T, p, Y0)) - h0

    Teq = brentq(g, 1000.0, 3400.0, xtol=1e-10, rtol=1e-14)
    return Teq, gibbs_equilibrium_TP(npc, mech, Teq, p, Y0)


def _premixed(mech, phi=1.0):
    from synth import fields
    return fields.premixed_h2_air(mech, phi)[:, 0]


def test_equilibrium_solver_stationarity(npchem, h2_mech):
    """The Gibbs solver itself: element totals kept, and a perturbation
    that keeps element totals never lowers G."""
    Y0 = _premixed(h2_mech)
    T, p = 2300.0, P0
    Y = gibbs_equilibrium_TP(npchem, h2_mech, T, p, Y0)
    A = h2_mech.composition.astype(float)
    W = h2_mech.molar_mass * 1e-3
    np.testing.assert_allclose(A.T @ (Y / W), A.T @ (Y0 / W), rtol=1e-12)

    def G(n):
        N = n.sum()
        mu0 = (npchem.h_RT(T) - npchem.s_R(T)) + np.log(p / P0)
        return np.sum(n * (mu0 + np.log(np.maximum(n, 1e-300) / N)))

    n = Y / W
    G0 = G(n)
    # null-space directions of the element matrix
    _, _, vt = np.linalg.svd(A.T)
    null = vt[A.shape[1]:]
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = null.T @ rng.normal(size=null.shape[0])
        d *= 1e-4 * n.min() / np.abs(d).max()
        assert G(n + d) >= G0 - 1e-15 * abs(G0)


def test_hp_equilibrium_temperature_from_300K(npchem, h2_mech):
    """Mechanism acceptance: the adiabatic equilibrium from 300 K, phi = 1,
    lies in [2000, 3000] K."""
    Teq, _ = hp_equilibrium(npchem, h2_mech, 300.0, P0, _premixed(h2_mech))
    assert 2000.0 <= Teq <= 3000.0


@pytest.mark.slow
@pytest.mark.parametrize("T0,phi", [(1200.0, 1.0), (1500.0, 0.6)])
def test_P8_long_time_limit_is_hp_equilibrium(h2_oracle, npchem, h2_mech, T0, phi):
    import oracle
    Y0 = _premixed(h2_mech, phi)
    Teq, Yeq = hp_equilibrium(npchem, h2_mech, T0, P0, Y0)
    o = oracle.default_opts(rtol=1e-10, atol_Y=1e-16, max_steps=1000000)
    r = h2_oracle.chem_step(np.array([T0]), np.array([P0]), Y0[:, None], 1.0, opts=o)
    assert r["status"][0] == 0
    assert abs(r["T"][0] - Teq) <= 1e-6 * Teq
    big = Yeq > 1e-4
    np.testing.assert_allclose(r["Y"][big, 0], Yeq[big], rtol=2e-5)
