"""Pins of the oracle's thermo, rate constants and right-hand side.

Each pin is fixed by mathematics or physics rather than by re-evaluating the
oracle's own formula: calculus identities of the thermo polynomials,
conservation laws of the reactor, limits of the falloff form, detailed
balance at equilibrium, and an independent NumPy evaluation.
"""
import numpy as np
import pytest

from conftest import random_states

R = 8.31446261815324


def _d5(f, x, h):
    """5-point central difference (error O(h^4))."""
    return (-f(x + 2 * h) + 8 * f(x + h) - 8 * f(x - h) + f(x - 2 * h)) / (12 * h)


@pytest.mark.parametrize("T", [300.0, 800.0, 1500.0, 2500.0, 3400.0])
def test_P1_enthalpy_derivative_is_cp(h2_oracle, T):
    cp, h, s, g = h2_oracle.thermo(T)
    H = lambda t: h2_oracle.thermo(t)[1] * t          # H/R
    S = lambda t: h2_oracle.thermo(t)[2]              # S/R
    np.testing.assert_allclose(_d5(H, T, 0.5), cp, rtol=1e-9)
    np.testing.assert_allclose(_d5(S, T, 0.5) * T, cp, rtol=1e-9)
    np.testing.assert_allclose(g, h - s, rtol=0, atol=1e-12 * np.abs(s).max())


def test_mixture_ideal_gas(h2_oracle, h2_mech):
    for T, Y in random_states(h2_mech, 5):
        Wbar, rho, cp, hm = h2_oracle.mixture(T, 2e5, Y)
        W = h2_mech.molar_mass * 1e-3
        assert abs(Wbar - 1 / np.sum(Y / W)) < 1e-15
        assert abs(rho - 2e5 * Wbar / (R * T)) < 1e-12 * rho
        cpk = h2_oracle.thermo(T)[0] * R / W
        assert abs(cp - np.sum(Y * cpk)) < 1e-12 * cp


def test_P3_conservation(h2_oracle, h2_mech):
    W = h2_mech.molar_mass * 1e-3
    A = h2_mech.composition
    for T, Y in random_states(h2_mech, 20):
        p = 101325.0 * 3
        kf, kr, q, wdot = h2_oracle.rates(T, p, Y)
        scale = np.abs(q).max() * 1e6
        # elements: sum_k a_ek wdot_k = 0
        np.testing.assert_allclose(A.T @ wdot, 0, atol=1e-13 * scale * 4)
        # mass: sum_k W_k wdot_k = 0
        assert abs(np.sum(W * wdot)) < 1e-13 * scale * 0.04
        # enthalpy at constant p: sum_k h_k dY_k/dt + cp dT/dt = 0
        y = np.concatenate([[T], Y])
        f = h2_oracle.rhs(p, y)
        _, _, cp, _ = h2_oracle.mixture(T, p, Y)
        hk = h2_oracle.thermo(T)[1] * R * T / W
        lhs = np.sum(hk * f[1:]) + cp * f[0]
        assert abs(lhs) <= 1e-12 * np.sum(np.abs(hk * f[1:]))
        # sum Y stays 1
        assert abs(np.sum(f[1:])) <= 1e-13 * np.abs(f[1:]).sum()


def test_numpy_rhs_agrees(h2_oracle, npchem, h2_mech):
    for T, Y in random_states(h2_mech, 10, seed=3):
        y = np.concatenate([[T], Y])
        a = h2_oracle.rhs(101325.0, y)
        b = npchem.rhs(101325.0, y)
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-12 * np.abs(b).max())


def test_P2_detailed_balance_equilibrium_constant(h2_oracle, h2_mech, npchem):
    """At a state in chemical equilibrium every reaction's net rate vanishes.

    The equilibrium composition is found by an independent Gibbs
    minimisation (element potentials) at fixed T, p; at that composition the
    forward and reverse terms of each reaction must balance.
    """
    from test_oracle_equilibrium import gibbs_equilibrium_TP
    T, p = 2200.0, 101325.0
    Y0 = np.zeros(h2_mech.n_species)
    Y0[h2_mech.index("H2")], Y0[h2_mech.index("O2")], Y0[h2_mech.index("N2")] = 0.0285, 0.2264, 0.7451
    Yeq = gibbs_equilibrium_TP(npchem, h2_mech, T, p, Y0)
    kf, kr, q, wdot = h2_oracle.rates(T, p, Yeq)
    W = h2_mech.molar_mass * 1e-3
    _, rho, _, _ = h2_oracle.mixture(T, p, Yeq)
    c = rho * Yeq / W * 1e-6
    for j in range(h2_mech.n_reactions):
        fwd = kf[j] * np.prod(c ** h2_mech.nu_reac[j])
        if h2_mech.reaction_type[j] == 1:
            fwd *= np.sum(h2_mech.efficiency[j] * c)
        assert abs(q[j]) <= 1e-8 * fwd, (j, q[j], fwd)


def _one_reaction_mech(h2_mech, j):
    import copy
    m = copy.deepcopy(h2_mech)
    keep = [j]
    for key in ("reaction_type", "nu_reac", "nu_prod", "arrhenius", "efficiency", "falloff_low", "troe"):
        setattr(m, key, getattr(m, key)[keep])
    return m


def test_troe_limits(h2_mech, tmp_path):
    """Falloff limits at extreme [M] and the Lindemann form when F_cent = 1."""
    import copy
    import oracle
    import synth
    j = int(np.where(h2_mech.reaction_type == 2)[0][0])
    m = _one_reaction_mech(h2_mech, j)
    A, b, Ta = m.arrhenius[0]
    A0, b0, Ta0 = m.falloff_low[0]
    T = 1300.0
    kinf = A * T ** b * np.exp(-Ta / T)
    k0 = A0 * T ** b0 * np.exp(-Ta0 / T)
    path = tmp_path / "one.mech"
    synth.write_mech(path, m)
    om = oracle.Mech(path)
    Y = np.full(9, 1.0 / 9)
    # Lindemann special case: alpha = 1, T* huge, T** huge -> F_cent = 1 -> F = 1
    ml = copy.deepcopy(m)
    ml.troe[0] = (1.0, 100.0, 1e30, 1e30)
    pl = tmp_path / "lind.mech"
    synth.write_mech(pl, ml)
    oml = oracle.Mech(pl)
    for p in (1e2, 1e4, 1e5, 1e6, 1e8):
        _, rho, _, _ = oml.mixture(T, p, Y)
        c = rho * Y / (m.molar_mass * 1e-3) * 1e-6
        M = np.sum(m.efficiency[0] * c)
        kf = oml.rates(T, p, Y)[0][0]
        Pr = k0 * M / kinf
        np.testing.assert_allclose(kf, kinf * Pr / (1 + Pr), rtol=1e-12)
    # pressure limits of the full Troe form: as log10 Pr -> +-inf the
    # broadening exponent 1/(1 + f1^2) tends to 1/(1 + (1/0.14)^2), so
    # k -> k_inf F_lim (high [M]) and k -> k_0 [M] F_lim (low [M])
    al, T3, T1, T2 = m.troe[0]
    Fc = (1 - al) * np.exp(-T / T3) + al * np.exp(-T / T1) + np.exp(-T2 / T)
    F_lim = Fc ** (1.0 / (1.0 + (1.0 / 0.14) ** 2))
    kf_hi = om.rates(T, 1e200, Y)[0][0]
    assert abs(kf_hi / (kinf * F_lim) - 1) < 5e-3
    p_lo = 1e-200
    _, rho, _, _ = om.mixture(T, p_lo, Y)
    c = rho * Y / (m.molar_mass * 1e-3) * 1e-6
    M = np.sum(m.efficiency[0] * c)
    kf_lo = om.rates(T, p_lo, Y)[0][0]
    assert abs(kf_lo / (k0 * M * F_lim) - 1) < 5e-3


def test_troe_centre_equals_fcent(h2_mech, tmp_path):
    """At the centre of the falloff curve (log10 Pr = -c) the broadening factor
    equals F_cent, so k = k_inf Pr/(1+Pr) F_cent."""
    import oracle
    import synth
    j = int(np.where(h2_mech.reaction_type == 2)[0][0])
    m = _one_reaction_mech(h2_mech, j)
    A, b, Ta = m.arrhenius[0]
    A0, b0, Ta0 = m.falloff_low[0]
    al, T3, T1, T2 = m.troe[0]
    T = 1500.0
    Fc = (1 - al) * np.exp(-T / T3) + al * np.exp(-T / T1) + np.exp(-T2 / T)
    c = -0.4 - 0.67 * np.log10(Fc)
    Pr_target = 10 ** (-c)
    kinf = A * T ** b * np.exp(-Ta / T)
    k0 = A0 * T ** b0 * np.exp(-Ta0 / T)
    # choose p so that [M] gives Pr_target (all efficiencies weighted by Y)
    Y = np.full(9, 1.0 / 9)
    path = tmp_path / "one.mech"
    synth.write_mech(path, m)
    om = oracle.Mech(path)
    _, rho1, _, _ = om.mixture(T, 1.0, Y)
    M1 = np.sum(m.efficiency[0] * rho1 * Y / (m.molar_mass * 1e-3) * 1e-6)   # [M] per Pa
    p = Pr_target * kinf / k0 / M1
    kf = om.rates(T, p, Y)[0][0]
    np.testing.assert_allclose(kf, kinf * Pr_target / (1 + Pr_target) * Fc, rtol=1e-9)
