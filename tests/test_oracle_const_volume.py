"""Pins of the oracle's constant-volume reactor (the df0DFoam constant-volume case: density
fixed, pressure following from the state).  Checked against an independent NumPy right-hand
side (tests/npchem.py), complex-step derivatives of it, SciPy's Radau solver, and the
conservation laws of the closed, rigid, adiabatic reactor: total mass, elements and the
mixture internal energy; at long times every net rate of progress vanishes."""
import numpy as np
import pytest

from synth import fields

R = 8.31446261815324


def _states(h2_mech, h2_oracle, n=4, seed=9):
    f = fields.ignition_cells(h2_mech, n=n, seed=seed)
    rho = np.array([h2_oracle.mixture(f["T"][i], f["p"][i], f["Y"][:, i])[1] for i in range(n)])
    return f, rho


def test_rhs_and_jacobian(h2_mech, h2_oracle, npchem):
    rng = np.random.default_rng(3)
    f, rho = _states(h2_mech, h2_oracle)
    for i in range(4):
        Y = f["Y"][:, i] + rng.uniform(0, 1e-3, h2_mech.n_species)
        y = np.concatenate([[f["T"][i] + rng.uniform(0, 500)], Y / Y.sum()])
        fo = h2_oracle.rhs_v(rho[i], y)
        fn = npchem.rhs_v(rho[i], y)
        assert np.max(np.abs(fo - fn)) <= 1e-12 * np.max(np.abs(fn))
        J = h2_oracle.jacobian_v(rho[i], y)
        Jc = npchem.jac_v_complex_step(rho[i], y)
        assert np.max(np.abs(J - Jc)) <= 1e-9 * np.max(np.abs(Jc))


def test_conservation_over_a_step(h2_mech, h2_oracle, npchem):
    f, rho = _states(h2_mech, h2_oracle, n=6, seed=12)
    o = h2_oracle.chem_step_v(f["T"], rho, f["Y"], 2e-4, h_inout=np.zeros(6))
    assert np.all(o["status"] == 0)
    W = np.asarray(h2_mech.molar_mass)
    comp = np.asarray(h2_mech.composition, dtype=float)
    for i in range(6):
        Y0, Y1 = f["Y"][:, i], o["Y"][:, i]
        assert abs(Y1.sum() - Y0.sum()) < 1e-12
        assert np.allclose(comp.T @ (Y1 / W), comp.T @ (Y0 / W), rtol=1e-10, atol=1e-14)
        u0, u1 = npchem.u_mass(f["T"][i], Y0), npchem.u_mass(o["T"][i], Y1)
        cv = np.sum(Y1 * (npchem.cp_R(o["T"][i]) - 1.0) * R / npchem.W)
        assert abs(u1 - u0) <= 10 * 1e-8 * cv * o["T"][i]
    # the pressure rises with the heat release at fixed volume
    hot = o["T"] > f["T"] + 100
    assert hot.any()


def test_against_radau(h2_mech, h2_oracle, npchem):
    from scipy.integrate import solve_ivp
    f, rho = _states(h2_mech, h2_oracle, n=2, seed=21)
    dt = 1e-4
    o = h2_oracle.chem_step_v(f["T"], rho, f["Y"], dt, h_inout=np.zeros(2))
    for i in range(2):
        y0 = np.concatenate([[f["T"][i]], f["Y"][:, i]])
        r = solve_ivp(lambda t, y: npchem.rhs_v(rho[i], y), (0, dt), y0, method="Radau", rtol=1e-12,
                      atol=np.concatenate([[1e-9], np.full(h2_mech.n_species, 1e-16)]),
                      jac=lambda t, y: npchem.jac_v_complex_step(rho[i], y))
        yr = r.y[:, -1]
        assert abs(o["T"][i] - yr[0]) <= 1e-6 * yr[0]
        big = yr[1:] > 1e-8
        assert np.max(np.abs(o["Y"][big, i] - yr[1:][big]) / yr[1:][big]) < 1e-5


def test_long_time_limit_is_equilibrium(h2_mech, h2_oracle):
    """After 1 s every net rate of progress is below 1e-6 of the largest forward rate."""
    f, rho = _states(h2_mech, h2_oracle, n=2, seed=5)
    o = h2_oracle.chem_step_v(f["T"], rho, f["Y"], 1.0, h_inout=np.zeros(2))
    assert np.all(o["status"] == 0)
    W = np.asarray(h2_mech.molar_mass) * 1e-3
    nu_r = np.asarray(h2_mech.nu_reac)
    eff = np.asarray(h2_mech.efficiency)
    for i in range(2):
        Y = o["Y"][:, i]
        p = rho[i] * R * o["T"][i] * np.sum(Y / W)
        kf, _, q, _ = h2_oracle.rates(o["T"][i], p, Y)
        c = 1e-6 * rho[i] * Y / W
        Mq = np.where(np.asarray(h2_mech.reaction_type) == 1, eff @ c, 1.0)
        fwd = kf * np.prod(c[None, :] ** nu_r, axis=1) * Mq
        assert np.max(np.abs(q)) < 1e-6 * np.max(fwd)
