"""Pins of the oracle's chemistry step (P6 closed forms, P7, P9-P12)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import synth
from synth import testmechs

R = 8.31446261815324
P0 = 101325.0


def _mech(tmp_path, m, name):
    p = tmp_path / f"{name}.mech"
    synth.write_mech(p, m)
    return oracle.Mech(p)


def test_P6_isomerisation_closed_form(tmp_path):
    m = testmechs.isomerisation()
    om = _mech(tmp_path, m, "iso")
    kf = m.arrhenius[0, 0]
    kr = kf / np.exp(m.nasa7[1, 6] - m.nasa7[0, 6])
    n = 5
    YA0 = np.linspace(0.1, 0.9, n)
    Y = np.vstack([YA0, 1 - YA0])
    T = np.full(n, 900.0)
    dt = 1e-5
    r = om.chem_step(T, np.full(n, P0), Y, dt)
    assert np.all(r["status"] == 0)
    YAeq = kr / (kf + kr)
    exact = YAeq + (YA0 - YAeq) * np.exp(-(kf + kr) * dt)
    np.testing.assert_allclose(r["Y"][0], exact, rtol=1e-7)
    np.testing.assert_allclose(r["T"], 900.0, rtol=1e-14)


@pytest.mark.parametrize("third_body", [False, True])
def test_P6_bimolecular_closed_form(tmp_path, third_body):
    """Second-order kinetics in mol/cm^3 pins the unit handling (CGS rate
    constants, concentrations rho Y / W) and, with a third body, [M] with
    efficiencies."""
    k = 1.0e11 if not third_body else 3.0e15
    m = testmechs.bimolecular(k=k, third_body=third_body)
    om = _mech(tmp_path, m, "bi")
    T0 = 1000.0
    Y = np.array([[0.05], [0.08], [0.0], [0.87]])
    dt = 2e-5
    r = om.chem_step(np.array([T0]), np.array([P0]), Y, dt)
    assert r["status"][0] == 0
    W = 20e-3
    rho = P0 * W / (R * T0)
    A0, B0 = rho * 0.05 / W * 1e-6, rho * 0.08 / W * 1e-6
    keff = k
    if third_body:
        ctot = rho / W * 1e-6
        keff = k * (ctot * (1 - 0.87) + 3.0 * ctot * 0.87)
    D = B0 - A0
    A_t = A0 * D / (B0 * np.exp(D * keff * dt) - A0)
    YA_exact = A_t * 1e6 * W / rho
    assert abs(r["Y"][0, 0] / YA_exact - 1) < 1e-7
    assert 0.2 < YA_exact / 0.05 < 0.8          # the reaction is well under way


def test_P9_linear_invariants(h2_oracle, h2_mech, cfg1):
    r = h2_oracle.chem_step(cfg1["T"], cfg1["p"], cfg1["Y"], 1e-6)
    assert np.all(r["status"] == 0)
    W = h2_mech.molar_mass * 1e-3
    A = h2_mech.composition.astype(float)
    e0 = A.T @ (cfg1["Y"] / W[:, None])
    e1 = A.T @ (r["Y"] / W[:, None])
    np.testing.assert_allclose(e1, e0, rtol=1e-13)
    np.testing.assert_allclose(r["Y"].sum(axis=0), 1.0, rtol=0, atol=2e-14)


def test_P10_enthalpy_conserved(h2_oracle, cfg1):
    r = h2_oracle.chem_step(cfg1["T"], cfg1["p"], cfg1["Y"], 1e-6)
    for i in range(0, 1024, 37):
        _, _, cp0, h0 = h2_oracle.mixture(cfg1["T"][i], P0, cfg1["Y"][:, i])
        _, _, _, h1 = h2_oracle.mixture(r["T"][i], P0, r["Y"][:, i])
        assert abs(h1 - h0) <= 10 * 1e-8 * cp0 * cfg1["T"][i]


def _radau(npchem, y0, dt, p=P0):
    sol = solve_ivp(lambda t, y: npchem.rhs(p, y), (0.0, dt), y0, method="Radau", rtol=1e-12,
                    atol=np.concatenate([[1e-10], np.full(y0.size - 1, 1e-20)]),
                    jac=lambda t, y: npchem.jac_complex_step(p, y))
    assert sol.success
    return sol.y[:, -1]


@pytest.mark.slow
def test_P7_matches_radau(h2_oracle, npchem, cfg1):
    idx = [0, 17, 311, 702]
    r = h2_oracle.chem_step(cfg1["T"][idx], cfg1["p"][idx], cfg1["Y"][:, idx], 1e-6)
    for c, i in enumerate(idx):
        y0 = np.concatenate([[cfg1["T"][i]], cfg1["Y"][:, i]])
        ye = _radau(npchem, y0, 1e-6)
        assert abs(r["T"][c] - ye[0]) <= 10 * 1e-8 * ye[0]
        big = ye[1:] > 1e-6
        np.testing.assert_allclose(r["Y"][big, c], ye[1:][big], rtol=10 * 1e-8 * 5)


def test_P12_brute_force_rk4_tiny_horizon(h2_oracle, npchem, cfg1):
    """On a 1e-10 s horizon the system is not stiff: classical RK4 with many
    fixed steps is the reference."""
    i = 5
    y0 = np.concatenate([[cfg1["T"][i]], cfg1["Y"][:, i]])
    dt = 1e-10
    n = 2000
    h = dt / n
    y = y0.copy()
    f = lambda v: npchem.rhs(P0, v)
    for _ in range(n):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    r = h2_oracle.chem_step(np.array([y0[0]]), np.array([P0]), y0[1:, None], dt)
    assert abs(r["T"][0] - y[0]) <= 1e-8 * y[0]
    dY_ref = y[1:] - y0[1:]
    dY = r["Y"][:, 0] - y0[1:]
    big = np.abs(dY_ref) > 1e-12
    np.testing.assert_allclose(dY[big], dY_ref[big], rtol=1e-5)


def _idt(om, T0, dt, t_end, mech):
    from synth import fields
    Y = fields.premixed_h2_air(mech, 1.0)
    T = np.array([T0])
    p = np.array([P0])
    h = np.array([0.0])
    ts, Ts = [0.0], [T0]
    t = 0.0
    while t < t_end - 1e-15:
        r = om.chem_step(T, p, Y, dt, h_inout=h)
        assert r["status"][0] == 0
        T, Y, h = r["T"], r["Y"], r["h"]
        t += dt
        ts.append(t)
        Ts.append(T[0])
    Ts = np.array(Ts)
    rate = np.diff(Ts) / dt
    i = int(np.argmax(rate))
    # parabola through the three rates around the maximum (rates sit at mid-points)
    if 0 < i < len(rate) - 1:
        a, b, c = rate[i - 1], rate[i], rate[i + 1]
        off = 0.5 * (a - c) / (a - 2 * b + c)
    else:
        off = 0.0
    return (i + 0.5 + off) * dt


@pytest.mark.slow
def test_P11_ignition_delay_converges(h2_oracle, h2_mech):
    T0 = 1000.0
    dts = [4e-6, 2e-6, 1e-6]
    idts = [_idt(h2_oracle, T0, dt, 1.2e-3, h2_mech) for dt in dts]
    d1 = abs(idts[0] - idts[1])
    d2 = abs(idts[1] - idts[2])
    assert d2 < d1
    assert d2 < 1e-3 * idts[2]
