"""Pins of the oracle's forward sensitivities of the chemistry step (oracle/sensitivity.py).

The sensitivities d y(dt) / d(T0, Y0, ln A) of the integration with its accepted sub-step
lengths frozen are checked against what holds independently of that code:
  * its right-hand side and dual-number Jacobian against the C oracle's own (separately
    written, analytic) f and J;
  * the C oracle's record of a cell's accepted sub-steps, replayed, reproducing that cell's
    integration exactly;
  * central finite differences (relative step 1e-6) of the C oracle's replay;
  * invariants of the exact step: every sub-step conserves total mass (sum of Y) and each
    element, for every input, so the sensitivities of those sums are known exactly;
  * a single short sub-step of length h, whose derivative is I + h J (and h df/dlnA) up to
    O(h^2): the error must fall fourfold when h is halved.
"""
import numpy as np
import pytest

import oracle
from oracle import sensitivity as sens
from synth import fields

DT = 1e-5


@pytest.fixture(scope="module")
def kin(h2_mech):
    return sens.Kinetics(h2_mech)


@pytest.fixture(scope="module")
def tab():
    return oracle.rodas4_tableau()


def _cell(h2_mech, i, n=8, seed=4):
    f = fields.ignition_cells(h2_mech, n=n, seed=seed)
    return f["T"][i], f["p"][i], f["Y"][:, i].copy()


def test_rhs_and_jacobian_match_c_oracle(h2_mech, h2_oracle, kin):
    rng = np.random.default_rng(7)
    f = fields.ignition_cells(h2_mech, n=6, seed=11)
    for i in range(6):
        Y = f["Y"][:, i] + rng.uniform(0, 1e-3, size=h2_mech.n_species)   # radicals present too
        y = np.concatenate([[f["T"][i] + rng.uniform(-200, 400)], Y / Y.sum()])
        p = f["p"][i]
        fc = h2_oracle.rhs(p, y)
        fn = kin.rhs(y[None], p)[0]
        assert np.max(np.abs(fn - fc)) <= 1e-12 * np.max(np.abs(fc))
        Jc = h2_oracle.jacobian(p, y)
        Jn = kin.jacobian(y[None], p)[0]
        assert np.max(np.abs(Jn - Jc)) <= 1e-11 * np.max(np.abs(Jc))


def test_record_replay_reproduces_the_integration(h2_mech, h2_oracle):
    T, p, Y = _cell(h2_mech, 0)
    Te, Ye, st, hs, _ = h2_oracle.record(T, p, Y, DT)
    assert st == 0 and hs.size > 10
    assert abs(hs.sum() - DT) <= 1e-12 * DT
    o = h2_oracle.chem_step(np.array([T]), np.array([p]), Y[:, None], DT, h_inout=np.zeros(1))
    assert o["T"][0] == Te and np.array_equal(o["Y"][:, 0], Ye)
    y0 = np.concatenate([[T], Y])
    assert np.array_equal(h2_oracle.replay(p, y0, hs), np.concatenate([[Te], Ye]))
    assert np.array_equal(h2_oracle.replay(p, y0, hs[:0]), y0)


def _fd(om, p, y, hs, M):
    N = y.size
    S = np.zeros((N, N + M))
    for c in range(N):
        d = 1e-6 * max(abs(y[c]), 1e-3 if c else 1.0)
        yp, ym = y.copy(), y.copy()
        yp[c] += d
        ym[c] -= d
        S[:, c] = (om.replay(p, yp, hs) - om.replay(p, ym, hs)) / (2 * d)
    for j in range(M):
        d = 1e-6
        om.scale_A(j, np.exp(d))
        a = om.replay(p, y, hs)
        om.scale_A(j, np.exp(-2 * d))
        b = om.replay(p, y, hs)
        om.scale_A(j, np.exp(d))
        S[:, N + j] = (a - b) / (2 * d)
    return S


@pytest.mark.parametrize("i", [1, 5])
def test_sensitivities_match_central_differences(h2_mech, h2_path, kin, tab, i):
    om = oracle.Mech(h2_path)   # a private handle: the FD loop scales A in place
    T, p, Y = _cell(h2_mech, i)
    _, _, st, hs, _ = om.record(T, p, Y, DT)
    assert st == 0
    y0 = np.concatenate([[T], Y])
    ye, S = sens.sensitivities(kin, tab, p, y0, hs)
    assert np.max(np.abs(ye - om.replay(p, y0, hs)) / (np.abs(ye) + 1e-12)) < 1e-11
    Sfd = _fd(om, p, y0, hs, kin.M)
    row = np.abs(S).max(axis=1, keepdims=True)
    err = np.abs(S - Sfd) / row
    assert np.max(err) < 1e-5, np.max(err)
    assert np.median(err) < 1e-9, np.median(err)


def test_sensitivities_respect_conservation(h2_mech, h2_oracle, kin, tab):
    T, p, Y = _cell(h2_mech, 2)
    _, _, st, hs, _ = h2_oracle.record(T, p, Y, DT)
    y0 = np.concatenate([[T], Y])
    _, S = sens.sensitivities(kin, tab, p, y0, hs)
    N = kin.N
    K = N - 1
    # sum_k Y_k(dt) = sum_k Y0_k for every input
    assert np.max(np.abs(S[1:, 1:N].sum(axis=0) - 1.0)) < 1e-12
    assert abs(S[1:, 0].sum()) < 1e-12 * np.abs(S[1:, 0]).max()
    assert np.max(np.abs(S[1:, N:].sum(axis=0))) < 1e-12 * np.abs(S[1:, N:]).max()
    # element mass fractions: sum_k a_ek / W_k Y_k is conserved
    E = np.asarray(h2_mech.composition, dtype=float).T / np.asarray(h2_mech.molar_mass)   # [E, K]
    got = E @ S[1:, :]
    want = np.zeros_like(got)
    want[:, 1:N] = E
    assert np.max(np.abs(got - want)) < 1e-12 * np.abs(E).max()
    assert K == E.shape[1]


def test_one_short_substep_is_explicit_euler_to_second_order(h2_mech, h2_path, kin, tab):
    om = oracle.Mech(h2_path)
    T, p, Y = _cell(h2_mech, 3)
    Y = Y + 1e-4
    Y /= Y.sum()
    y0 = np.concatenate([[T], Y])
    N, M = kin.N, kin.M
    J = om.jacobian(p, y0)
    # df/dlnA_j from the C oracle's progress rates: f_k = W_k wdot_k / rho, f_T = -sum h_k wdot_k/(rho cp),
    # with d q_j / d lnA_j = q_j d ln kf_j / d ln A_j (kr = kf / Kc scales with kf); the last factor is 1
    # for Arrhenius rows and is taken by a central difference of the oracle's kf for falloff rows
    _, rho, cp, _ = om.mixture(T, p, Y)
    kf, _, q, _ = om.rates(T, p, Y)
    dlnkf = np.ones(M)
    for j in range(M):
        om.scale_A(j, np.exp(1e-6))
        a = om.rates(T, p, Y)[0][j]
        om.scale_A(j, np.exp(-2e-6))
        b = om.rates(T, p, Y)[0][j]
        om.scale_A(j, np.exp(1e-6))
        dlnkf[j] = (np.log(a) - np.log(b)) / 2e-6
    assert np.allclose(dlnkf[np.asarray(h2_mech.reaction_type) != 2], 1.0, atol=1e-8)
    _, hRT, _, _ = om.thermo(T)
    nu = (np.asarray(h2_mech.nu_prod) - np.asarray(h2_mech.nu_reac)).astype(float)   # [M, K]
    W = np.asarray(h2_mech.molar_mass) * 1e-3
    dw = 1e6 * nu * (q * dlnkf)[:, None]                # d wdot / d lnA_j, [M, K]
    dfY = dw * W / rho
    dfT = -(dw * hRT * 8.31446261815324 * T).sum(axis=1) / (rho * cp)
    fth = np.concatenate([dfT[None, :], dfY.T], axis=0)  # [N, M]
    h0 = 1e-3 / np.max(np.abs(J))
    errs = []
    for h in (h0, h0 / 2):
        _, S = sens.sensitivities(kin, tab, p, y0, [h])
        ref = np.concatenate([np.eye(N) + h * J, h * fth], axis=1)
        errs.append(np.max(np.abs(S - ref) / np.maximum(np.abs(ref).max(axis=0), 1.0)))
    assert errs[0] < 1e-4, errs
    assert 3.0 < errs[0] / errs[1] < 5.0, errs
