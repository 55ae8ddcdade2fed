"""Pins of the oracle on the synthetic 53-species hydrocarbon mechanism (the size class of the
paper's complex-fuel outlook) and of the mechanism generator.

The oracle's C code is generic in the species count and is pinned in detail on the hydrogen
mechanism and the closed-form mechanisms; here it is checked at K = 53 against what holds
independently of it:
  * its right-hand side against the vectorised NumPy kinetics of oracle/sensitivity.py
    (written separately) and against tests/npchem.py, and its analytic Jacobian against the
    exact dual-number derivative of that NumPy right-hand side;
  * invariants of a step: total mass, every element's mass and, at constant pressure, the
    mixture enthalpy are conserved;
  * the generator's own rules: element balance, every reactive species in some reaction,
    exchanges in the direction of negative Gibbs energy at 1000 K, one <-> two reactions in
    the direction of negative enthalpy at 298.15 K, the stored file equal to the generator's
    output for the accepted seed.
"""
import os

import numpy as np
import pytest

import synth
from oracle import sensitivity as sens
from synth import fields
from synth.mechgen_large import generate_large_mechanism, DEFAULT_LARGE_SEED

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC_MECH = os.path.join(ROOT, "synth", "data", "hc_synth_53sp_325r.mech")
R = 8.31446261815324


@pytest.fixture(scope="module")
def hc_mech():
    return synth.read_mech(HC_MECH)


@pytest.fixture(scope="module")
def hc_oracle():
    import oracle
    return oracle.Mech(HC_MECH)


def _states(mech, n=4, seed=7):
    f = fields.hydrocarbon_field(mech, n=64)
    rng = np.random.default_rng(seed)
    idx = np.argsort(f["T"])[np.linspace(8, 63, n).astype(int)]
    out = []
    for i in idx:
        Y = f["Y"][:, i] + rng.uniform(0, 1e-4, mech.n_species)
        out.append((f["p"][i], np.concatenate([[f["T"][i]], Y / Y.sum()])))
    return out


def test_generator_rules(hc_mech):
    m = generate_large_mechanism(DEFAULT_LARGE_SEED)
    assert m.n_species == 53 and m.n_reactions == 325 and len(m.elements) == 5
    assert np.bincount(np.asarray(m.reaction_type)).tolist() == [270, 25, 30]
    nu = np.asarray(m.nu_prod) - np.asarray(m.nu_reac)
    assert np.all(nu @ np.asarray(m.composition) == 0)
    used = np.any(np.asarray(m.nu_reac) + np.asarray(m.nu_prod) > 0, axis=0)
    assert used.sum() == 52 and not used[m.index("AR")]
    a = np.asarray(m.nasa7)
    h298 = sum(a[:, i] * 298.15 ** (i + 1) / (i + 1) for i in range(5)) + a[:, 5]
    T1 = 1000.0
    g1 = (sum(a[:, i] * T1 ** i / (i + 1) for i in range(5)) + a[:, 5] / T1
          - (a[:, 0] * np.log(T1) + sum(a[:, i] * T1 ** i / i for i in range(1, 5)) + a[:, 6]))
    t = np.asarray(m.reaction_type)
    assert np.all(nu[t == 0] @ g1 <= 0.0)
    assert np.all(nu[t != 0] @ h298 < 0.0)
    # the file is the generator's output
    assert np.allclose(np.asarray(hc_mech.arrhenius), np.asarray(m.arrhenius), rtol=1e-15)
    assert np.array_equal(np.asarray(hc_mech.nu_reac), np.asarray(m.nu_reac))
    assert np.allclose(np.asarray(hc_mech.nasa7), np.asarray(m.nasa7), rtol=1e-15, atol=0)


def test_rhs_and_jacobian_against_numpy(hc_mech, hc_oracle, npchem_hc):
    kin = sens.Kinetics(hc_mech)
    for p, y in _states(hc_mech):
        fc = hc_oracle.rhs(p, y)
        fn = kin.rhs(y[None], p)[0]
        assert np.max(np.abs(fn - fc)) <= 1e-11 * np.max(np.abs(fc))
        assert np.max(np.abs(npchem_hc.rhs(p, y) - fc)) <= 1e-11 * np.max(np.abs(fc))
        Jc = hc_oracle.jacobian(p, y)
        Jn = kin.jacobian(y[None], p)[0]
        scale = np.maximum(np.abs(Jn).max(axis=1, keepdims=True), 1e-300)   # the inert AR row is zero
        assert np.max(np.abs(Jn - Jc) / scale) < 1e-10


@pytest.fixture(scope="module")
def npchem_hc(hc_mech):
    from npchem import NpChem
    return NpChem(hc_mech)


def test_step_conserves_mass_elements_and_enthalpy(hc_mech, hc_oracle, npchem_hc):
    f = fields.hydrocarbon_field(hc_mech, n=64)
    idx = np.argsort(f["T"])[[5, 30, 50, 60]]
    T, p, Y = f["T"][idx], f["p"][idx], np.ascontiguousarray(f["Y"][:, idx])
    r = hc_oracle.chem_step(T, p, Y, 1e-6, h_inout=np.zeros(idx.size))
    assert np.all(r["status"] == 0)
    assert np.max(np.abs(r["Y"].sum(axis=0) - Y.sum(axis=0))) < 1e-13
    E = np.asarray(hc_mech.composition, dtype=float).T / np.asarray(hc_mech.molar_mass)
    assert np.max(np.abs(E @ r["Y"] - E @ Y)) < 1e-13 * np.abs(E @ Y).max()
    for i in range(idx.size):
        h0 = npchem_hc.h_mass(T[i], Y[:, i])
        h1 = npchem_hc.h_mass(r["T"][i], r["Y"][:, i])
        cp = npchem_hc.cp_mass(r["T"][i], r["Y"][:, i])
        assert abs(h1 - h0) <= 10 * 1e-8 * cp * r["T"][i]
    assert np.any(np.abs(r["T"] - T) > 1e-3)   # the step does something
