"""Seeded inputs: mechanism catalogue, file format and fields."""
import os

import numpy as np

import synth
from synth import fields
from synth.mechgen import H2_COMPOSITION, H2_SPECIES, reaction_catalogue


def test_catalogue_size():
    comp = np.array([H2_COMPOSITION[s] for s in H2_SPECIES])
    exch, recomb = reaction_catalogue(H2_SPECIES, comp, H2_SPECIES[:8])
    assert len(exch) == 19 and len(recomb) == 11


def test_h2_mechanism_shape_and_balance(h2_mech):
    m = h2_mech
    assert m.n_species == 9 and m.n_elements == 3 and m.n_reactions == 24
    assert np.count_nonzero(m.reaction_type == 1) == 4
    assert np.count_nonzero(m.reaction_type == 2) == 2
    # element balance of every reaction
    assert np.all((m.nu_prod - m.nu_reac) @ m.composition == 0)
    # N2 is inert
    iN2 = m.index("N2")
    assert np.all(m.nu_reac[:, iN2] == 0) and np.all(m.nu_prod[:, iN2] == 0)
    # parameter ranges of the recipe
    A, b, Ta = m.arrhenius.T
    assert np.all((A >= 1e6) & (A <= 1e16)) and np.all(np.abs(b) <= 2) and np.all((Ta >= 0) & (Ta <= 25000))
    # molar masses follow from composition
    np.testing.assert_allclose(m.molar_mass, m.composition @ m.element_mass, rtol=1e-15)


def test_reactions_written_exothermic(h2_mech, h2_oracle):
    m = h2_mech
    _, h_RT, _, _ = h2_oracle.thermo(298.15)
    dh = (m.nu_prod - m.nu_reac) @ h_RT
    assert np.all(dh <= 0)


def test_committed_file_is_reproducible(tmp_path, h2_path):
    m = synth.generate_h2_mechanism()
    p = tmp_path / "m.mech"
    synth.write_mech(p, m)
    a = synth.read_mech(p)
    b = synth.read_mech(h2_path)
    for key in ("nasa7", "arrhenius", "efficiency", "falloff_low", "troe", "nu_reac", "nu_prod", "reaction_type"):
        np.testing.assert_array_equal(getattr(a, key), getattr(b, key))
    assert a.species == b.species and a.seed == b.seed


def test_file_roundtrip_exact(tmp_path, h2_mech):
    p = tmp_path / "rt.mech"
    synth.write_mech(p, h2_mech)
    m2 = synth.read_mech(p)
    np.testing.assert_array_equal(m2.nasa7, h2_mech.nasa7)
    np.testing.assert_array_equal(m2.arrhenius, h2_mech.arrhenius)


def test_h2_air_composition_at_phi_1(h2_mech):
    # stoichiometric H2/air with O2:N2 = 1:3.76 by moles and real atomic masses
    Y = fields.premixed_h2_air(h2_mech, 1.0)[:, 0]
    assert abs(Y[h2_mech.index("H2")] - 0.02852) < 5e-5
    assert abs(Y[h2_mech.index("O2")] - 0.22635) < 5e-5
    assert abs(Y[h2_mech.index("N2")] - 0.74512) < 5e-5
    assert abs(Y.sum() - 1) < 1e-15


def test_fields_shapes(h2_mech):
    f1 = fields.ignition_cells(h2_mech)
    assert f1["T"].shape == (1024,) and f1["Y"].shape == (9, 1024)
    assert f1["T"].min() >= 1000 and f1["T"].max() <= 1600
    f2 = fields.hot_kernel_field_2d(h2_mech)
    assert f2["T"].shape == (65536,) and f2["T"].max() <= 1800.0 and f2["T"].min() >= 300.0
    np.testing.assert_allclose(f2["Y"].sum(axis=0), 1.0, rtol=1e-14)
