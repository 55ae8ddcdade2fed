"""GPU parity of the one-wavefront-per-cell integrator (df_chem_step with mapping 3, and the
automatic choice for the 53-species hydrocarbon mechanism) against the CPU oracle, at the bar of
the other integrator kernels: max relative difference <= 1e-8 in T and in Y_k > 1e-10 on cells
with the oracle's accept/reject sequence, rare flipped cells within 10 tolerance units.

Cases: the hydrogen mechanism's 1001 ignition cells through the wave kernel (ragged: ld > n);
cells of the hydrocarbon field stratified by temperature; the full 262,144-cell field
(conservation on every cell, sampled oracle parity); per-cell step lengths; the cost-ordered
launch; unusable input and an empty call."""
import os

import numpy as np
import pytest

import synth
from synth import fields
from test_gpu_chem import _gpu_step, compare

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC_MECH = os.path.join(ROOT, "synth", "data", "hc_synth_53sp_325r.mech")
R = 8.31446261815324


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def hc():
    import oracle
    import paper_2210_07094_amd as df
    return synth.read_mech(HC_MECH), oracle.Mech(HC_MECH), df.Mechanism(HC_MECH)


def _subset(f, idx):
    return {"T": f["T"][idx].copy(), "p": f["p"][idx].copy(), "Y": np.ascontiguousarray(f["Y"][:, idx])}


def test_wave_kernel_hydrogen_parity(h2_path, h2_mech, h2_oracle):
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = fields.ignition_cells(h2_mech, n=1001, seed=41)
    g = _gpu_step(gm, f, 1e-5, h=np.zeros(1001), rr=True, ld=1100, opts=df.chem_opts(mapping=3))
    o = h2_oracle.chem_step(f["T"], f["p"], f["Y"], 1e-5, h_inout=np.zeros(1001), want_rr=True)
    assert np.array_equal(g["status"], o["status"])
    worst, flipped, tol_err = compare(g, o)
    assert worst <= 1e-8, worst
    assert flipped <= 3 and tol_err <= 10.0, (flipped, tol_err)
    same = (g["n_acc"] == o["n_acc"]) & (g["n_rej"] == o["n_rej"])
    scale = np.abs(o["rr"]).max()
    assert np.max(np.abs(g["rr"] - o["rr"])[:, same]) <= 1e-8 * scale
    assert np.all(g["Y_full"][:, 1001:] == 0.0)     # the padding columns are untouched


def test_wave_kernel_hydrocarbon_parity(hc):
    mech, om, gm = hc
    f = fields.hydrocarbon_field(mech, n=4096)
    idx = np.argsort(f["T"])[np.linspace(0, 4095, 96).astype(int)]
    s = _subset(f, idx)
    g = _gpu_step(gm, s, 1e-6, h=np.zeros(96), ld=100)
    o = om.chem_step(s["T"], s["p"], s["Y"], 1e-6, h_inout=np.zeros(96), nthreads=16)
    assert np.all(o["status"] == 0) and np.array_equal(g["status"], o["status"])
    worst, flipped, tol_err = compare(g, o)
    print(f"hydrocarbon: worst {worst:.3e}, flipped {flipped}, tol_err {tol_err:.3f}, "
          f"sub-steps mean {o['n_acc'].mean():.0f} max {o['n_acc'].max()}")
    assert worst <= 1e-8, worst
    assert flipped <= 5 and tol_err <= 10.0, (flipped, tol_err)
    assert np.max(np.abs(g["h"] - o["h"]) / o["h"]) < 1e-6 or flipped > 0


def test_wave_kernel_full_field(hc, npchem_factory):
    """The benchmark's 262,144-cell field: every cell OK, mass and enthalpy conserved, the oracle
    matched on a sample (the 8 hottest cells and 16 spread over the field)."""
    mech, om, gm = hc
    npc = npchem_factory(mech)
    f = fields.hydrocarbon_field(mech)
    n = f["T"].size
    g = _gpu_step(gm, f, 1e-6, h=np.zeros(n))
    assert np.all(g["status"] == 0), np.bincount(g["status"])
    assert np.max(np.abs(g["Y"].sum(axis=0) - f["Y"].sum(axis=0))) < 1e-12
    rng = np.random.default_rng(5)
    for i in rng.choice(n, 200, replace=False):
        h0 = npc.h_mass(f["T"][i], f["Y"][:, i])
        h1 = npc.h_mass(g["T"][i], g["Y"][:, i])
        assert abs(h1 - h0) <= 10 * 1e-8 * npc.cp_mass(g["T"][i], g["Y"][:, i]) * g["T"][i]
    sample = np.concatenate([np.argsort(f["T"])[-8:], np.arange(0, n, n // 16)])
    s = _subset(f, sample)
    o = om.chem_step(s["T"], s["p"], s["Y"], 1e-6, h_inout=np.zeros(sample.size), nthreads=16)
    gs = {k: (v[:, sample] if v.ndim == 2 and k != "Y_full" else v[sample]) for k, v in g.items() if k != "Y_full"}
    worst, flipped, tol_err = compare(gs, o)
    assert worst <= 1e-8 and flipped <= 3 and tol_err <= 10.0, (worst, flipped, tol_err)


@pytest.fixture(scope="module")
def npchem_factory():
    from npchem import NpChem
    return NpChem


def test_wave_kernel_per_cell_dt_and_ordering(hc):
    torch = _torch()
    import paper_2210_07094_amd as df
    mech, om, gm = hc
    f = fields.hydrocarbon_field(mech, n=512)
    idx = np.argsort(f["T"])[::8]
    s = _subset(f, idx)
    n = idx.size
    dts = np.random.default_rng(9).uniform(1e-7, 2e-6, n)
    g = _gpu_step(gm, s, torch.tensor(dts, device="cuda:0"), h=np.zeros(n))
    o = om.chem_step(s["T"], s["p"], s["Y"], dts, h_inout=np.zeros(n), nthreads=16)
    worst, flipped, tol_err = compare(g, o)
    assert worst <= 1e-8 and flipped <= 3 and tol_err <= 10.0, (worst, flipped, tol_err)
    # the cost-ordered launch (workspace) integrates the same cells to the same bits
    g1 = _gpu_step(gm, s, 1e-6, h=np.zeros(n))
    g2 = _gpu_step(gm, s, 1e-6, h=np.zeros(n), ordered=True)
    assert np.array_equal(g1["T"], g2["T"]) and np.array_equal(g1["Y"], g2["Y"])
    assert np.array_equal(g1["n_acc"], g2["n_acc"])
    # mapping 3 is the automatic choice for this mechanism
    g3 = _gpu_step(gm, s, 1e-6, h=np.zeros(n), opts=df.chem_opts(mapping=3))
    assert np.array_equal(g1["T"], g3["T"]) and np.array_equal(g1["Y"], g3["Y"])


def test_wave_kernel_edges(hc):
    torch = _torch()
    import paper_2210_07094_amd as df
    mech, om, gm = hc
    f = fields.hydrocarbon_field(mech, n=64)
    s = _subset(f, np.arange(64))
    s["p"][3] = 0.0
    s["T"][4] = np.nan
    s["Y"][7, 5] = np.inf
    g = _gpu_step(gm, s, 1e-7, rr=True)
    bad = [3, 4, 5]
    assert np.all(g["status"][bad] == df.CELL_NONFINITE)
    assert np.all(g["rr"][:, bad] == 0.0) and np.all(g["n_acc"][bad] == 0)
    assert np.all(np.delete(g["status"], bad) == df.CELL_OK)
    e = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    gm.chem_step(e, e, torch.zeros(mech.n_species, 0, dtype=torch.float64, device="cuda:0"), 1e-6)
    # the queue schedule has no kernel for this mechanism and needs a workspace anyway
    with pytest.raises(df.DfError):
        gm.chem_step(e, e, torch.zeros(mech.n_species, 0, dtype=torch.float64, device="cuda:0"), 1e-6,
                     opts=df.chem_opts(schedule=2))
