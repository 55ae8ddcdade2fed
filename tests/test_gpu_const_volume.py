"""GPU checks of the constant-volume reactor (df_chem_step_const_volume) against the oracle's
constant-volume step: the parity bar of the constant-pressure integrator (1e-8 relative in T
and in Y_k > 1e-10 on cells with the oracle's accept/reject sequence), unusable input, a
ragged count with ld > n, and conservation of the mixture internal energy at full size."""
import numpy as np
import pytest

from synth import fields
from test_gpu_chem import compare

pytestmark = pytest.mark.gpu

R = 8.31446261815324


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _run(gm, f, rho, dt, ld=None):
    torch = _torch()
    n = f["T"].size
    K = f["Y"].shape[0]
    ld = ld or n
    d = "cuda:0"
    Yh = np.zeros((K, ld))
    Yh[:, :n] = f["Y"]
    T = torch.tensor(f["T"], dtype=torch.float64, device=d)
    Y = torch.tensor(Yh, dtype=torch.float64, device=d)
    r = torch.tensor(rho, dtype=torch.float64, device=d)
    st = torch.full((n,), -7, dtype=torch.int32, device=d)
    ns = torch.full((2 * n,), -7, dtype=torch.int32, device=d)
    gm.chem_step_const_volume(T, r, Y, dt, h=torch.zeros(n, dtype=torch.float64, device=d), status=st, n_steps=ns)
    torch.cuda.synchronize()
    return {"T": T.cpu().numpy(), "Y": Y.cpu().numpy()[:, :n], "status": st.cpu().numpy(),
            "n_acc": ns[:n].cpu().numpy(), "n_rej": ns[n:].cpu().numpy()}


def _rho(h2_oracle, f):
    return np.array([h2_oracle.mixture(f["T"][i], f["p"][i], f["Y"][:, i])[1] for i in range(f["T"].size)])


@pytest.mark.parametrize("dt", [1e-5, 2e-4])
def test_parity_with_oracle(h2_path, h2_mech, h2_oracle, dt):
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = fields.ignition_cells(h2_mech, n=1001, seed=41)
    rho = _rho(h2_oracle, f)
    g = _run(gm, f, rho, dt, ld=1100)
    o = h2_oracle.chem_step_v(f["T"], rho, f["Y"], dt, h_inout=np.zeros(1001))
    assert np.array_equal(g["status"], o["status"])
    worst, flipped, tol_err = compare(g, o)
    assert worst <= 1e-8, worst
    assert flipped <= 3 and tol_err <= 10.0, (flipped, tol_err)
    if dt > 1e-4:
        assert np.max(o["T"] - f["T"]) > 100.0   # cells ignite within the step


def test_unusable_input(h2_path, h2_mech, h2_oracle):
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = fields.ignition_cells(h2_mech, n=64, seed=2)
    rho = _rho(h2_oracle, f)
    rho[3], rho[4] = 0.0, np.nan
    f["T"][5] = -1.0
    g = _run(gm, f, rho, 1e-6)
    bad = [3, 4, 5]
    assert np.all(g["status"][bad] == df.CELL_NONFINITE)
    assert np.array_equal(g["Y"][:, bad], f["Y"][:, bad])
    assert np.all(np.delete(g["status"], bad) == df.CELL_OK)


def test_internal_energy_conserved_full_field(h2_path, h2_mech, h2_oracle, npchem):
    """The 65,536-cell hot-kernel field held at constant volume for 1e-5 s."""
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = fields.hot_kernel_field_2d(h2_mech)
    n = f["T"].size
    rho = np.empty(n)
    W = np.asarray(h2_mech.molar_mass) * 1e-3
    rho[:] = f["p"] / (R * f["T"] * np.sum(f["Y"] / W[:, None], axis=0))
    g = _run(gm, f, rho, 1e-5)
    assert np.all(g["status"] == df.CELL_OK)
    sample = np.concatenate([np.argsort(f["T"])[-200:], np.arange(0, n, 997)])
    for i in sample:
        u0 = npchem.u_mass(f["T"][i], f["Y"][:, i])
        u1 = npchem.u_mass(g["T"][i], g["Y"][:, i])
        cv = np.sum(g["Y"][:, i] * (npchem.cp_R(g["T"][i]) - 1.0) * R / npchem.W)
        assert abs(u1 - u0) <= 10 * 1e-8 * cv * g["T"][i]
    assert np.max(np.abs(g["Y"].sum(axis=0) - f["Y"].sum(axis=0))) < 1e-12
    # sampled parity with the oracle at full size
    o = h2_oracle.chem_step_v(f["T"][sample], rho[sample], f["Y"][:, sample], 1e-5, h_inout=np.zeros(sample.size))
    gs = {k: (v[:, sample] if v.ndim == 2 else v[sample]) for k, v in g.items()}
    worst, flipped, tol_err = compare(gs, o)
    assert worst <= 1e-8 and flipped <= 3 and tol_err <= 10.0


def test_parity_large_mechanism():
    """The 53-species mechanism at constant volume (one wavefront per cell): 48 cells of the
    hydrocarbon field spread over the temperature range, at the parity bar, and the mixture
    internal energy conserved on every cell."""
    import os
    import oracle
    import synth
    import paper_2210_07094_amd as df
    from npchem import NpChem
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(root, "synth", "data", "hc_synth_53sp_325r.mech")
    mech, om, gm = synth.read_mech(path), oracle.Mech(path), df.Mechanism(path)
    npc = NpChem(mech)
    g = fields.hydrocarbon_field(mech, n=512)
    idx = np.argsort(g["T"])[np.linspace(0, 511, 48).astype(int)]
    f = {"T": g["T"][idx].copy(), "p": g["p"][idx].copy(), "Y": np.ascontiguousarray(g["Y"][:, idx])}
    W = np.asarray(mech.molar_mass) * 1e-3
    rho = f["p"] / (R * f["T"] * np.sum(f["Y"] / W[:, None], axis=0))
    out = _run(gm, f, rho, 1e-6, ld=50)
    o = om.chem_step_v(f["T"], rho, f["Y"], 1e-6, h_inout=np.zeros(48), nthreads=16)
    assert np.all(o["status"] == 0) and np.array_equal(out["status"], o["status"])
    worst, flipped, tol_err = compare(out, o)
    assert worst <= 1e-8 and flipped <= 3 and tol_err <= 10.0, (worst, flipped, tol_err)
    for i in range(48):
        u0 = npc.u_mass(f["T"][i], f["Y"][:, i])
        u1 = npc.u_mass(out["T"][i], out["Y"][:, i])
        cv = np.sum(out["Y"][:, i] * (npc.cp_R(out["T"][i]) - 1.0) * R / npc.W)
        assert abs(u1 - u0) <= 10 * 1e-8 * cv * out["T"][i]
