"""GPU checks of the 0-D rollouts (df_rollout): the integrator's trajectories and ignition
delays against the oracle's rollout, and the DNN rollout against repeated df_dnn_step calls
and the ignition-delay definition applied to its own trajectory.  How far the DNN's delays
lie from the integrator's depends on the fitted weights, not on this code: the benchmark
reports it."""
import os

import numpy as np
import pytest

import oracle
from oracle import rollout as ro
from synth import fields

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DNN = os.path.join(ROOT, "paper_2210_07094_amd", "data", "h2_dnn_1600_800_400.dfdnn")
DT = 1e-6


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _cells(mech, n=48):
    """Premixed H2/air at phi 0.7, 1, 1.5, T0 from 1000 to 1300 K, 1 atm."""
    phis = [0.7, 1.0, 1.5]
    T = np.tile(np.linspace(1000.0, 1300.0, n // 3), 3)
    Y = np.concatenate([np.repeat(fields.premixed_h2_air(mech, ph).reshape(-1, 1), n // 3, axis=1) for ph in phis],
                       axis=1)
    return T, np.full(n, 101325.0), np.ascontiguousarray(Y)


def test_integrator_rollout_matches_oracle(h2_path, h2_mech, h2_oracle):
    import paper_2210_07094_amd as df
    torch = _torch()
    gm = df.Mechanism(h2_path)
    T0, p, Y0 = _cells(h2_mech)
    d = "cuda:0"
    T = torch.tensor(T0, device=d)
    Y = torch.tensor(Y0, device=d)
    steps = 700
    idt, traj = gm.rollout(T, torch.tensor(p, device=d), Y, DT, steps, trajectory=True)
    traj_o, Y_o, idt_o = ro.integrator_rollout(h2_oracle, T0, p, Y0, DT, steps)
    tg = traj.cpu().numpy()
    assert tg.shape == (steps + 1, T0.size)
    assert np.max(np.abs(tg - traj_o) / traj_o) < 1e-7
    ig = idt.cpu().numpy()
    fin = np.isfinite(idt_o)
    assert fin.sum() >= T0.size // 2
    assert np.array_equal(np.isfinite(ig), fin)
    assert np.max(np.abs(ig[fin] - idt_o[fin]) / idt_o[fin]) < 1e-6
    # the device's delay is the definition applied to its own trajectory
    assert np.allclose(ig[fin], ro.ignition_delay(tg, DT)[fin], rtol=1e-12, atol=0)


def test_constant_volume_rollout_matches_oracle(h2_path, h2_mech, h2_oracle, npchem):
    """The constant-volume integrator rollout: the paper's case (phi = 1, 1000 K, 0.5 atm) and the
    48 premixed cells at their 1 atm densities."""
    import paper_2210_07094_amd as df
    torch = _torch()
    gm = df.Mechanism(h2_path)
    R = 8.31446261815324
    T0, p0, Y0 = _cells(h2_mech)
    T0 = np.concatenate([[1000.0], T0])
    p0 = np.concatenate([[0.5 * 101325.0], p0])
    Y0 = np.ascontiguousarray(np.concatenate([fields.premixed_h2_air(h2_mech, 1.0).reshape(-1, 1), Y0], axis=1))
    rho = p0 / (R * T0 * np.sum(Y0 / npchem.W[:, None], axis=0))
    d = "cuda:0"
    T, Y = torch.tensor(T0, device=d), torch.tensor(Y0, device=d)
    steps = 2500
    idt, traj = gm.rollout(T, torch.tensor(rho, device=d), Y, DT, steps, trajectory=True, constant_volume=True)
    traj_o, Y_o, idt_o = ro.integrator_rollout(h2_oracle, T0, rho, Y0, DT, steps, constant_volume=True)
    tg = traj.cpu().numpy()
    assert np.max(np.abs(tg - traj_o) / traj_o) < 1e-7
    mask = Y_o > 1e-10
    assert np.max(np.abs(Y.cpu().numpy() - Y_o)[mask] / Y_o[mask]) < 1e-6
    ig = idt.cpu().numpy()
    fin = np.isfinite(idt_o)
    assert fin[0] and fin.sum() >= T0.size // 2
    assert np.array_equal(np.isfinite(ig), fin)
    assert np.max(np.abs(ig[fin] - idt_o[fin]) / idt_o[fin]) < 1e-6
    with pytest.raises(df.DfError):
        gm.rollout(T, torch.tensor(rho, device=d), Y, DT, 2, dnn=df.DNN(DNN, gm), constant_volume=True)


def test_dnn_rollout(h2_path, h2_mech):
    import paper_2210_07094_amd as df
    torch = _torch()
    gm = df.Mechanism(h2_path)
    dnn = df.DNN(DNN, gm)
    T0, p0, Y0 = _cells(h2_mech)
    d = "cuda:0"
    p = torch.tensor(p0, device=d)
    T = torch.tensor(T0, device=d)
    Y = torch.tensor(Y0, device=d)
    steps = 700
    idt, traj = gm.rollout(T, p, Y, DT, steps, dnn=dnn, trajectory=True)
    # the same steps one call at a time
    T2, Y2 = torch.tensor(T0, device=d), torch.tensor(Y0, device=d)
    ws = dnn.workspace(T0.size)
    for _ in range(steps):
        dnn.step(T2, p, Y2, DT, workspace=ws)
    assert torch.equal(T, T2) and torch.equal(Y, Y2)
    tg = traj.cpu().numpy()
    ig = idt.cpu().numpy()
    ref = ro.ignition_delay(tg, DT)
    assert np.array_equal(np.isfinite(ig), np.isfinite(ref))
    fin = np.isfinite(ig)
    assert np.allclose(ig[fin], ref[fin], rtol=1e-12, atol=0)


def test_rollout_edges(h2_path, h2_mech):
    import paper_2210_07094_amd as df
    torch = _torch()
    gm = df.Mechanism(h2_path)
    T0, p0, Y0 = _cells(h2_mech, n=6)
    d = "cuda:0"
    T, Y, p = torch.tensor(T0, device=d), torch.tensor(Y0, device=d), torch.tensor(p0, device=d)
    idt, _ = gm.rollout(T, p, Y, DT, 1)
    assert torch.all(torch.isnan(idt))           # one step: the maximum is on an end step
    with pytest.raises(df.DfError):
        gm.rollout(T, p, Y, DT, 0)
    e = torch.zeros(0, dtype=torch.float64, device=d)
    idt0, _ = gm.rollout(e, e, torch.zeros(h2_mech.n_species, 0, dtype=torch.float64, device=d), DT, 5)
    assert idt0.numel() == 0


def test_rollout_large_mechanism():
    """df_rollout through the one-wavefront-per-cell integrator (53 species, sub-step hints carried
    from step to step) against the oracle's rollout: 6 hydrocarbon cells, 20 steps of 1 us."""
    import synth
    import paper_2210_07094_amd as df
    torch = _torch()
    path = os.path.join(ROOT, "synth", "data", "hc_synth_53sp_325r.mech")
    mech = synth.read_mech(path)
    om = oracle.Mech(path)
    gm = df.Mechanism(path)
    f = fields.hydrocarbon_field(mech, n=256)
    idx = np.argsort(f["T"])[np.linspace(0, 200, 6).astype(int)]
    T0, p0, Y0 = f["T"][idx], f["p"][idx], np.ascontiguousarray(f["Y"][:, idx])
    d = "cuda:0"
    T, Y = torch.tensor(T0, device=d), torch.tensor(Y0, device=d)
    steps = 20
    _, traj = gm.rollout(T, torch.tensor(p0, device=d), Y, DT, steps, trajectory=True)
    traj_o, Y_o, _ = ro.integrator_rollout(om, T0, p0, Y0, DT, steps, nthreads=6)
    assert np.max(np.abs(traj.cpu().numpy() - traj_o) / traj_o) < 1e-7
    mask = Y_o > 1e-10
    assert np.max(np.abs(Y.cpu().numpy() - Y_o)[mask] / Y_o[mask]) < 1e-6
