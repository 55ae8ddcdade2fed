"""GPU parity of the DNN chemistry step at the size of the 53-species hydrocarbon mechanism:
a 55-3200-1600-800-53 BF16 network (seeded weights; no trained network exists for this
mechanism) against the oracle's BF16-emulated network, at the bar of the hydrogen network's
test: per output feature in z = BoxCox(Y) space with renormalisation off, max |du| <= 2^-8
max|u|, 99th percentile <= 1e-3 max|u|, median <= 1e-5 max|u|; T' within the bound implied
by the difference in Y'.  Also: cells outside the training box go to the one-wavefront-per-cell
integrator and match the oracle's integrator."""
import os

import numpy as np
import pytest

import oracle
import synth
from synth import dnnfile, fields

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC_MECH = os.path.join(ROOT, "synth", "data", "hc_synth_53sp_325r.mech")
LAM = 0.1
R = 8.31446261815324


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def hc():
    import paper_2210_07094_amd as df
    _torch()
    return synth.read_mech(HC_MECH), oracle.Mech(HC_MECH), df.Mechanism(HC_MECH)


def _step(dnn, f, renormalise=0, fallback=1):
    import paper_2210_07094_amd as df
    torch = _torch()
    d = "cuda:0"
    T = torch.tensor(f["T"], device=d)
    p = torch.tensor(f["p"], device=d)
    Y = torch.tensor(np.ascontiguousarray(f["Y"]), device=d)
    st = torch.full((f["T"].size,), -7, dtype=torch.int32, device=d)
    dnn.step(T, p, Y, 1e-6, status=st, opts=df.dnn_opts(renormalise=renormalise, fallback=fallback))
    torch.cuda.synchronize()
    return {"T": T.cpu().numpy(), "Y": Y.cpu().numpy(), "status": st.cpu().numpy()}


def _bct(Y):
    return (np.maximum(Y, 0.0) ** LAM - 1.0) / LAM


def test_large_network_parity(tmp_path, hc):
    import paper_2210_07094_amd as df
    mech, om, gm = hc
    f = fields.hydrocarbon_field(mech, n=1024)
    path = tmp_path / "hc.dfdnn"
    dnnfile.write_seeded_network(path, mech.n_species, f["T"], f["p"], f["Y"], (3200, 1600, 800), seed=3)
    print("case: seeded 55-3200-1600-800-53 network, 1024 hydrocarbon cells", flush=True)
    g = _step(df.DNN(path, gm), f)
    o = oracle.DNN(path).step(om, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=1)
    assert np.all(g["status"] == 0) and np.all(o["status"] == 0)
    z0, zo, zg = _bct(f["Y"]), _bct(o["Y"]), _bct(g["Y"])
    ok = o["Y"] > 0
    u_o = np.where(ok, (zo - z0) / 0.02, 0.0)
    du = np.where(ok, np.abs(zg - zo) / 0.02, 0.0)
    umax = np.abs(u_o).max(axis=1)
    print("max |du| / max|u| per output (largest 5):", np.sort(du.max(axis=1) / umax)[-5:])
    assert np.all(du.max(axis=1) <= 2.0 ** -8 * umax)
    assert np.all(np.percentile(du, 99, axis=1) <= 1e-3 * umax)
    assert np.all(np.median(du, axis=1) <= 1e-5 * umax)
    W = np.asarray(mech.molar_mass) * 1e-3
    for i in range(0, 1024, 7):
        _, hRT, _, _ = om.thermo(o["T"][i])
        _, _, cp, _ = om.mixture(o["T"][i], f["p"][i], o["Y"][:, i])
        bound = np.sum(np.abs(hRT * R * o["T"][i] / W) * np.abs(g["Y"][:, i] - o["Y"][:, i])) / cp
        assert abs(g["T"][i] - o["T"][i]) <= 2 * bound + 1e-8


def test_large_network_fallback(tmp_path, hc):
    """Cells outside the training box are integrated by the one-wavefront-per-cell kernel."""
    import paper_2210_07094_amd as df
    mech, om, gm = hc
    f = fields.hydrocarbon_field(mech, n=256)
    idx = np.argsort(f["T"])
    cold, rest = idx[:32], idx[32:]
    # a box fitted to the field shifted 2000 K up leaves the colder cells (the 32 coldest among them) outside
    path = tmp_path / "hc_box.dfdnn"
    dnnfile.write_seeded_network(path, mech.n_species, f["T"][rest] + 2000.0, f["p"][rest], f["Y"][:, rest],
                                 (3200, 1600, 800), seed=4)
    g = _step(df.DNN(path, gm), f, renormalise=1)
    fb = g["status"] == df.CELL_DNN_FALLBACK
    assert np.all(fb[cold]) and np.all(g["status"][~fb] == df.CELL_OK)
    s = {"T": f["T"][fb], "p": f["p"][fb], "Y": np.ascontiguousarray(f["Y"][:, fb])}
    o = om.chem_step(s["T"], s["p"], s["Y"], 1e-6, nthreads=16)
    mask = o["Y"] > 1e-10
    assert np.max(np.abs(g["T"][fb] - o["T"]) / o["T"]) < 1e-7
    assert np.max(np.abs(g["Y"][:, fb] - o["Y"])[mask] / o["Y"][mask]) < 1e-6
