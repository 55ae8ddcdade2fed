"""GPU parity of the DNN chemistry step (df_dnn_step) against the oracle.

P13: the BF16 MFMA network against the oracle's BF16-emulated network
(bf16 inputs, weights and activations, fp32 accumulation).  The two sum the
fp32 products in different orders; most cells then agree exactly after the
bf16 rounding of each activation, but where an activation sits within an
fp32 rounding of a bf16 rounding boundary it lands one bf16 ulp (2^-8
relative) apart and the difference propagates to the output.  The bar, per
output feature over all cells: max |du| <= 2^-8 max|u| (one bf16 ulp of the
output scale), 99th percentile <= 1e-3 max|u|, median <= 1e-5 max|u|.  It is
checked in z = BoxCox(Y) space with renormalisation off, where
z' - z = u sig_out + mu_out exactly.
"""
import numpy as np
import pytest

import oracle
from synth import dnnfile, fields

pytestmark = pytest.mark.gpu

LAM = 0.1


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def bct(Y):
    return (np.maximum(Y, 0.0) ** LAM - 1.0) / LAM


def _net(path, K=9, hidden=(1600, 800, 400), seed=0, zero_out=False, box=None, scale=1.0):
    rng = np.random.default_rng(seed)
    dims = [K + 2, *hidden, K]
    W = [rng.normal(0, scale / np.sqrt(dims[l]), (dims[l + 1], dims[l])).astype(np.float32)
         for l in range(len(dims) - 1)]
    b = [rng.normal(0, 0.1, dims[l + 1]).astype(np.float32) for l in range(len(dims) - 1)]
    if zero_out:
        W[-1][:] = 0
        b[-1][:] = 0
    mu_in = np.concatenate([[1300.0, 101325.0], np.full(K, -5.0)])
    sig_in = np.concatenate([[300.0, 1.0], np.full(K, 3.0)])
    lo, hi = box if box is not None else (np.full(K + 2, -1e300), np.full(K + 2, 1e300))
    dnnfile.write_dnn(path, W, b, K, LAM, 1e-6, mu_in, sig_in, np.zeros(K), np.full(K, 0.02), lo, hi)


def _gpu_dnn(dnn, f, dt=1e-6, renormalise=1, fallback=1, ld=None, rr=False):
    import paper_2210_07094_amd as df
    torch = _torch()
    n = f["T"].size
    K = f["Y"].shape[0]
    ld = ld or n
    dev = "cuda:0"
    T = torch.tensor(f["T"], dtype=torch.float64, device=dev)
    p = torch.tensor(f["p"], dtype=torch.float64, device=dev)
    Yh = np.zeros((K, ld))
    Yh[:, :n] = f["Y"]
    Y = torch.tensor(Yh, dtype=torch.float64, device=dev)
    st = torch.full((n,), -7, dtype=torch.int32, device=dev)
    rrt = torch.zeros((K, ld), dtype=torch.float64, device=dev) if rr else None
    dnn.step(T, p, Y, dt, rr=rrt, status=st, opts=df.dnn_opts(renormalise=renormalise, fallback=fallback))
    torch.cuda.synchronize()
    out = {"T": T.cpu().numpy(), "Y": Y.cpu().numpy()[:, :n], "status": st.cpu().numpy(),
           "Y_full": Y.cpu().numpy()}
    if rr:
        out["rr"] = rrt.cpu().numpy()[:, :n]
    return out


@pytest.fixture(scope="module")
def gmech(h2_path):
    import paper_2210_07094_amd as df
    _torch()
    return df.Mechanism(h2_path)


def _cells(h2_mech, n, seed):
    """Ignition cells with some radicals present (all z finite and varied)."""
    f = fields.ignition_cells(h2_mech, n=n, seed=seed)
    rng = np.random.default_rng(seed)
    Y = f["Y"] + rng.uniform(0, 1, f["Y"].shape) ** 4 * 1e-3
    f["Y"] = Y / Y.sum(axis=0, keepdims=True)
    return f


@pytest.mark.parametrize("n", [1024, 1000])
def test_P13_network_parity(tmp_path, gmech, h2_oracle, h2_mech, n):
    import paper_2210_07094_amd as df
    path = tmp_path / "net.dfdnn"
    _net(path)
    d = df.DNN(path, gmech)
    od = oracle.DNN(path)
    f = _cells(h2_mech, n, seed=21 + n)
    print(f"case: random 11-1600-800-400-9 network, n={n}", flush=True)
    g = _gpu_dnn(d, f, renormalise=0)
    o = od.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=1)
    assert np.all(g["status"] == 0) and np.all(o["status"] == 0)
    z0 = bct(f["Y"])
    zo = bct(o["Y"])
    zg = bct(g["Y"])
    u_o = (zo - z0) / 0.02
    ok = o["Y"] > 0          # inverse transform not clamped
    du = np.where(ok, np.abs(zg - zo) / 0.02, 0.0)
    umax = np.abs(np.where(ok, u_o, 0.0)).max(axis=1)
    print("max |du| / max|u| per output:", du.max(axis=1) / umax)
    assert np.all(du.max(axis=1) <= 2.0 ** -8 * umax)
    assert np.all(np.percentile(du, 99, axis=1) <= 1e-3 * umax)
    assert np.all(np.median(du, axis=1) <= 1e-5 * umax)
    # T' follows from h(T', Y') = h0, so its difference is the one implied by the
    # difference in Y': |dT| <= sum_k |h_k| |dY_k| / cp (factor 2 for the Newton tolerance)
    W = h2_mech.molar_mass * 1e-3
    for i in range(n):
        cpR, hRT, _, _ = h2_oracle.thermo(o["T"][i])
        _, _, cp, _ = h2_oracle.mixture(o["T"][i], 101325.0, o["Y"][:, i])
        hk = hRT * 8.31446261815324 * o["T"][i] / W
        bound_T = np.sum(np.abs(hk) * np.abs(g["Y"][:, i] - o["Y"][:, i])) / cp
        assert abs(g["T"][i] - o["T"][i]) <= 2 * bound_T + 1e-8


def test_P16_identity_and_rr(tmp_path, gmech, h2_oracle, h2_mech):
    import paper_2210_07094_amd as df
    path = tmp_path / "id.dfdnn"
    _net(path, hidden=(160, 160, 160), zero_out=True)
    d = df.DNN(path, gmech)
    f = _cells(h2_mech, 300, seed=3)
    print("case: identity network", flush=True)
    g = _gpu_dnn(d, f, renormalise=1, rr=True)
    assert np.all(g["status"] == 0)
    np.testing.assert_allclose(g["Y"], f["Y"], rtol=1e-12)
    np.testing.assert_allclose(g["T"], f["T"], rtol=1e-12)
    assert np.abs(g["rr"]).max() < 1e-3


def test_fallback_and_nonfinite(tmp_path, gmech, h2_oracle, h2_mech):
    import paper_2210_07094_amd as df
    K = 9
    path = tmp_path / "box.dfdnn"
    lo = np.concatenate([[1300.0, 0.0], np.full(K, -1e9)])
    hi = np.concatenate([[5000.0, 1e9], np.full(K, 1e9)])
    _net(path, hidden=(160, 320, 160), box=(lo, hi))
    d = df.DNN(path, gmech)
    f = fields.ignition_cells(h2_mech, n=500, seed=31)
    f["T"][7] = np.nan
    print("case: fallback below 1300 K + one NaN cell", flush=True)
    g = _gpu_dnn(d, f)
    cold = f["T"] < 1300.0
    assert g["status"][7] == 3
    assert np.all(g["status"][cold] == 4)
    warm = ~cold
    warm[7] = False
    assert np.all(g["status"][warm] == 0)
    ref = h2_oracle.chem_step(f["T"][cold], f["p"][cold], f["Y"][:, cold], 1e-6)
    relT = np.abs(g["T"][cold] - ref["T"]) / ref["T"]
    mask = ref["Y"] > 1e-10
    relY = np.where(mask, np.abs(g["Y"][:, cold] - ref["Y"]) / np.where(mask, ref["Y"], 1), 0)
    assert max(relT.max(), relY.max()) <= 1e-8
    # fallback off: out-of-range cells untouched, flagged
    g0 = _gpu_dnn(d, f, fallback=0)
    assert np.all(g0["status"][cold] == 4)
    np.testing.assert_array_equal(g0["T"][cold], f["T"][cold])


def test_errors(tmp_path, gmech, h2_mech):
    import paper_2210_07094_amd as df
    torch = _torch()
    path = tmp_path / "e.dfdnn"
    _net(path, hidden=(160, 160, 160))
    d = df.DNN(path, gmech)
    f = _cells(h2_mech, 64, seed=4)
    T = torch.tensor(f["T"], device="cuda:0")
    p = torch.tensor(f["p"], device="cuda:0")
    Y = torch.tensor(f["Y"], device="cuda:0")
    with pytest.raises(df.DfError) as e:
        d.step(T, p, Y, 2e-6)
    assert e.value.code == -2
    small = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(df.DfError) as e:
        d.step(T, p, Y, 1e-6, workspace=small)
    assert e.value.code == -1
    assert d.dims == [11, 160, 160, 160, 9] and abs(d.dt_train - 1e-6) < 1e-20
