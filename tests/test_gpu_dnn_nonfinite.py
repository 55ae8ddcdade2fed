"""Non-finite values inside the network of the DNN step, BF16 and FP8, against the oracle.

A NaN or an overflow inside the network must reach the cell's status as DF_CELL_NONFINITE, with
the state NaN, on the GPU as in the oracle (mode 1 for BF16, mode 2 for FP8): E4M3FN has no
infinity, so an infinite or out-of-range activation quantises to NaN, and the inverse Box-Cox
keeps a NaN output NaN (its clamp at zero applies to negative bases only).
  * a NaN weight in the first layer: one hidden unit is NaN in every cell, so every output is;
  * a NaN weight in the output layer: one output is NaN in every cell;
  * an overflowing first layer: one hidden unit is 2^127 x0 with x0 the normalised temperature,
    +inf where x0 >= 2 and beyond E4M3FN's range where 0 < x0 < 2, and -0 for x0 <= 0.  The
    activation maximum is then infinite, so the FP8 layer quantises at scale 1 on both sides:
    the cells with x0 > 0 become NaN and the others are held to the FP8 parity bars.
"""
import numpy as np
import pytest

import oracle
from synth import dnnfile
from test_gpu_dnn import _cells, bct

pytestmark = pytest.mark.gpu

K = 9
LAM = 0.1


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def gmech(h2_path):
    import paper_2210_07094_amd as df
    _torch()
    return df.Mechanism(h2_path)


def _write(path, edit, mu_T=1300.0, sig_T=300.0, seed=0):
    rng = np.random.default_rng(seed)
    dims = [K + 2, 160, 160, 160, K]
    W = [rng.normal(0, 1.0 / np.sqrt(dims[l]), (dims[l + 1], dims[l])).astype(np.float32) for l in range(4)]
    b = [rng.normal(0, 0.1, dims[l + 1]).astype(np.float32) for l in range(4)]
    edit(W, b)
    mu_in = np.concatenate([[mu_T, 101325.0], np.full(K, -5.0)])
    sig_in = np.concatenate([[sig_T, 1.0], np.full(K, 3.0)])
    dnnfile.write_dnn(path, W, b, K, LAM, 1e-6, mu_in, sig_in, np.zeros(K), np.full(K, 0.02),
                      np.full(K + 2, -1e300), np.full(K + 2, 1e300))


def _step(dnn, f, precision):
    import paper_2210_07094_amd as df
    torch = _torch()
    d = "cuda:0"
    T = torch.tensor(f["T"], device=d)
    p = torch.tensor(f["p"], device=d)
    Y = torch.tensor(np.ascontiguousarray(f["Y"]), device=d)
    st = torch.full((f["T"].size,), -7, dtype=torch.int32, device=d)
    dnn.step(T, p, Y, 1e-6, status=st, opts=df.dnn_opts(renormalise=0, precision=precision))
    torch.cuda.synchronize()
    return {"T": T.cpu().numpy(), "Y": Y.cpu().numpy(), "status": st.cpu().numpy()}


def _same_nonfinite(g, o):
    np.testing.assert_array_equal(g["status"], o["status"])
    bad = o["status"] == 3
    assert np.all(np.isnan(g["T"][bad])) and np.all(np.isnan(o["T"][bad]))
    np.testing.assert_array_equal(np.isnan(g["Y"]), np.isnan(o["Y"]))
    return bad


@pytest.mark.parametrize("where", ["first", "output"])
def test_nan_weight(tmp_path, gmech, h2_oracle, h2_mech, where):
    import paper_2210_07094_amd as df

    def edit(W, b):
        if where == "first":
            W[0][5, 3] = np.nan
        else:
            W[3][2, 17] = np.nan

    path = tmp_path / "nan.dfdnn"
    _write(path, edit)
    d = df.DNN(path, gmech)
    od = oracle.DNN(path)
    f = _cells(h2_mech, 300, seed=12)
    print(f"case: NaN weight in the {where} layer, 300 cells, BF16 and FP8", flush=True)
    for precision, mode in ((0, 1), (1, 2)):
        g = _step(d, f, precision)
        o = od.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=mode)
        bad = _same_nonfinite(g, o)
        assert np.all(bad), "every cell has a NaN output"
        if where == "output":
            assert np.all(np.isnan(g["Y"][2])) and not np.any(np.isnan(np.delete(g["Y"], 2, axis=0)))


def test_overflowing_layer_fp8(tmp_path, gmech, h2_oracle, h2_mech):
    import paper_2210_07094_amd as df

    def edit(W, b):
        W[0][0, :] = 0.0
        W[0][0, 0] = 2.0 ** 127
        b[0][0] = 0.0

    path = tmp_path / "ovf.dfdnn"
    # x0 = (T - 1150)/150 lies in [-1, 3] for T0 in [1000, 1600] K
    _write(path, edit, mu_T=1150.0, sig_T=150.0)
    d = df.DNN(path, gmech)
    od = oracle.DNN(path)
    f = _cells(h2_mech, 600, seed=14)
    print("case: overflowing first layer, 600 cells, FP8", flush=True)
    g = _step(d, f, 1)
    o = od.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=2)
    bad = _same_nonfinite(g, o)
    x0 = np.array([np.float32(v) for v in (f["T"] - 1150.0) / 150.0])
    assert np.array_equal(bad, x0 > 0)
    assert 0 < bad.sum() < bad.size
    ok = ~bad
    zo, zg, z0 = bct(o["Y"][:, ok]), bct(g["Y"][:, ok]), bct(f["Y"][:, ok])
    m = o["Y"][:, ok] > 0
    u = np.where(m, (zo - z0) / 0.02, 0.0)
    du = np.where(m, np.abs(zg - zo) / 0.02, 0.0)
    umax = np.abs(u).max(axis=1)
    print("max |du| / max|u| per output:", np.array2string(du.max(axis=1) / umax, precision=2), flush=True)
    assert np.all(du.max(axis=1) <= 2.0 ** -5 * umax)
    assert np.all(np.median(du, axis=1) <= 1e-3 * umax)
