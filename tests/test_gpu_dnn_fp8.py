"""GPU parity of the DNN step with FP8 hidden-to-hidden layers (df_dnn_opts.precision = 1)
against the oracle's FP8 forward (mode 2): E4M3FN quantisation with power-of-two scales (one per
row and block of 32 for the activations, one per row for the weights), exact sums on the oracle's
side, fp32 sums of the block-scaled MFMAs on the GPU's.

The bar.  Both sides quantise bf16 activations to E4M3FN with the same rule, but the two sum the
products differently: the oracle exactly, the MFMA with an internal accumulation that differs
from the exact sum of each 32-product block by up to 2^-12 of the block's sum of |products|
(measured on gfx950 with exactly representable operands).  Over the 1600- and 800-term sums of the
hidden layers that error is about 2^-12 sqrt(n_blocks) x 32 |p| against |sum| ~ sqrt(n) |p|, i.e.
~1e-3 relative, a quarter of a bf16 ulp (2^-8): a large share of the hidden activations round
one bf16 ulp apart (and one in sixteen of those one FP8 step, 2^-3 of the value, in the next
layer's input), so almost every output differs by a small amount instead of a few by one ulp as
in the BF16 path.  Per output feature over all cells, in z = BoxCox(Y) space with renormalisation
off: max |du| <= 2^-5 max|u|, 99th percentile <= 1e-2 max|u|, median <= 1e-3 max|u|; and, as the
check that the quantisation itself is the oracle's (a wrong scale, byte order or subnormal rule
moves results by the size of the quantisation effect), the median |GPU - oracle| is at most a
tenth of the median |FP8 - BF16| of the oracle.  The stats are printed before the checks."""
import os

import numpy as np
import pytest

import oracle
from synth import dnnfile, fields
from test_gpu_dnn import _cells, _net, bct

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HC_MECH = os.path.join(ROOT, "synth", "data", "hc_synth_53sp_325r.mech")


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def gmech(h2_path):
    import paper_2210_07094_amd as df
    _torch()
    return df.Mechanism(h2_path)


def _step(dnn, f, precision=1, renormalise=0, fallback=1):
    import paper_2210_07094_amd as df
    torch = _torch()
    d = "cuda:0"
    T = torch.tensor(f["T"], device=d)
    p = torch.tensor(f["p"], device=d)
    Y = torch.tensor(np.ascontiguousarray(f["Y"]), device=d)
    st = torch.full((f["T"].size,), -7, dtype=torch.int32, device=d)
    dnn.step(T, p, Y, 1e-6, status=st,
             opts=df.dnn_opts(renormalise=renormalise, fallback=fallback, precision=precision))
    torch.cuda.synchronize()
    return {"T": T.cpu().numpy(), "Y": Y.cpu().numpy(), "status": st.cpu().numpy()}


def _check(f, g, o, mask=None, tag="", o_bf16=None):
    z0, zo, zg = bct(f["Y"]), bct(o["Y"]), bct(g["Y"])
    ok = o["Y"] > 0
    if mask is not None:
        ok = ok & mask[None, :]
    u = np.where(ok, (zo - z0) / 0.02, 0.0)
    du = np.where(ok, np.abs(zg - zo) / 0.02, 0.0)
    umax = np.abs(u).max(axis=1)
    r_max = du.max(axis=1) / umax
    r_99 = np.percentile(du, 99, axis=1) / umax
    r_50 = np.median(du, axis=1) / umax
    print(f"{tag} per output, largest: max {r_max.max():.3e}, p99 {r_99.max():.3e}, median {r_50.max():.3e}; "
          f"outputs equal {np.mean(du == 0):.4f}", flush=True)
    if o_bf16 is not None:
        dq = np.where(ok, np.abs(bct(o_bf16["Y"]) - zo) / 0.02, 0.0)
        print(f"{tag} median |GPU - oracle| {np.median(du[ok]):.3e}, median |FP8 - BF16| (oracle) "
              f"{np.median(dq[ok]):.3e}", flush=True)
        assert np.median(du[ok]) <= 0.1 * np.median(dq[ok])
    assert np.all(r_max <= 2.0 ** -5)
    assert np.all(r_99 <= 1e-2)
    assert np.all(r_50 <= 1e-3)


@pytest.mark.parametrize("n", [1024, 1001])
def test_fp8_network_parity(tmp_path, gmech, h2_oracle, h2_mech, n):
    import paper_2210_07094_amd as df
    path = tmp_path / "net.dfdnn"
    _net(path)
    d = df.DNN(path, gmech)
    f = _cells(h2_mech, n, seed=31 + n)
    print(f"case: random 11-1600-800-400-9 network in FP8, n={n}", flush=True)
    g = _step(d, f)
    od = oracle.DNN(path)
    o = od.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=2)
    ob = od.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=1)
    assert np.all(g["status"] == 0) and np.all(o["status"] == 0)
    _check(f, g, o, tag=f"n={n}", o_bf16=ob)
    # the quantisation is there: FP8 and BF16 results differ by more than the parity bar's median
    gb = _step(d, f, precision=0)
    assert np.max(np.abs(bct(gb["Y"]) - bct(g["Y"]))) > 1e-4 * 0.02


def test_fp8_out_of_box_cells_count_as_zero_input(tmp_path, gmech, h2_oracle, h2_mech):
    """Cells outside the training box are left (fallback off) and enter the activation scale as the
    response to a zero input, on both sides."""
    import paper_2210_07094_amd as df
    K = 9
    f = _cells(h2_mech, 600, seed=5)
    x0 = f["T"]
    lo = np.concatenate([[np.percentile(x0, 20)], np.full(K + 1, -1e300)])
    hi = np.full(K + 2, 1e300)
    path = tmp_path / "box.dfdnn"
    _net(path, box=(lo, hi), seed=2)
    d = df.DNN(path, gmech)
    g = _step(d, f, fallback=0)
    o = oracle.DNN(path).step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=2, fallback=False)
    out = g["status"] == df.CELL_DNN_FALLBACK
    assert 100 <= out.sum() <= 140 and np.array_equal(out, o["status"] == 4)
    assert np.array_equal(g["Y"][:, out], f["Y"][:, out]) and np.array_equal(g["T"][out], f["T"][out])
    _check(f, g, o, mask=~out, tag="box")


def test_fp8_repeat_then_smaller_call(tmp_path, gmech, h2_oracle, h2_mech):
    """The activation maxima start from zero on every call: a repeated call gives the same bits,
    and a smaller call after a larger one takes its own scales (the oracle's for that batch)."""
    import paper_2210_07094_amd as df
    path = tmp_path / "net.dfdnn"
    _net(path, seed=3)
    d = df.DNN(path, gmech)
    f = _cells(h2_mech, 768, seed=8)
    g1 = _step(d, f)
    g2 = _step(d, f)
    assert np.array_equal(g1["Y"], g2["Y"]) and np.array_equal(g1["T"], g2["T"])
    # the 200 coldest cells alone: smaller activations, so possibly a smaller scale than the full call's
    idx = np.argsort(f["T"])[:200]
    s = {"T": f["T"][idx].copy(), "p": f["p"][idx].copy(), "Y": np.ascontiguousarray(f["Y"][:, idx])}
    g3 = _step(d, s)
    o3 = oracle.DNN(path).step(h2_oracle, s["T"], s["p"], s["Y"], 1e-6, renormalise=False, mode=2)
    _check(s, g3, o3, tag="smaller")


def test_fp8_one_hidden_layer_is_bf16(tmp_path, gmech, h2_mech):
    import paper_2210_07094_amd as df
    path = tmp_path / "one.dfdnn"
    _net(path, hidden=(320,), seed=4)
    d = df.DNN(path, gmech)
    f = _cells(h2_mech, 300, seed=9)
    a = _step(d, f, precision=0)
    b = _step(d, f, precision=1)
    assert np.array_equal(a["Y"], b["Y"]) and np.array_equal(a["T"], b["T"])


def test_fp8_bad_precision(tmp_path, gmech, h2_mech):
    import paper_2210_07094_amd as df
    path = tmp_path / "net.dfdnn"
    _net(path, hidden=(160, 160))
    d = df.DNN(path, gmech)
    f = _cells(h2_mech, 64, seed=1)
    with pytest.raises(df.DfError):
        _step(d, f, precision=2)
    with pytest.raises(TypeError):
        df.dnn_opts(precison=1)


def test_fp8_large_network_parity(tmp_path):
    """The 55-3200-1600-800-53 network of the 53-species mechanism (seeded weights)."""
    import paper_2210_07094_amd as df
    import synth
    mech = synth.read_mech(HC_MECH)
    om, gm = oracle.Mech(HC_MECH), df.Mechanism(HC_MECH)
    f = fields.hydrocarbon_field(mech, n=1024)
    path = tmp_path / "hc.dfdnn"
    dnnfile.write_seeded_network(path, mech.n_species, f["T"], f["p"], f["Y"], (3200, 1600, 800), seed=3)
    print("case: seeded 55-3200-1600-800-53 network in FP8, 1024 hydrocarbon cells", flush=True)
    g = _step(df.DNN(path, gm), f)
    od = oracle.DNN(path)
    o = od.step(om, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=2)
    ob = od.step(om, f["T"], f["p"], f["Y"], 1e-6, renormalise=False, mode=1)
    assert np.all(g["status"] == 0) and np.all(o["status"] == 0)
    _check(f, g, o, tag="53 species", o_bf16=ob)
