"""Pins of the oracle's DNN form (P14-P16, BF16 emulation, MLP forward)."""
import numpy as np
import pytest
from scipy.special import erf

import oracle
from synth import dnnfile, fields

LAM = 0.1


def _write_net(path, K, hidden, rng=None, zero_out=False, mu_out=None, sig_out=None, box=None, scale=0.3):
    rng = rng or np.random.default_rng(0)
    dims = [K + 2, *hidden, K]
    W = [rng.normal(0, scale / np.sqrt(dims[l]), (dims[l + 1], dims[l])).astype(np.float32) for l in range(len(dims) - 1)]
    b = [rng.normal(0, 0.05, dims[l + 1]).astype(np.float32) for l in range(len(dims) - 1)]
    if zero_out:
        W[-1][:] = 0
        b[-1][:] = 0
    mu_in = np.concatenate([[1200.0, 101325.0], np.full(K, -5.0)])
    sig_in = np.concatenate([[400.0, 1.0], np.full(K, 3.0)])
    mu_out = np.zeros(K) if mu_out is None else mu_out
    sig_out = np.full(K, 0.01) if sig_out is None else sig_out
    lo, hi = box if box is not None else (np.full(K + 2, -1e300), np.full(K + 2, 1e300))
    dnnfile.write_dnn(path, W, b, K, LAM, 1e-6, mu_in, sig_in, mu_out, sig_out, lo, hi)
    return W, b


def test_P14_boxcox_roundtrip_and_log_limit():
    for Y in [1e-12, 1e-6, 0.01, 0.3, 0.999, 1.0]:
        z = oracle.bct(Y, LAM)
        assert abs(oracle.bct_inv(z, LAM) / Y - 1) < 1e-13
        # lambda -> 0 gives the logarithm
        assert abs(oracle.bct(Y, 1e-9) - np.log(Y)) < 1e-6 * max(1.0, abs(np.log(Y)))
    # clamping: Y <= 0 maps to -1/lambda, and the inverse clamps its base at 0
    assert oracle.bct(0.0, LAM) == -1.0 / LAM
    assert oracle.bct(-1e-3, LAM) == -1.0 / LAM
    assert oracle.bct_inv(-20.0, LAM) == 0.0


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.normal(0, 3, 2000), rng.normal(0, 1e-3, 500), [0.0, -0.0, 1.0, 1.00390625,
                         1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 65504.0, 3.3895e38, -2.5e-39]]).astype(np.float32)
    ref = torch.tensor(xs).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle.bf16_round(float(v)) for v in xs], dtype=np.float32)
    np.testing.assert_array_equal(got, ref)


def test_mlp_forward_closed_form(tmp_path):
    """Hidden unit 0 copies x0 and later layers pass it on: u = w GELU(... GELU(x0))."""
    K = 9
    path = tmp_path / "cf.dfdnn"
    dims = [K + 2, 4, K]
    W = [np.zeros((4, K + 2), np.float32), np.zeros((K, 4), np.float32)]
    W[0][0, 0] = 1.0
    w_out = np.linspace(-1, 1, K).astype(np.float32)
    W[1][:, 0] = w_out
    b = [np.zeros(4, np.float32), np.full(K, 0.25, np.float32)]
    dnnfile.write_dnn(path, W, b, K, LAM, 1e-6, np.zeros(K + 2), np.ones(K + 2), np.zeros(K), np.ones(K),
                      np.full(K + 2, -1e300), np.full(K + 2, 1e300))
    d = oracle.DNN(path)
    for x0 in (-2.3, -0.4, 0.0, 0.7, 3.1):
        x = np.zeros(K + 2)
        x[0] = x0
        g = 0.5 * x0 * (1 + erf(x0 / np.sqrt(2)))
        np.testing.assert_allclose(d.mlp(x, mode=0), w_out.astype(np.float64) * g + 0.25, rtol=1e-14, atol=1e-15)
        # bf16 mode: x and the activation are rounded to bf16, products and sums in fp32
        import torch
        xb = float(torch.tensor(x0, dtype=torch.float32).to(torch.bfloat16))
        gb = float(torch.tensor(0.5 * xb * (1 + erf(xb / np.sqrt(2))), dtype=torch.float32).to(torch.bfloat16))
        ref = (np.float32(w_out) * np.float32(gb) + np.float32(0.25)).astype(np.float64)
        np.testing.assert_allclose(d.mlp(x, mode=1), ref, rtol=1e-6, atol=1e-7)


def test_mlp_matches_float64_reference(tmp_path):
    """FP64 mode equals a float64 matrix product chain of the same (bf16-valued)
    weights; BF16 mode stays within the bf16 rounding bound of it."""
    K = 9
    path = tmp_path / "r.dfdnn"
    rng = np.random.default_rng(5)
    _write_net(path, K, [64, 48, 32], rng)
    net = dnnfile.read_dnn(path)
    d = oracle.DNN(path)
    for _ in range(5):
        x = rng.normal(0, 1, K + 2)
        a = x
        for l in range(3):
            a = net["W"][l].astype(np.float64) @ a + net["b"][l]
            a = 0.5 * a * (1 + erf(a / np.sqrt(2)))
        u = net["W"][3].astype(np.float64) @ a + net["b"][3]
        np.testing.assert_allclose(d.mlp(x, 0), u, rtol=1e-12, atol=1e-12)
        assert np.abs(d.mlp(x, 1) - u).max() <= 0.03 * np.abs(u).max()


def test_P15_temperature_recovery(h2_oracle, h2_mech):
    f = fields.ignition_cells(h2_mech, n=8, seed=9)
    for i in range(8):
        Y = f["Y"][:, i]
        _, _, _, h0 = h2_oracle.mixture(f["T"][i], 101325.0, Y)
        T, it = oracle.T_from_h(h2_oracle, h0, Y, f["T"][i] + 150.0)
        assert it > 0 and abs(T - f["T"][i]) <= 1e-12 * f["T"][i] * 10


def test_P16_identity_network(tmp_path, h2_oracle, h2_mech):
    """Zero output layer and zero output mean: dz = 0, so Y and T come back unchanged."""
    path = tmp_path / "id.dfdnn"
    _write_net(path, 9, [32, 16, 8], zero_out=True)
    d = oracle.DNN(path)
    f = fields.ignition_cells(h2_mech, n=40, seed=11)
    r = d.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=True, mode=1, want_rr=True)
    assert np.all(r["status"] == 0)
    np.testing.assert_allclose(r["Y"], f["Y"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(r["T"], f["T"], rtol=1e-12)
    assert np.abs(r["rr"]).max() < 1e-3


def test_fallback_cells_use_the_integrator(tmp_path, h2_oracle, h2_mech):
    """Cells outside the training box are advanced by the integrator."""
    K = 9
    path = tmp_path / "box.dfdnn"
    lo = np.concatenate([[1300.0, 0.0], np.full(K, -1e9)])
    hi = np.concatenate([[5000.0, 1e9], np.full(K, 1e9)])
    _write_net(path, K, [16, 16, 16], zero_out=True, box=(lo, hi))
    d = oracle.DNN(path)
    f = fields.ignition_cells(h2_mech, n=64, seed=12)
    r = d.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6)
    cold = f["T"] < 1300.0
    assert np.all(r["status"][cold] == 4) and np.all(r["status"][~cold] == 0)
    ref = h2_oracle.chem_step(f["T"][cold], f["p"][cold], f["Y"][:, cold], 1e-6)
    np.testing.assert_array_equal(r["T"][cold], ref["T"])
    np.testing.assert_array_equal(r["Y"][:, cold], ref["Y"])
    r0 = d.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, fallback=False)
    np.testing.assert_array_equal(r0["T"][cold], f["T"][cold])


def _stage3_reference(npc, T0, p, Y0, u, mu_out, sig_out, lam, dt, renormalise):
    """Stage 3 of the DNN step written out from its definition with NumPy: the increment of
    z = BoxCox(Y) is u sig_out + mu_out; Y' = max(1 + lam z', 0)^(1/lam); optionally Y' / sum Y';
    T' solves h(T', Y') = h(T0, Y0) (bisection on the independent NumPy enthalpy, no Newton);
    rr = rho0 (Y' - Y0) / dt with rho0 = p Wbar0 / (R T0)."""
    from npchem import R
    z0 = (np.maximum(Y0, 0.0) ** lam - 1.0) / lam
    z1 = z0 + (u * sig_out + mu_out)
    Y1 = np.maximum(1.0 + lam * z1, 0.0) ** (1.0 / lam)
    if renormalise:
        Y1 = Y1 / Y1.sum()
    h0 = npc.h_mass(T0, Y0)
    lo, hi = 200.0, 4000.0
    assert npc.h_mass(lo, Y1) < h0 < npc.h_mass(hi, Y1)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if npc.h_mass(mid, Y1) < h0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-13 * mid:
            break
    T1 = 0.5 * (lo + hi)
    Wbar0 = 1.0 / np.sum(Y0 / npc.W)
    rho0 = p * Wbar0 / (R * T0)
    return T1, Y1, rho0 * (Y1 - Y0) / dt


@pytest.mark.parametrize("renormalise", [True, False])
@pytest.mark.parametrize("mode", [0, 1])
def test_stage3_against_definition(tmp_path, h2_oracle, h2_mech, npchem, renormalise, mode):
    """Stage 3 of the DNN step (inverse normalisation, inverse Box-Cox, renormalisation, T from
    the enthalpy, rr), Sec. "Description of the new classes": the output layer has zero weights
    and a chosen bias, so u equals the bias exactly in either precision, and the mean and scale
    of the outputs differ per species and from each other.  Swapping sig_out and mu_out, a sign
    of the increment, a missing renormalisation, the clamp of the inverse transform or a wrong
    density in rr each change the result far beyond the bar."""
    K = 9
    path = tmp_path / "s3.dfdnn"
    rng = np.random.default_rng(17)
    dims = [K + 2, 24, 16, 12, K]
    W = [rng.normal(0, 0.3, (dims[l + 1], dims[l])).astype(np.float32) for l in range(4)]
    b = [rng.normal(0, 0.05, dims[l + 1]).astype(np.float32) for l in range(4)]
    W[-1][:] = 0.0
    # output bias in float32; species 6 (HO2) gets an increment below -1/lambda - z0, so the
    # inverse transform clamps it to zero
    b[-1] = np.array([0.75, -1.25, 0.5, 2.0, -0.5, 1.5, -60.0, 0.25, -0.75], np.float32)
    mu_out = np.array([0.011, -0.023, 0.017, 0.05, -0.031, 0.029, 0.0, -0.013, 0.002])
    sig_out = np.array([0.04, 0.09, 0.06, 0.5, 0.3, 0.2, 1.0, 0.7, 0.01])
    mu_in = np.concatenate([[1300.0, 101325.0], np.full(K, -5.0)])
    sig_in = np.concatenate([[300.0, 1.0], np.full(K, 3.0)])
    dnnfile.write_dnn(path, W, b, K, LAM, 1e-6, mu_in, sig_in, mu_out, sig_out,
                      np.full(K + 2, -1e300), np.full(K + 2, 1e300))
    d = oracle.DNN(path)
    f = fields.ignition_cells(h2_mech, n=24, seed=29)
    Y = f["Y"] + rng.uniform(0, 1, f["Y"].shape) ** 4 * 1e-3
    f["Y"] = Y / Y.sum(axis=0, keepdims=True)
    r = d.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, renormalise=renormalise, mode=mode, want_rr=True)
    assert np.all(r["status"] == 0)
    u = b[-1].astype(np.float64)
    for i in range(f["T"].size):
        T1, Y1, rr = _stage3_reference(npchem, f["T"][i], f["p"][i], f["Y"][:, i], u, mu_out, sig_out, LAM,
                                       1e-6, renormalise)
        assert Y1[6] == 0.0 and r["Y"][6, i] == 0.0
        np.testing.assert_allclose(r["Y"][:, i], Y1, rtol=1e-12, atol=0)
        assert abs(r["T"][i] - T1) <= 1e-10 * T1
        np.testing.assert_allclose(r["rr"][:, i], rr, rtol=1e-9, atol=1e-9 * np.abs(rr).max())
        if not renormalise:
            assert abs(Y1.sum() - 1.0) > 1e-3   # the case really tests the switch
