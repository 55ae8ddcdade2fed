"""Pins of the oracle's DNN training (oracle/mlp_train.py), checked against what holds
independently of it: central differences of its loss for the gradients, a difference quotient
of GELU, the closed form of Adam's first step, the C oracle's float64 forward pass of the same
network, and the C oracle's Box-Cox transform for the training pairs."""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp_train as mt
from synth.dnnfile import read_dnn

DNN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2210_07094_amd", "data",
                   "h2_dnn_1600_800_400.dfdnn")


def _tiny(seed=0):
    rng = np.random.default_rng(seed)
    dims = [5, 7, 6, 3]
    Ws = [rng.standard_normal((dims[i + 1], dims[i])) * 0.7 for i in range(3)]
    bs = [rng.standard_normal(dims[i + 1]) * 0.3 for i in range(3)]
    x = rng.standard_normal((4, 5))
    t = rng.standard_normal((4, 3))
    return Ws, bs, x, t


def test_gradients_match_central_differences():
    Ws, bs, x, t = _tiny()
    L, dW, db = mt.loss_and_grads(Ws, bs, x, t)
    h = 1e-6
    for l in range(3):
        for idx in np.ndindex(*Ws[l].shape):
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (mt.loss_and_grads(Wp, bs, x, t)[0] - mt.loss_and_grads(Wm, bs, x, t)[0]) / (2 * h)
            assert abs(fd - dW[l][idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx)
        for i in range(bs[l].size):
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[l][i] += h
            bm[l][i] -= h
            fd = (mt.loss_and_grads(Ws, bp, x, t)[0] - mt.loss_and_grads(Ws, bm, x, t)[0]) / (2 * h)
            assert abs(fd - db[l][i]) <= 1e-7 * max(1.0, abs(fd)), (l, i)
    # the loss itself: mean over batch and outputs
    u = mt.forward(Ws, bs, x)[2]
    assert L == pytest.approx(np.mean((u - t) ** 2), rel=1e-14)


def test_gelu_grad():
    a = np.linspace(-6, 6, 121)
    h = 1e-6
    fd = (mt.gelu(a + h) - mt.gelu(a - h)) / (2 * h)
    assert np.max(np.abs(fd - mt.gelu_grad(a))) < 1e-8
    assert mt.gelu_grad(np.array([0.0]))[0] == 0.5


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    w, g = rng.standard_normal(50), rng.standard_normal(50)
    w1, m, v = mt.adam(w, g, np.zeros(50), np.zeros(50), 1, 1e-3, 0.9, 0.999, 1e-8)
    # m/(1-b1) = g and v/(1-b2) = g^2 at the first step
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_forward_matches_c_oracle_network():
    net = read_dnn(DNN)
    od = oracle.DNN(DNN)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, net["dims"][0]))
    Ws = [w.astype(np.float64) for w in net["W"]]
    bs = [b.astype(np.float64) for b in net["b"]]
    u = mt.forward(Ws, bs, x)[2]
    for i in range(3):
        assert np.allclose(u[i], od.mlp(x[i], mode=0), rtol=1e-12, atol=1e-12)


def test_make_batch_matches_c_box_cox(h2_mech, h2_oracle):
    from synth import fields
    net = read_dnn(DNN)
    f = fields.ignition_cells(h2_mech, n=20, seed=6)
    o = h2_oracle.chem_step(f["T"], f["p"], f["Y"], net["dt_train"], h_inout=np.zeros(20))
    x, t, valid = mt.make_batch(net, f["T"], f["p"], f["Y"], o["Y"])
    lam = net["lambda"]
    for i in range(20):
        z0 = np.array([oracle.bct(y, lam) for y in f["Y"][:, i]])
        z1 = np.array([oracle.bct(y, lam) for y in o["Y"][:, i]])
        feat = np.concatenate([[f["T"][i], f["p"][i]], z0])
        assert np.allclose(x[i], (feat - net["mu_in"]) / net["sig_in"], rtol=1e-12, atol=1e-12)
        assert np.allclose(t[i], ((z1 - z0) - net["mu_out"]) / net["sig_out"], rtol=1e-10, atol=1e-10)
    assert valid.dtype == bool
