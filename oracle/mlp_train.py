"""Training of the DNN chemistry integrator -- test infrastructure only.

Plain float64 NumPy, written from the definitions, to check the device training kernels:
  * the network of the DNN form (Sec. "Chemistry Integration"): z-scored inputs
    (T, p, Box-Cox(Y)), hidden layers h_l = GELU(W_l h_{l-1} + b_l) with the exact erf
    GELU, a linear output layer u = W h + b giving the z-scored Box-Cox increments;
  * the loss L = 1/(B O) sum_b sum_o (u_bo - t_bo)^2;
  * its gradients by the chain rule, layer by layer from the output back:
      du = 2 (u - t)/(B O),  dW_out = du^T h,  db_out = sum_b du,  dh = du W_out,
      da_l = dh_l * GELU'(a_l),  dW_l = da_l^T h_{l-1},  db_l = sum_b da_l,  dh_{l-1} = da_l W_l,
    with GELU'(a) = Phi(a) + a phi(a);
  * one Adam step (Kingma and Ba, ICLR 2015, Algorithm 1):
      m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
      w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
  * the training pairs from an integrator step: x = z-score of (T, p, Box-Cox(Y0)),
    target = z-score of Box-Cox(Y1) - Box-Cox(Y0).
Weights come from the network file (the stored bf16 values, exactly, as float64).  Shares
nothing with the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    return 0.5 * (1.0 + erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def forward(Ws, bs, x):
    """Activations of every layer: (pre-activations a_l, outputs h_l) of the hidden layers and u."""
    h = [np.asarray(x, dtype=np.float64)]
    a = []
    for W, b in zip(Ws[:-1], bs[:-1]):
        a.append(h[-1] @ W.T + b)
        h.append(gelu(a[-1]))
    u = h[-1] @ Ws[-1].T + bs[-1]
    return a, h, u


def loss_and_grads(Ws, bs, x, t):
    """L and its gradients (lists dW, db in layer order) for a batch x [B, n_in], t [B, O]."""
    a, h, u = forward(Ws, bs, x)
    B, O = t.shape
    e = u - t
    L = float(np.sum(e * e) / (B * O))
    du = 2.0 * e / (B * O)
    dW = [None] * len(Ws)
    db = [None] * len(Ws)
    dW[-1] = du.T @ h[-1]
    db[-1] = du.sum(axis=0)
    dh = du @ Ws[-1]
    for l in range(len(Ws) - 2, -1, -1):
        da = dh * gelu_grad(a[l])
        dW[l] = da.T @ h[l]
        db[l] = da.sum(axis=0)
        dh = da @ Ws[l]
    return L, dW, db


def adam(w, g, m, v, t, lr, b1, b2, eps):
    """One Adam step at step count t (1-based); returns (w, m, v) new."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    w = w - lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    return w, m, v


def make_batch(net, T, p, Y0, Y1):
    """(x [n, K+2], target [n, K], valid [n]) from states before and after a step; net is the
    dict synth.dnnfile.read_dnn returns."""
    lam = net["lambda"]

    def bct(Y):
        return (np.power(np.maximum(Y, 0.0), lam) - 1.0) / lam

    z0, z1 = bct(np.asarray(Y0, dtype=np.float64)), bct(np.asarray(Y1, dtype=np.float64))
    f = np.concatenate([np.asarray(T, dtype=np.float64)[None, :], np.asarray(p, dtype=np.float64)[None, :], z0], axis=0)
    x = ((f.T - net["mu_in"]) / net["sig_in"])
    tgt = (((z1 - z0).T - net["mu_out"]) / net["sig_out"])
    valid = np.all((f.T >= net["box_lo"]) & (f.T <= net["box_hi"]), axis=1)
    return np.ascontiguousarray(x), np.ascontiguousarray(tgt), valid
