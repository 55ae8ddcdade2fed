"""DNN weights file ("DFDNN01"), writer and reader.

Little-endian binary::

    char[8]  "DFDNN01\\0"
    int32    L                      number of layers (hidden + output)
    int32    dims[L+1]              widths, dims[0] = K + 2 inputs, dims[L] = K outputs
    int32    K, reserved
    float64  lambda, dt_train       Box-Cox exponent, time step of the training labels
    float64  mu_in[K+2], sig_in[K+2], mu_out[K], sig_out[K]
    float64  box_lo[K+2], box_hi[K+2]     training range of the raw inputs (T, p, z_1..z_K)
    per layer l: uint16 W[dims[l+1]][dims[l]] (bfloat16 bits, row-major), float32 b[dims[l+1]]

Inputs are x = (T, p, z_1..z_K) with z = BoxCox(Y); the network maps
(x - mu_in)/sig_in through GELU hidden layers to the normalised increment of
z over dt_train, u = (dz - mu_out)/sig_out.
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = b"DFDNN01\0"


def f32_to_bf16_bits(a):
    """Round float32 values to bfloat16 (nearest, ties to even); returns uint16 bits."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    r[nan] = 0x7FC0
    return r


def bf16_bits_to_f32(b):
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def write_dnn(path, weights, biases, K, lam, dt_train, mu_in, sig_in, mu_out, sig_out, box_lo, box_hi):
    """weights[l]: float array [out, in] (rounded to bf16 on write); biases[l]: [out] float32."""
    L = len(weights)
    dims = [weights[0].shape[1]] + [w.shape[0] for w in weights]
    assert dims[0] == K + 2 and dims[-1] == K
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<i", L))
        f.write(struct.pack(f"<{L + 1}i", *dims))
        f.write(struct.pack("<ii", K, 0))
        f.write(struct.pack("<dd", lam, dt_train))
        for arr, n in ((mu_in, K + 2), (sig_in, K + 2), (mu_out, K), (sig_out, K), (box_lo, K + 2),
                       (box_hi, K + 2)):
            a = np.ascontiguousarray(arr, dtype="<f8")
            assert a.size == n
            f.write(a.tobytes())
        for w, b in zip(weights, biases):
            f.write(f32_to_bf16_bits(np.asarray(w, dtype=np.float32)).astype("<u2").tobytes())
            f.write(np.ascontiguousarray(b, dtype="<f4").tobytes())


def read_dnn(path):
    with open(path, "rb") as f:
        data = f.read()
    assert data[:8] == MAGIC, "not a DFDNN01 file"
    off = 8
    (L,) = struct.unpack_from("<i", data, off)
    off += 4
    dims = list(struct.unpack_from(f"<{L + 1}i", data, off))
    off += 4 * (L + 1)
    K, _ = struct.unpack_from("<ii", data, off)
    off += 8
    lam, dtt = struct.unpack_from("<dd", data, off)
    off += 16
    out = {"L": L, "dims": dims, "K": K, "lambda": lam, "dt_train": dtt}
    for name, n in (("mu_in", K + 2), ("sig_in", K + 2), ("mu_out", K), ("sig_out", K), ("box_lo", K + 2),
                    ("box_hi", K + 2)):
        out[name] = np.frombuffer(data, dtype="<f8", count=n, offset=off).copy()
        off += 8 * n
    Ws, bs = [], []
    for l in range(L):
        n = dims[l + 1] * dims[l]
        Ws.append(bf16_bits_to_f32(np.frombuffer(data, dtype="<u2", count=n, offset=off)).reshape(dims[l + 1], dims[l]))
        off += 2 * n
        bs.append(np.frombuffer(data, dtype="<f4", count=dims[l + 1], offset=off).copy())
        off += 4 * dims[l + 1]
    out["W"], out["b"] = Ws, bs
    return out


def write_seeded_network(path, K, T, p, Y, hidden, seed=0, lam=0.1, dt_train=1e-6, out_scale=0.02):
    """A DFDNN01 network with seeded random weights (no training): inputs normalised by the mean
    and standard deviation of (T, p, BoxCox(Y)) over the given cells, He-scaled hidden layers,
    an output layer scaled down so the increments stay small, output scale out_scale in z, and
    a training box wide enough that every given cell is inside it.  For throughput and parity
    work where no trained weights exist."""
    rng = np.random.default_rng(seed)
    z = (np.maximum(np.asarray(Y), 0.0) ** lam - 1.0) / lam
    X = np.vstack([np.asarray(T)[None, :], np.asarray(p)[None, :], z])
    mu_in = X.mean(axis=1)
    sig_in = np.maximum(X.std(axis=1), 1e-6 * np.maximum(np.abs(mu_in), 1.0))
    dims = [K + 2, *hidden, K]
    W = [rng.normal(0, np.sqrt(2.0 / dims[l]), (dims[l + 1], dims[l])).astype(np.float32)
         for l in range(len(dims) - 1)]
    W[-1] *= 0.1
    b = [rng.normal(0, 0.05, dims[l + 1]).astype(np.float32) for l in range(len(dims) - 1)]
    lo = X.min(axis=1) - 1.0 * sig_in
    hi = X.max(axis=1) + 1.0 * sig_in
    write_dnn(path, W, b, K, lam, dt_train, mu_in, sig_in, np.zeros(K), np.full(K, out_scale), lo, hi)
