"""Pins of the oracle's FP8 inference (OCP E4M3FN, power-of-two scales) against what the format
and the mathematics fix: the rounding against torch's own float8_e4m3fn conversion (a library
routine) and against hand-worked ties and subnormals; the scale rule against hand cases; the
batched FP8 forward (a scale per row and block of 32 activations) against a brute-force
recomputation (quantisation by torch, products summed by numpy) on a small network; and the special case of a network with one hidden layer, which has
no hidden-to-hidden layer and must give the BF16-emulated forward exactly."""
import math

import numpy as np
import pytest

import oracle
from synth import dnnfile

torch = pytest.importorskip("torch")


def test_e4m3_rounding_matches_torch():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(40000) * np.exp(rng.uniform(-14, 6.2, 40000))
    # every representable value, the midpoints between neighbours (ties) and points just off them
    grid = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    grid = np.unique(grid[np.isfinite(grid) & (grid >= 0)])
    mids = 0.5 * (grid[1:] + grid[:-1])
    x = np.concatenate([x, grid, -grid, mids, -mids, mids * (1 + 2.0 ** -20), mids * (1 - 2.0 ** -20)])
    # fp32 inputs, as the GPU path converts (torch converts fp64 through fp32, rounding twice)
    x = x[np.abs(x) <= 448.0].astype(np.float32)
    ref = torch.tensor(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    x = x.astype(np.float64)
    got = np.array([oracle.fp8_e4m3_round(v) for v in x])
    assert np.array_equal(got, ref)


def test_e4m3_hand_values():
    r = oracle.fp8_e4m3_round
    assert r(448.0) == 448.0 and r(-448.0) == -448.0
    assert r(1.0625) == 1.0            # tie between 1 and 1.125: even mantissa 000
    assert r(1.1875) == 1.25           # tie between 1.125 and 1.25: even mantissa 010
    assert r(2.0 ** -6) == 2.0 ** -6   # smallest normal
    assert r(2.0 ** -9) == 2.0 ** -9   # smallest subnormal
    assert r(2.0 ** -10) == 0.0        # tie between 0 and 2^-9: to zero
    assert r(3 * 2.0 ** -10) == 2.0 ** -8  # tie between 2^-9 and 2^-8: even mantissa 010
    assert r(0.3) == 0.3125            # 0.3 = 1.2 * 2^-2, nearest 1.25 * 2^-2
    assert r(449.0) == 448.0 and r(464.0) == 448.0   # 464: tie between 448 and 480, to even
    assert math.isnan(r(470.0)) and math.isnan(r(float("inf")))  # rounds beyond 448: not a value


def test_scale_exponent():
    s = oracle.fp8_scale_exp
    assert s(448.0) == 0 and s(448.0 * (1 + 1e-15)) == 1
    assert s(1.0) == -8 and s(1.75) == -8 and s(1.76) == -7
    assert s(0.0) == 0 and s(896.0) == 1 and s(896.1) == 2
    assert s(float("inf")) == 0 and s(float("nan")) == 0   # no finite scale: left to the values
    assert s(448.0 * 2.0 ** -127) == -127 and s(448.0 * 2.0 ** -128) == -127 and s(1e-300) == -127  # E8M0 floor
    rng = np.random.default_rng(2)
    for a in np.exp(rng.uniform(-40, 40, 500)):
        e = s(a)
        assert 224.0 < math.ldexp(a, -e) <= 448.0


def _bf16(x):
    return torch.tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)


def _q(x):
    return torch.tensor(x, dtype=torch.float64).to(torch.float8_e4m3fn).to(torch.float64).numpy()


def _gelu(z):
    return 0.5 * z * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))


def _brute_force(net, X):
    """The FP8 forward recomputed: torch quantises, numpy sums (exactly, at these sizes)."""
    W, b, L = net["W"], net["b"], net["L"]
    a = _bf16(X)
    for l in range(L):
        if 1 <= l <= L - 2:
            ew = np.array([oracle.fp8_scale_exp(np.abs(w).max()) for w in W[l]])
            wq = _q(np.ldexp(W[l].astype(np.float64), -ew[:, None]))
            acc = np.zeros((a.shape[0], W[l].shape[0]))
            for c0 in range(0, a.shape[1], 32):      # blocks of 32 inputs of each row
                blk = a[:, c0:c0 + 32]
                ea = np.array([oracle.fp8_scale_exp(np.abs(r).max()) for r in blk])
                aq = _q(np.ldexp(blk, -ea[:, None]))
                acc += np.ldexp(aq @ wq[:, c0:c0 + 32].T, ea[:, None])
            z = np.ldexp(acc, ew[None, :]) + b[l].astype(np.float64)[None, :]
        else:
            # fp32 products and running fp32 sums, in input order
            acc = np.zeros((a.shape[0], W[l].shape[0]), dtype=np.float32)
            for c in range(W[l].shape[1]):
                acc = (acc + np.float32(a[:, c:c + 1]).astype(np.float32) * W[l][:, c][None, :]).astype(np.float32)
            z = (acc + b[l][None, :]).astype(np.float32).astype(np.float64)
        a = _bf16(_gelu(z)) if l < L - 1 else z
    return a


def test_fp8_forward_brute_force(tmp_path):
    K = 9
    rng = np.random.default_rng(4)
    T = rng.uniform(800, 2000, 64)
    p = np.full(64, 101325.0)
    Y = rng.dirichlet(np.ones(K), 64).T
    path = tmp_path / "net.dfdnn"
    dnnfile.write_seeded_network(path, K, T, p, Y, (48, 40, 32), seed=5)   # 48 and 40 inputs: a short last block
    net = dnnfile.read_dnn(path)
    X = rng.standard_normal((200, K + 2))
    X[7] = 0.0                         # a cell the network does not predict
    U = oracle.DNN(path).mlp_fp8(X)
    ref = _brute_force(net, X)
    scale = np.abs(ref).max()
    # the two could differ only where the C and numpy erf round a GELU output to different bf16;
    # at this seed they agree everywhere
    assert np.array_equal(U, ref)
    # the quantisation is there: the FP8 forward differs from the BF16 one by a few per cent
    U1 = np.array([oracle.DNN(path).mlp(x, mode=1) for x in X])
    assert 1e-3 * scale < np.max(np.abs(U - U1)) < 0.1 * scale


def test_fp8_forward_without_hidden_to_hidden_layer_is_bf16(tmp_path):
    K = 4
    rng = np.random.default_rng(6)
    T = rng.uniform(800, 2000, 32)
    p = np.full(32, 101325.0)
    Y = rng.dirichlet(np.ones(K), 32).T
    path = tmp_path / "one.dfdnn"
    dnnfile.write_seeded_network(path, K, T, p, Y, (40,), seed=7)
    d = oracle.DNN(path)
    X = rng.standard_normal((50, K + 2))
    U = d.mlp_fp8(X)
    for i in range(50):
        assert np.array_equal(U[i], d.mlp(X[i], mode=1))


def test_fp8_step_without_hidden_to_hidden_layer_is_bf16(tmp_path, h2_mech, h2_oracle):
    from synth import fields
    f = fields.ignition_cells(h2_mech, n=64, seed=3)
    path = tmp_path / "h2one.dfdnn"
    dnnfile.write_seeded_network(path, h2_mech.n_species, f["T"][8:], f["p"][8:], f["Y"][:, 8:], (64,), seed=8)
    d = oracle.DNN(path)
    a = d.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, mode=1, fallback=False)
    b = d.step(h2_oracle, f["T"], f["p"], f["Y"], 1e-6, mode=2, fallback=False)
    for k in ("T", "Y", "status"):
        assert np.array_equal(a[k], b[k], equal_nan=True)
