"""The Phi table of the inference GELU (paper_2210_07094_amd/csrc/df_phi_table.h).

GELU(x) = x Phi(x) is the hidden-layer activation of the DNN chemistry integrator (Sec.
"Acceleration from Machine Learning").  The device evaluates Phi from a table of one cubic per
interval of 12/256 on [-6, 6]; these tests check the committed header against its generator
and the device arithmetic, emulated in float32 here, against the definition (math.erf in double),
against printed values of the standard normal distribution, and at the special inputs.
"""
import importlib.util
import math
import os
import re

import numpy as np

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2210_07094_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_phi_table", os.path.join(CSRC, "gen_phi_table.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _table():
    text = open(os.path.join(CSRC, "df_phi_table.h")).read()
    body = text[text.index("= {") + 3:text.index("};")]
    vals = np.array([float(v) for v in re.findall(r"([-+0-9.eE]+)f,", body)], dtype=np.float64)
    t = vals.astype(np.float32)
    assert np.array_equal(t.astype(np.float64), vals), "every literal is a float32 value"
    return t.reshape(-1, 4)


def _f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def gelu_device(x):
    """The kernel's steps in float32: position s = x 256/12 clamped to [-129, 128] (NaN to -129),
    entry floor(s) + 129 and fraction, Horner's rule in fused multiply-adds (each rounded once:
    exact product and sum in double, then float32), product with x."""
    tab = _table()
    x = _f32(x)
    n = 256
    s = _f32(x.astype(np.float64) * np.float64(np.float32(n / 12.0)))
    s = np.where(np.isnan(s), np.float32(-n / 2 - 1), s)
    s = np.minimum(np.maximum(s, np.float32(-n / 2 - 1)), np.float32(n / 2))
    fl = np.floor(s)
    k = fl.astype(np.int64) + n // 2 + 1
    u = _f32(s.astype(np.float64) - fl)
    c = tab[k].astype(np.float64)
    u64 = u.astype(np.float64)
    q = _f32(c[:, 3] * u64 + c[:, 2]).astype(np.float64)
    q = _f32(q * u64 + c[:, 1]).astype(np.float64)
    phi = _f32(q * u64 + c[:, 0])
    with np.errstate(invalid="ignore"):
        return _f32(x.astype(np.float64) * phi.astype(np.float64)), phi


def gelu_exact(x):
    return np.array([v * 0.5 * (1.0 + math.erf(v / math.sqrt(2.0))) for v in np.asarray(x, np.float64)])


def test_header_is_the_generator_output():
    assert open(os.path.join(CSRC, "df_phi_table.h")).read() == _gen().text()


def test_table_layout():
    t = _table()
    assert t.shape == (258, 4)
    assert np.all(t[0] == 0.0) and np.all(t[257] == [1.0, 0.0, 0.0, 0.0])
    assert abs(t[129, 0] - 0.5) <= 2.0 ** -25                         # Phi(0) = 1/2
    # each cubic ends where the next one starts (Phi is continuous) to within the fit's error
    ends = t[1:257].astype(np.float64).sum(axis=1)
    assert np.all(np.abs(ends[:-1] - t[2:257, 0]) <= 2e-9 + 1e-7 * t[2:257, 0])
    assert abs(ends[-1] - 1.0) <= 1e-7


def test_interpolated_gelu_within_bound_of_definition():
    rng = np.random.default_rng(0)
    x = np.concatenate([np.linspace(-6, 8, 400_001), rng.normal(0, 2, 200_000),
                        -6 + 12 * np.arange(257) / 256.0, rng.uniform(-1e-3, 1e-3, 1000)])
    x = _f32(x)
    g, _ = gelu_device(x)
    e = gelu_exact(x.astype(np.float64))
    # the cubic's error (1.5e-9 absolute, about 1e-6 relative at -6) and the float32 roundings: of
    # the coefficients, Horner's rule and the product (about 2e-7 relative), and of the position
    # x 256/12, which moves the argument by up to 6e-8 relative, i.e. Phi by up to
    # 6e-8 |x phi(x) / Phi(x)| relative, about 6e-8 (1 + x^2) for negative x
    err = np.abs(g.astype(np.float64) - e)
    rel = err / np.maximum(np.abs(e), 1e-300)
    nz = (x != 0) & (x >= -6)          # below -6 Phi is 0 (test_below_the_table)
    bound = 2e-7 + 1e-7 * x.astype(np.float64) ** 2 + np.where(x < -5, 2e-6, 0.0)
    assert np.all(rel[nz] <= bound[nz]), float(np.max(rel[nz] / bound[nz]))
    # on the bulk of the activations, |x| <= 2, the error is that of a few float32 roundings
    m = nz & (np.abs(x) <= 2)
    assert rel[m].max() <= 6e-7 and np.mean(rel[m]) <= 1.5e-7


def test_below_the_table():
    x = _f32(np.array([-6.05, -7.0, -50.0, -1e30]))
    g, phi = gelu_device(x)
    assert np.all(phi == 0.0) and np.all(g == 0.0) and np.all(np.signbit(g))


def test_printed_normal_distribution_values():
    # values of the standard normal distribution function as printed in statistical tables
    # (Abramowitz & Stegun, Table 26.1): Phi(1) = 0.8413447461, Phi(1.96) = 0.9750021049,
    # Phi(-3) = 0.0013498980, Phi(2.5) = 0.9937903347
    for xv, pv in ((1.0, 0.8413447461), (1.96, 0.9750021049), (-3.0, 0.0013498980), (2.5, 0.9937903347)):
        _, phi = gelu_device(np.array([xv]))
        assert abs(float(phi[0]) - pv) <= 1.5e-10 + 6e-8 * pv, (xv, float(phi[0]), pv)


def test_special_inputs():
    x = np.array([np.nan, np.inf, -np.inf, 1e30, -1e30, 0.0, -0.0, 6.0, -6.0, 100.0, -100.0], dtype=np.float32)
    g, _ = gelu_device(x)
    assert np.isnan(g[0]) and g[1] == np.inf and np.isnan(g[2])
    assert g[3] == np.float32(1e30) and g[4] == 0.0
    assert g[5] == 0.0 and g[6] == 0.0 and g[7] == 6.0 and abs(g[8] / (-6 * 9.8658765e-10) - 1) <= 3e-6
    assert g[9] == 100.0 and g[10] == 0.0
