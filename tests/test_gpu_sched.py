"""GPU checks of the schedules of the detailed-chemistry step: per-cell step lengths
(df_chem_step_cells), the persistent work-queue schedule and the schedule autotuner.

Parity bar as in test_gpu_chem: <= 1e-8 relative in T and in Y_k > 1e-10 against the
CPU oracle on cells with the oracle's accept/reject sequence, the integration tolerance
(|dy| <= 10 (atol + rtol |y|)) on the rare cells where rounding flipped a decision.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import fields
from test_gpu_chem import compare

pytestmark = pytest.mark.gpu

RTOL_PARITY = 1e-8


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _cells(mech, n=1001, seed=31):
    """Ignition cells with a cold tail, and a log-uniform step length per cell."""
    f = fields.ignition_cells(mech, n=n, seed=seed)
    f["T"][::7] = np.linspace(300.0, 480.0, f["T"][::7].size)
    rng = np.random.default_rng(seed + 1)
    f["dt"] = np.exp(rng.uniform(np.log(1e-7), np.log(2e-6), size=n))
    return f


def _run(gm, f, opts, ld=None, rr=False, dt=None):
    import paper_2210_07094_amd as df  # noqa: F401
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
    dts = torch.tensor(f["dt"] if dt is None else dt, dtype=torch.float64, device=dev)
    st = torch.full((n,), -7, dtype=torch.int32, device=dev)
    ns = torch.full((2 * n,), -7, dtype=torch.int32, device=dev)
    rrt = torch.full((K, ld), -7.0, dtype=torch.float64, device=dev) if rr else None
    gm.chem_step(T, p, Y, dts, rr=rrt, status=st, n_steps=ns, workspace=gm.workspace(n), opts=opts)
    torch.cuda.synchronize()
    out = {"T": T.cpu().numpy(), "Y": Y.cpu().numpy()[:, :n], "status": st.cpu().numpy(),
           "n_acc": ns[:n].cpu().numpy(), "n_rej": ns[n:].cpu().numpy()}
    if rr:
        out["rr"] = rrt.cpu().numpy()[:, :n]
    return out


SCHEDULES = [
    ("static, one cell per lane", dict(schedule=1, mapping=1)),
    ("static, 16 lanes per cell", dict(schedule=1, mapping=2)),
    ("static, 32 lanes per cell", dict(schedule=1, mapping=4)),
    ("static, 32 lanes for the head of the cost order, 16 for the rest", dict(schedule=1, mapping=5)),
    ("queue, all waves 16-lane groups", dict(schedule=2, coop_blocks=0)),
    ("queue, 8 waves 16-lane groups from the start", dict(schedule=2, coop_blocks=8)),
    ("queue, every wave first takes cold cells per lane", dict(schedule=2, coop_blocks=-1)),
]


@pytest.mark.parametrize("label,kw", SCHEDULES, ids=[s[0] for s in SCHEDULES])
def test_per_cell_dt_parity(h2_path, h2_mech, h2_oracle, label, kw):
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = _cells(h2_mech)
    g = _run(gm, f, df.chem_opts(**kw), ld=1100, rr=True)
    o = h2_oracle.chem_step(f["T"], f["p"], f["Y"], f["dt"], h_inout=np.zeros(f["T"].size), want_rr=True)
    assert np.array_equal(g["status"], o["status"]), label
    worst, flipped, tol_err = compare(g, o)
    assert worst <= RTOL_PARITY, f"{label}: {worst:.3e}"
    assert flipped <= 3 and tol_err <= 10.0, (label, flipped, tol_err)
    # rr = rho0 (Y - Y0) / dt of each cell's own step length
    ok = (g["n_acc"] == o["n_acc"]) & (g["n_rej"] == o["n_rej"])
    scale = np.abs(o["rr"]).max(axis=0) + 1e-300
    assert np.max(np.abs(g["rr"] - o["rr"])[:, ok] / scale[ok]) < 1e-6


def test_unusable_step_lengths(h2_path, h2_mech):
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = _cells(h2_mech, n=200)
    dt = f["dt"].copy()
    bad = [3, 50, 51, 199]
    dt[bad] = [0.0, -1e-6, np.nan, np.inf]
    for kw in (dict(schedule=1, mapping=2), dict(schedule=1, mapping=1), dict(schedule=2, coop_blocks=-1)):
        g = _run(gm, f, df.chem_opts(**kw), rr=True, dt=dt)
        assert np.all(g["status"][bad] == df.CELL_NONFINITE), kw
        assert np.array_equal(g["T"][bad], f["T"][bad]) and np.array_equal(g["Y"][:, bad], f["Y"][:, bad])
        assert np.all(g["n_acc"][bad] == 0) and np.all(g["rr"][:, bad] == 0.0)
        good = np.setdiff1d(np.arange(200), bad)
        assert np.all(g["status"][good] == df.CELL_OK), kw


def test_queue_equals_static_bitwise(h2_path, h2_mech):
    """The 16-lane body does the same arithmetic for a cell whichever group takes it, and the
    32-lane layout (the second 16 lanes taking half the rate constants) the same as the 16-lane
    one, also when only the head of the cost order (512 of the 4096 cells) takes it."""
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = fields.hot_kernel_field_2d(h2_mech, nx=64, ny=64)
    f["dt"] = np.full(f["T"].size, 1e-6)
    a = _run(gm, f, df.chem_opts(schedule=1, mapping=2))
    b = _run(gm, f, df.chem_opts(schedule=2, coop_blocks=0))
    c = _run(gm, f, df.chem_opts(schedule=2, coop_blocks=5))
    d = _run(gm, f, df.chem_opts(schedule=1, mapping=4))
    e = _run(gm, f, df.chem_opts(schedule=1, mapping=5))
    z = _run(gm, f, df.chem_opts(schedule=1, mapping=0))
    for k in ("status", "n_acc", "n_rej", "T", "Y"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], d[k]), k
        assert np.array_equal(a[k], e[k]), k
        assert np.array_equal(a[k], z[k]), k
    # with five group waves the cold cells go one per lane first (rounding may differ there);
    # the hot cells go to 16-lane groups in every schedule: bitwise equal results
    assert np.array_equal(a["status"], c["status"])
    hot = f["T"] > 600.0
    assert hot.sum() > 100
    for k in ("n_acc", "n_rej", "T"):
        assert np.array_equal(a[k][hot], c[k][hot]), k
    assert np.array_equal(a["Y"][:, hot], c["Y"][:, hot])


@pytest.mark.parametrize("n", [300, 1])
def test_head_variant_smaller_than_its_head(h2_path, h2_mech, n):
    """Fewer cells than the 32-lane head of the cost order (512): every cell is a 32-lane cell and
    no 16-lane block runs; same bits as 16 lanes per cell."""
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = _cells(h2_mech, n=n, seed=17)
    print(f"case: head variant, {n} cells", flush=True)
    a = _run(gm, f, df.chem_opts(schedule=1, mapping=2))
    e = _run(gm, f, df.chem_opts(schedule=1, mapping=5))
    for k in ("status", "n_acc", "n_rej", "T", "Y"):
        assert np.array_equal(a[k], e[k]), k
    assert np.all(a["status"] == df.CELL_OK)


def test_queue_needs_workspace(h2_path, h2_mech):
    import paper_2210_07094_amd as df
    torch = _torch()
    gm = df.Mechanism(h2_path)
    f = _cells(h2_mech, n=64)
    T = torch.tensor(f["T"], device="cuda:0")
    p = torch.tensor(f["p"], device="cuda:0")
    Y = torch.tensor(f["Y"], device="cuda:0")
    with pytest.raises(df.DfError):
        gm.chem_step(T, p, Y, 1e-6, workspace=None, opts=df.chem_opts(schedule=2))


def test_mixing_layer_full_size_sampled(h2_path, h2_mech, h2_oracle):
    """The 1,000,000-cell mixing layer with per-cell dt, queue schedule as the benchmark runs
    it; the oracle integrates a sample of cells one by one (the 500 hottest and 1000 random)."""
    import paper_2210_07094_amd as df
    gm = df.Mechanism(h2_path)
    f = fields.mixing_layer_3d(h2_mech)
    g = _run(gm, f, df.chem_opts(schedule=2))
    assert np.all(g["status"] == df.CELL_OK)
    rng = np.random.default_rng(9)
    n = f["T"].size
    idx = np.unique(np.concatenate([np.argsort(f["T"])[-500:], rng.choice(n, 1000, replace=False)]))
    o = h2_oracle.chem_step(f["T"][idx], f["p"][idx], f["Y"][:, idx], f["dt"][idx], h_inout=np.zeros(idx.size))
    gs = {k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in g.items()}
    worst, flipped, tol_err = compare(gs, o)
    assert worst <= RTOL_PARITY, worst
    assert flipped <= 10 and tol_err <= 10.0, (flipped, tol_err)


def test_autotune_picks_a_valid_schedule(h2_path, h2_mech, h2_oracle):
    import paper_2210_07094_amd as df
    torch = _torch()
    gm = df.Mechanism(h2_path)
    f = _cells(h2_mech, n=2048, seed=5)
    dev = "cuda:0"
    T = torch.tensor(f["T"], device=dev)
    p = torch.tensor(f["p"], device=dev)
    Y = torch.tensor(f["Y"], device=dev)
    dt = torch.tensor(f["dt"], device=dev)
    o = gm.autotune(T, p, Y, dt)
    torch.cuda.synchronize()
    assert o.schedule in (1, 2) and o.coop_blocks >= -1 and o.mapping in (0, 1, 4)
    # inputs untouched
    assert np.array_equal(T.cpu().numpy(), f["T"]) and np.array_equal(Y.cpu().numpy(), f["Y"])
    g = _run(gm, f, o)
    ro = h2_oracle.chem_step(f["T"], f["p"], f["Y"], f["dt"], h_inout=np.zeros(f["T"].size))
    worst, flipped, tol_err = compare(g, ro)
    assert worst <= RTOL_PARITY and flipped <= 3 and tol_err <= 10.0
