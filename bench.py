"""Benchmark of the per-cell chemistry step on one MI355X.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu]

Workload: the 256 x 256 = 65,536-cell hot-kernel field (premixed H2/air at
phi = 1, 300 K background with eight Gaussian hot kernels up to 1800 K,
p = 1 atm) with the seeded 9-species / 24-reaction mechanism, dt = 1 us.
One step is one pass of the whole hot path over the field: the FP64
RODAS4 integrator (df_chem_step) and the BF16 DNN step with its FP64
fallback (df_dnn_step), each starting from the same resident input state.
`value` is cells per second of that step; the per-form rates, the DNN's
error against the oracle integrator, the roofline of the dominant kernel
and the oracle timed on the host cores are printed in the same JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MECH = os.path.join(ROOT, "synth", "data", "h2_synth_9sp_24r.mech")
HC_MECH = os.path.join(ROOT, "synth", "data", "hc_synth_53sp_325r.mech")
DNN_W = os.path.join(ROOT, "paper_2210_07094_amd", "data", "h2_dnn_1600_800_400.dfdnn")
DT = 1e-6

# MI355X peaks (datasheet): FP64 vector 78.6 TFLOP/s = 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA);
# dense BF16 MFMA 2.5 PFLOP/s
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0

# cost of operations without a native FP64 instruction, in FP64 lane-ops (an FMA is one lane-op)
TRANSCENDENTAL_OPS = 25
DIVISION_OPS = 10


def integrator_lane_ops(mech):
    """Algorithmic FP64 lane-ops of one RODAS4 attempt (Jacobian, LU, 6 stages, error test).

    Counted from the method's steps for the given mechanism (not from the
    instructions the compiler emitted): polynomial thermo, rate constants,
    mass action, third-body sums, Troe falloff, analytic Jacobian in
    concentration space and its mapping to (T, Y), LU of the N x N iteration
    matrix, six triangular solves, stage combinations and the error norm.
    """
    K, M = mech.n_species, mech.n_reactions
    N = K + 1
    T_, D_ = TRANSCENDENTAL_OPS, DIVISION_OPS
    nu = mech.nu_prod - mech.nu_reac
    nnz = (nu != 0).sum(axis=1)
    n_tb = int(np.count_nonzero(mech.reaction_type != 0))
    n_troe = int(np.count_nonzero(mech.reaction_type == 2))
    thermo = K * (18 + T_ + D_)                       # cp, h, s polynomials; exp(-G/RT) and its inverse; sums
    mixture = T_ + 3 * D_ + 4 + 2 * K                  # log T, 1/T, mean molar mass, density, p0/RT, concentrations
    rates = int(np.sum(41 + nnz)) + n_tb * (K + 1)     # kf, Kc, mass action, q, accumulation; [M]
    troe = n_troe * (7 * T_ + 4 * D_ + 25)
    out = 3 * K + 4 + D_
    rhs = thermo + mixture + rates + troe + out
    jac_extra = int(np.sum(41 + nnz * (K + 3))) + n_tb * K + n_troe * (32 + D_) + K * (2 * K + 6) + N * (K + 2) + \
        3 * K + D_
    jac = rhs + jac_extra
    lu = sum(j + j * j for j in range(N)) + N * D_
    solves = 6 * N * N
    form_w = N * N + D_
    stages = 15 * N * 2 + 5 * N + N + N * (5 + D_) + 2 * T_
    total = 5 * rhs + jac + lu + solves + form_w + stages
    return {"per_attempt": int(total), "rhs": int(rhs), "jacobian": int(jac), "lu": int(lu), "solves": int(solves),
            "stage_ops": int(stages + form_w)}


# HBM traffic of the integrator kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this
# benchmark scaled by what the same counters read for the benchmark's plain copy kernels
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "chem_coop_head_kernel_field65536_traffic.txt")
KERNEL_SOURCES = ["df_chem_coop.hip", "df_kinetics.h", "df_internal.h"]


def kernel_sources_sha256():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2210_07094_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Bytes per launch from the committed counter summary, or None when the kernel
    sources have changed since the counters were taken (or no summary exists)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return float(kv["traffic_bytes_per_launch"])


def mlp_flops(dims):
    return 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:]))


def dnn_error(T0, Y0, Td, Yd, To, Yo, status):
    """DNN result against the oracle integrator on the same inputs."""
    dT = np.abs(Td - To)
    dY = np.abs(Yd - Yo)
    inc_o = Yo - Y0
    inc_d = Yd - Y0
    rel_l2 = []
    for k in range(Y0.shape[0]):
        m = np.abs(inc_o[k]) > 1e-8
        rel_l2.append(float(np.linalg.norm(inc_d[k, m] - inc_o[k, m]) / np.linalg.norm(inc_o[k, m])) if m.any()
                      else None)
    return {"max_abs_dT_K": float(dT.max()), "mean_abs_dT_K": float(dT.mean()),
            "max_abs_dY_per_species": [float(v) for v in dY.max(axis=1)],
            "rel_l2_dY_increment_per_species": rel_l2,
            "fallback_frac": float(np.mean(status == 4))}


def batching_study(gm, mech_h, dev):
    """Uneven stiffness: the 100^3 = 1,000,000-cell mixing layer with a step length per cell
    (log-uniform 1e-7..1e-5 s), integrated with the naive schedule (one launch, one cell per
    lane, index order), the static 16-lane schedule in cost order, and the schedule the
    autotuner picks (persistent work queue for this workload)."""
    import torch
    import paper_2210_07094_amd as df
    from synth import fields
    f = fields.mixing_layer_3d(mech_h)
    n = f["T"].size
    T0 = torch.tensor(f["T"], dtype=torch.float64, device=dev)
    p = torch.tensor(f["p"], dtype=torch.float64, device=dev)
    Y0 = torch.tensor(f["Y"], dtype=torch.float64, device=dev)
    dts = torch.tensor(f["dt"], dtype=torch.float64, device=dev)
    ws = gm.workspace(n)
    ns = torch.zeros(2 * n, dtype=torch.int32, device=dev)
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def timed(opts, use_ws, reps):
        ms = []
        for _ in range(reps):
            T, Y = T0.clone(), Y0.clone()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gm.chem_step(T, p, Y, dts, status=st, n_steps=ns, workspace=ws if use_ws else None, opts=opts,
                         stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(min(ms))

    naive = timed(df.chem_opts(schedule=1, mapping=1), False, 1)
    static = timed(df.chem_opts(schedule=1, mapping=2), True, 2)
    tuned = gm.autotune(T0, p, Y0, dts)
    queue = timed(tuned, True, 3)
    nsh = ns.cpu().numpy()
    return {"workload": "mixing layer 100^3 = 1,000,000 cells, H2/N2 fuel vs air, T 300-2500 K, "
                        "dt per cell log-uniform 1e-7..1e-5 s", "n_cells": n,
            "attempts_total": int(nsh.sum()), "accepted_max": int(nsh[:n].max()),
            "status_counts": np.bincount(st.cpu().numpy()).tolist(),
            "naive_one_cell_per_lane_ms": naive, "static_16_lanes_cost_order_ms": static,
            "autotuned": {"schedule": int(tuned.schedule), "coop_blocks": int(tuned.coop_blocks), "ms": queue},
            "cells_per_s_autotuned": n / (queue * 1e-3), "speedup_vs_naive": naive / queue}


def adjoint_lane_ops(mech, ops):
    """Algorithmic FP64 lane-ops of the reverse sweep per accepted sub-step: the five stage
    states and the analytic Jacobian at each, six products with W^-T and five with J^T (N^2
    each), the first-order ln A terms of five stages (per species the production-rate weight,
    per reaction the seed through the stoichiometry and the factor of d q / d ln A), six
    second-order products in dual-number arithmetic, and the stage-adjoint updates.  A
    vector-Jacobian product is the right-hand side plus its reverse accumulation (per
    reaction: the seed through the stoichiometry, the temperature and slot derivatives, the
    third-body term, the falloff derivatives; per species: the mixture terms); dual numbers
    cost 3 lane-ops per operation."""
    K, M = mech.n_species, mech.n_reactions
    N = K + 1
    nu = mech.nu_prod - mech.nu_reac
    nnz = (nu != 0).sum(axis=1)
    n_tb = int(np.count_nonzero(mech.reaction_type != 0))
    n_troe = int(np.count_nonzero(mech.reaction_type == 2))
    reverse = int(np.sum(nnz + 25)) + n_tb * K + n_troe * (30 + 4 * DIVISION_OPS) + 20 * K
    vjp = ops["rhs"] + reverse
    lna = 3 * K + int(np.sum(nnz + 1))
    per_substep = 5 * (5 * N + ops["jacobian"] + lna) + 11 * N * N + 6 * 3 * vjp + 30 * N
    return {"per_substep": int(per_substep), "vjp": int(vjp)}


def adjoint_study(gm, mech_h, dev, with_cpu, threads):
    """Differentiation workload: 4096 cells, T0 1000-1600 K, phi 0.5-2, p = 1 atm, dt = 1e-5 s.
    The taped step (16 lanes per cell, recording the stage tape), one reverse sweep (the
    gradient of a scalar loss with respect to T0, Y0 and every ln A), and the full 10 x 34
    Jacobian per cell (one sweep per output component); the oracle's forward sensitivities
    (complex-step differentiation of its replay) on a sample of cells for the CPU rate."""
    import torch
    from synth import fields
    n = 4096
    dt = 1e-5
    cap = 1024
    f = fields.ignition_cells(mech_h, n=n, seed=2023)
    K = mech_h.n_species
    T0 = torch.tensor(f["T"], dtype=torch.float64, device=dev)
    p = torch.tensor(f["p"], dtype=torch.float64, device=dev)
    Y0 = torch.tensor(np.ascontiguousarray(f["Y"]), dtype=torch.float64, device=dev)
    ns = torch.zeros(2 * n, dtype=torch.int32, device=dev)
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    rng = np.random.default_rng(0)
    Tb = torch.tensor(rng.standard_normal(n), dtype=torch.float64, device=dev)
    Yb = torch.tensor(rng.standard_normal((K, n)), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    taped, sweep = [], []
    for it in range(3):
        T, Y = T0.clone(), Y0.clone()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        tape = gm.chem_step_taped(T, p, Y, dt, max_substeps=cap, status=st, n_steps=ns, stream=stream)
        e[1].record(stream)
        gm.chem_adjoint(p, tape, cap, Tb, Yb, stream=stream)
        e[2].record(stream)
        torch.cuda.synchronize()
        if it > 0:
            taped.append(e[0].elapsed_time(e[1]))
            sweep.append(e[1].elapsed_time(e[2]))
    t_tape, t_sweep = float(np.mean(taped)), float(np.mean(sweep))
    nsh = ns.cpu().numpy()
    acc = int(nsh[:n].sum())
    aops = adjoint_lane_ops(mech_h, integrator_lane_ops(mech_h))
    tflops = 2.0 * aops["per_substep"] * acc / (t_sweep * 1e-3) / 1e12
    out = {"workload": "4096 ignition cells, T0 1000-1600 K, phi 0.5-2, p=1 atm, dt=1e-5 s; gradients of "
                       "(T, Y) at dt w.r.t. T0, Y0 and 24 ln A on the frozen sub-step sequence",
           "n_cells": n, "accepted_total": acc, "accepted_max": int(nsh[:n].max()),
           "status_counts": np.bincount(st.cpu().numpy()).tolist(),
           "taped_step_ms": t_tape, "reverse_sweep_ms": t_sweep,
           "gradient_cells_per_s": n / ((t_tape + t_sweep) * 1e-3),
           "full_jacobian_cells_per_s": n / ((t_tape + (K + 1) * t_sweep) * 1e-3),
           "roofline": {"bound": "alu", "kernel": "adjoint_kernel<9> (FP64 VALU, 8 lanes per cell)",
                        "achieved": tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": tflops / PEAK_FP64_TFLOPS, "traffic": None, "lane_ops": aops}}
    if with_cpu:
        import oracle
        from oracle import sensitivity as sens
        om = oracle.Mech(MECH)
        kin = sens.Kinetics(mech_h)
        tab = oracle.rodas4_tableau()
        sample = [0, 1, 2]
        t1 = time.perf_counter()
        for i in sample:
            _, _, _, hs, _ = om.record(f["T"][i], f["p"][i], f["Y"][:, i], dt)
            sens.sensitivities(kin, tab, f["p"][i], np.concatenate([[f["T"][i]], f["Y"][:, i]]), hs)
        t_cpu = time.perf_counter() - t1
        out["cpu_oracle"] = {"value": len(sample) / t_cpu, "unit": "cells/s (full 10 x 34 Jacobian)", "cores": 1,
                             "kind": "oracle", "sample": f"forward sensitivities of cells {sample} ({t_cpu:.1f} s)"}
    return out


def training_study(gm, dnn_path, mech_h, dev):
    """Adam steps of the DNN on device-generated pairs: 8192 states (ignition cells and hotter
    states) advanced by the integrator over the network's dt, turned into (input, target) rows.
    The stored network already fits such pairs to the bf16 noise of its output, so the study
    first halves the output layer's weights and then times the steps that recover it (forward,
    loss, backward, Adam).  FLOPs of a step: the forward products, and twice as many backward
    (data and weight gradients)."""
    import torch
    import paper_2210_07094_amd as df
    from synth import fields
    dnn = df.DNN(dnn_path, gm)
    n = 8192
    f = fields.ignition_cells(mech_h, n=n, seed=99)
    f["T"][: n // 2] = np.random.default_rng(2).uniform(900.0, 2400.0, n // 2)
    p = torch.tensor(f["p"], device=dev)
    T0 = torch.tensor(f["T"], device=dev)
    Y0 = torch.tensor(np.ascontiguousarray(f["Y"]), device=dev)
    T1, Y1 = T0.clone(), Y0.clone()
    gm.chem_step(T1, p, Y1, dnn.dt_train, h=torch.zeros(n, dtype=torch.float64, device=dev))
    tr = df.Trainer(dnn, n)
    x, t, v = tr.make_batch(p, T0, Y0, Y1)
    keep = v.bool()
    x, t = x[keep].contiguous(), t[keep].contiguous()
    B = int(x.shape[0])
    Lo = len(dnn.dims) - 2
    tr.set(Lo, "W", 0.5 * tr.get(Lo, "W"))
    opts = df.adam_opts(lr=2e-4)
    stream = torch.cuda.current_stream()
    losses = []
    for _ in range(3):
        losses.append(float(tr.step(x, t, opts=opts).cpu()[0]))
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        last = tr.step(x, t, opts=opts)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 3.0 * mlp_flops(dnn.dims) * B
    tflops = flops / (ms * 1e-3) / 1e12
    return {"workload": "Adam steps (lr 2e-4) of the 11-1600-800-400-9 network, output layer halved first, on "
                        "pairs the integrator made from 8192 states (dt = network dt); batch = the states inside "
                        "the training box",
            "batch": B, "ms_per_step": ms, "samples_per_s": B / (ms * 1e-3),
            "loss_first": losses[0], "loss_after_13_steps": float(last.cpu()[0]),
            "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / PEAK_BF16_TFLOPS}}


def large_mechanism_study(dev, with_cpu, threads, n=65536):
    """The 53-species / 325-reaction hydrocarbon mechanism on one wavefront per cell: one
    chemistry step (dt = 1 us) of n cells of the hydrocarbon field recipe (T 300-2400 K,
    p 1-10 atm, CH4/air unburnt/product blend with log-uniform minor species).  FLOPs are the
    method's algorithmic lane-ops per attempt for this mechanism times the attempts the step
    made (an FMA counts 2).  The oracle is timed on 16 cells spread over the temperature range."""
    import torch
    import synth
    import paper_2210_07094_amd as df
    from synth import fields
    mech = synth.read_mech(HC_MECH)
    gm = df.Mechanism(HC_MECH)
    f = fields.hydrocarbon_field(mech, n=n)
    T0 = torch.tensor(f["T"], device=dev)
    p = torch.tensor(f["p"], device=dev)
    Y0 = torch.tensor(f["Y"], device=dev)
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    ns = torch.zeros(2 * n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    w = 2048
    gm.chem_step(T0[:w].clone(), p[:w], Y0[:, :w].clone(), DT)   # first launch
    T, Y = T0.clone(), Y0.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    gm.chem_step(T, p, Y, DT, status=st, n_steps=ns, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nsn = ns.cpu().numpy()
    attempts = int(nsn.sum())
    ops = integrator_lane_ops(mech)
    tflops = 2.0 * ops["per_attempt"] * attempts / (ms * 1e-3) / 1e12
    out = {"workload": f"hydrocarbon field recipe, {n} cells, 53 species / 325 reactions (seeded), dt = 1 us, "
                       "one wavefront per cell",
           "n_cells": n, "ms": ms, "cells_per_s": n / (ms * 1e-3), "attempts": attempts,
           "attempts_per_s": attempts / (ms * 1e-3), "accepted_mean": float(nsn[:n].mean()),
           "accepted_max": int(nsn[:n].max()), "status_counts": np.bincount(st.cpu().numpy()).tolist(),
           "roofline": {"bound": "alu", "kernel": "chem_wave_kernel<53> (FP64 VALU, one wavefront per cell)",
                        "achieved": tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": tflops / PEAK_FP64_TFLOPS, "lane_ops_per_attempt": ops}}
    # the DNN form at this size: a 55-3200-1600-800-53 BF16 network with seeded weights (no
    # trained network exists for this mechanism), its training box around the field
    import tempfile
    from synth import dnnfile
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "hc.dfdnn")
        dnnfile.write_seeded_network(path, mech.n_species, f["T"], f["p"], f["Y"], (3200, 1600, 800), seed=3)
        dnn = df.DNN(path, gm)
    ws = dnn.workspace(n)
    std = torch.zeros(n, dtype=torch.int32, device=dev)
    T, Y = T0.clone(), Y0.clone()
    dnn.step(T, p, Y, DT, status=std, workspace=ws, stream=stream)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        T.copy_(T0)
        Y.copy_(Y0)
        dnn.step(T, p, Y, DT, status=std, workspace=ws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_dnn = e0.elapsed_time(e1) / reps
    dflops = mlp_flops(dnn.dims) * n
    dt_ = dflops / (ms_dnn * 1e-3) / 1e12
    out["bf16_dnn"] = {"network": "55-3200-1600-800-53, seeded weights", "ms": ms_dnn,
                       "cells_per_s": n / (ms_dnn * 1e-3), "tflops": dt_, "mfma_frac": dt_ / PEAK_BF16_TFLOPS,
                       "fallback_frac": float((std == 4).float().mean()),
                       "speedup_vs_fp64_integrator": ms / ms_dnn}
    # the same network with its hidden-to-hidden layers in FP8
    fp8_opts = df.dnn_opts(precision=1)
    Tb, Yb = T.clone(), Y.clone()
    T.copy_(T0)
    Y.copy_(Y0)
    dnn.step(T, p, Y, DT, status=std, workspace=ws, stream=stream, opts=fp8_opts)
    torch.cuda.synchronize()
    dY = float((Y - Yb).abs().max())
    e0.record(stream)
    for _ in range(reps):
        T.copy_(T0)
        Y.copy_(Y0)
        dnn.step(T, p, Y, DT, status=std, workspace=ws, stream=stream, opts=fp8_opts)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fp8 = e0.elapsed_time(e1) / reps
    out["fp8_dnn"] = {"network": "55-3200-1600-800-53, 1600x3200 and 800x1600 layers in E4M3FN", "ms": ms_fp8,
                      "cells_per_s": n / (ms_fp8 * 1e-3), "tflops": dflops / (ms_fp8 * 1e-3) / 1e12,
                      "speedup_vs_bf16_dnn": ms_dnn / ms_fp8, "max_abs_dY_vs_bf16_dnn": dY}
    if with_cpu:
        import oracle
        om = oracle.Mech(HC_MECH)
        idx = np.argsort(f["T"])[np.linspace(0, n - 1, 16).astype(int)]
        t1 = time.perf_counter()
        om.chem_step(f["T"][idx], f["p"][idx], np.ascontiguousarray(f["Y"][:, idx]), DT, nthreads=threads)
        t_cpu = time.perf_counter() - t1
        out["cpu_oracle"] = {"value": idx.size / t_cpu, "unit": "cells/s", "cores": min(threads, idx.size),
                             "kind": "oracle", "sample": f"16 cells spread over the temperature range ({t_cpu:.1f} s)"}
    return out


def rollout_study(gm, dnn, mech_h, dev):
    """The paper's 0-D checks on the synthetic mechanism, as device rollouts of 1 us steps:
    the ignition delay (largest dT/dt) against T0 for stoichiometric H2/air at 1 atm from the
    integrator and from the DNN; the constant-volume case (phi = 1, 1000 K, 0.5 atm) with the
    integrator; and the time per rollout step of the constant-pressure case (phi = 1, 1400 K,
    1 atm) at several reactor counts, the paper's 0-D timing over grid sizes."""
    import torch
    from synth import fields
    R = 8.31446261815324
    Yphi = fields.premixed_h2_air(mech_h, 1.0).reshape(-1)
    W = np.asarray(mech_h.molar_mass) * 1e-3

    def cells(T0):
        n = T0.size
        Y = torch.tensor(np.ascontiguousarray(np.repeat(Yphi[:, None], n, axis=1)), device=dev)
        return torch.tensor(T0, device=dev), Y

    T0 = np.linspace(1000.0, 1500.0, 21)
    p = torch.full((T0.size,), 101325.0, dtype=torch.float64, device=dev)
    steps = 2000
    T, Y = cells(T0)
    idt_i, _ = gm.rollout(T, p, Y, 1e-6, steps)
    T, Y = cells(T0)
    idt_d, _ = gm.rollout(T, p, Y, 1e-6, steps, dnn=dnn)
    ii, dd = idt_i.cpu().numpy(), idt_d.cpu().numpy()
    both = np.isfinite(ii) & np.isfinite(dd)
    rel = np.abs(dd[both] - ii[both]) / ii[both]
    # constant volume: phi = 1, 1000 K, 0.5 atm
    rho = 0.5 * 101325.0 / (R * 1000.0 * np.sum(Yphi / W))
    T, Y = cells(np.array([1000.0]))
    idt_v, traj_v = gm.rollout(T, torch.tensor([rho], device=dev), Y, 1e-6, 2500, trajectory=True,
                               constant_volume=True)
    Yv = Y.cpu().numpy()[:, 0]
    Tv_end = float(T.cpu()[0])
    p_end = rho * R * Tv_end * np.sum(Yv / W)
    # time per rollout step of the 1400 K constant-pressure reactor, n copies
    timing = []
    stream = torch.cuda.current_stream()
    for n in (1, 1024, 65536):
        row = {"reactors": n}
        for name, net in (("integrator", None), ("dnn", dnn)):
            pn = torch.full((n,), 101325.0, dtype=torch.float64, device=dev)
            T, Y = cells(np.full(n, 1400.0))
            gm.rollout(T, pn, Y, 1e-6, 5, dnn=net)
            T, Y = cells(np.full(n, 1400.0))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gm.rollout(T, pn, Y, 1e-6, 100, dnn=net)
            e1.record(stream)
            torch.cuda.synchronize()
            row[f"{name}_ms_per_step"] = e0.elapsed_time(e1) / 100
        row["dnn_speedup"] = row["integrator_ms_per_step"] / row["dnn_ms_per_step"]
        timing.append(row)
    return {"workload": "0-D H2/air rollouts, 1 us steps: delay curve phi=1 1 atm T0 1000-1500 K (21 reactors, "
                        "2 ms); constant volume phi=1 1000 K 0.5 atm (2.5 ms); time per step of the 1400 K "
                        "reactor (100 steps) at 1, 1024, 65536 copies",
            "idt_curve": {"T0_K": T0.tolist(), "integrator_s": [None if not np.isfinite(v) else float(v) for v in ii],
                          "dnn_s": [None if not np.isfinite(v) else float(v) for v in dd]},
            "dnn_idt_rel_err": {"median": float(np.median(rel)) if rel.size else None,
                                "max": float(rel.max()) if rel.size else None,
                                "within_10pct": int(np.sum(rel <= 0.1)), "compared": int(both.sum()),
                                "dnn_no_ignition": int(np.sum(np.isfinite(ii) & ~np.isfinite(dd)))},
            "constant_volume": {"idt_s": float(idt_v.cpu()[0]), "T_end_K": Tv_end,
                                "T_max_rise_K": float((traj_v[:, 0] - traj_v[0, 0]).max().cpu()),
                                "p_end_over_p0": p_end / (0.5 * 101325.0)},
            "time_per_step": timing}


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def cpu_leg(out_path, threads):
    """The oracle timed on the host (run in a child process with the -O3 -march=native build): the
    integrator on every cell of snapshots 0 and S and of the 1,024 ignition cells with all threads,
    the BF16-emulated DNN step on every 16th cell of each snapshot, and one thread on every 64th
    cell (integrator) and every 256th cell (DNN) of snapshot 0.  Its results are also the reference
    of the DNN error statement.  Writes the oracle states to out_path, returns the timings."""
    import oracle
    import synth
    from synth import fields
    om = oracle.Mech(MECH)
    od = oracle.DNN(DNN_W)
    mech_h = synth.read_mech(MECH)
    res, tim = {}, {}
    for name, f in (("s0", fields.hot_kernel_field_2d(mech_h)), ("sS", fields.snapshot_s()),
                    ("c1", fields.ignition_cells(mech_h))):
        t1 = time.perf_counter()
        ro = om.chem_step(f["T"], f["p"], f["Y"], DT, nthreads=threads)
        tim[f"{name}_integrator_s"] = time.perf_counter() - t1
        res[f"{name}_T"], res[f"{name}_Y"] = ro["T"], ro["Y"]
        if name != "c1":
            smp = np.arange(0, f["T"].size, 16)
            t1 = time.perf_counter()
            od.step(om, f["T"][smp], f["p"][smp], f["Y"][:, smp], DT, mode=1, nthreads=threads)
            tim[f"{name}_dnn_s"] = time.perf_counter() - t1
            tim[f"{name}_dnn_cells"] = int(smp.size)
        tim[f"{name}_cells"] = int(f["T"].size)
        if name == "s0":
            smp = np.arange(0, f["T"].size, 64)
            t1 = time.perf_counter()
            om.chem_step(f["T"][smp], f["p"][smp], f["Y"][:, smp], DT, nthreads=1)
            tim["s0_integrator_1core_s"], tim["s0_integrator_1core_cells"] = time.perf_counter() - t1, int(smp.size)
            smp = np.arange(0, f["T"].size, 256)
            t1 = time.perf_counter()
            od.step(om, f["T"][smp], f["p"][smp], f["Y"][:, smp], DT, mode=1, nthreads=1)
            tim["s0_dnn_1core_s"], tim["s0_dnn_1core_cells"] = time.perf_counter() - t1, int(smp.size)
    np.savez(out_path, **res)
    return tim


def run_cpu_leg(threads):
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "oracle_states.npz")
        env = dict(os.environ, DF_ORACLE_NATIVE="1", OMP_NUM_THREADS=str(threads))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", path, "--threads", str(threads)],
                           capture_output=True, text=True, env=env, timeout=1200)
        if r.returncode != 0:
            raise RuntimeError(f"cpu leg failed:\n{r.stderr[-3000:]}")
        tim = json.loads(r.stdout.strip().splitlines()[-1])
        z = np.load(path)
        return tim, {k: z[k].copy() for k in z.files}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing (cpu_baseline null)")
    ap.add_argument("--no-batching", action="store_true", help="skip the 1M-cell scheduling study")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 4096-cell adjoint study")
    ap.add_argument("--no-training", action="store_true", help="skip the DNN training study")
    ap.add_argument("--no-rollout", action="store_true", help="skip the 0-D rollout study")
    ap.add_argument("--no-large", action="store_true", help="skip the 53-species mechanism study")
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--threads", type=int, default=1, help=argparse.SUPPRESS)
    a = ap.parse_args()
    if a.cpu_leg:
        print(json.dumps(cpu_leg(a.cpu_leg, a.threads)), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {a.gpus} is not supported (cells are independent, "
              "so N GPUs would each run this benchmark on their own shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2210_07094_amd as df
    import synth
    from synth import fields

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = "cuda:0"
    mech_h = synth.read_mech(MECH)
    f = fields.hot_kernel_field_2d(mech_h)
    n = f["T"].size
    K = mech_h.n_species
    gm = df.Mechanism(MECH)
    dnn = df.DNN(DNN_W, gm)
    ops = integrator_lane_ops(mech_h)
    dnn_cell_flops = mlp_flops(dnn.dims)

    T_in = torch.tensor(f["T"], dtype=torch.float64, device=dev)
    p = torch.tensor(f["p"], dtype=torch.float64, device=dev)
    Y_in = torch.tensor(f["Y"], dtype=torch.float64, device=dev)
    Tc, Yc = T_in.clone(), Y_in.clone()
    Td, Yd = T_in.clone(), Y_in.clone()
    st_c = torch.zeros(n, dtype=torch.int32, device=dev)
    st_d = torch.zeros(n, dtype=torch.int32, device=dev)
    nsteps = torch.zeros(2 * n, dtype=torch.int32, device=dev)
    ws = dnn.workspace(n)
    chem_ws = gm.workspace(n)
    stream = torch.cuda.current_stream()
    # the two forms are independent computations on separate buffers: the DNN step runs on a
    # second stream (default priority) beside the integrator, whose tail (the stiffest cells)
    # leaves most of the chip idle
    stream2 = torch.cuda.Stream()

    def step(ev=None):
        Tc.copy_(T_in)
        Yc.copy_(Y_in)
        Td.copy_(T_in)
        Yd.copy_(Y_in)
        stream2.wait_stream(stream)
        if ev:
            ev[0].record(stream)
            ev[2].record(stream2)
        gm.chem_step(Tc, p, Yc, DT, status=st_c, n_steps=nsteps, workspace=chem_ws, stream=stream)
        dnn.step(Td, p, Yd, DT, status=st_d, workspace=ws, stream=stream2)
        if ev:
            ev[1].record(stream)
            ev[3].record(stream2)
        stream.wait_stream(stream2)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(a.steps)]
    t0 = time.perf_counter()
    for s in range(a.steps):
        step(events[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    chem_ms = np.array([e[0].elapsed_time(e[1]) for e in events])
    dnn_ms = np.array([e[2].elapsed_time(e[3]) for e in events])
    ms_step = wall * 1e3 / a.steps
    ns = nsteps.cpu().numpy()
    attempts = int(ns.sum())
    chem_tflops = 2.0 * ops["per_attempt"] * attempts / (chem_ms.mean() * 1e-3) / 1e12
    T_c, Y_c, stc = Tc.cpu().numpy(), Yc.cpu().numpy(), st_c.cpu().numpy()
    T_d, Y_d, std = Td.cpu().numpy(), Yd.cpu().numpy(), st_d.cpu().numpy()

    # each form alone on a workload (outside the timed region): the kernels' own efficiency
    fp8_opts = df.dnn_opts(precision=1)

    def forms_alone(fld, reps):
        m = fld["T"].size
        T0 = torch.tensor(fld["T"], dtype=torch.float64, device=dev)
        p0 = torch.tensor(fld["p"], dtype=torch.float64, device=dev)
        Y0 = torch.tensor(np.ascontiguousarray(fld["Y"]), dtype=torch.float64, device=dev)
        Ta, Ya = T0.clone(), Y0.clone()
        sta = torch.zeros(m, dtype=torch.int32, device=dev)
        nsa = torch.zeros(2 * m, dtype=torch.int32, device=dev)
        wsa = dnn.workspace(m)
        cwa = gm.workspace(m)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # one copy of the inputs per timed call, so that the calls run back to back as in a
        # solver's loop (the host's marshalling of one call overlaps the device's work on the
        # previous one); Ta, Ya keep the last call's result
        Tc = [T0.clone() for _ in range(reps)]
        Yc = [Y0.clone() for _ in range(reps)]

        def timed(fn):
            Ta.copy_(T0)
            Ya.copy_(Y0)
            fn(Ta, Ya)  # warm-up
            for r in range(reps):
                Tc[r].copy_(T0)
                Yc[r].copy_(Y0)
            torch.cuda.synchronize()
            e0.record(stream)
            for r in range(reps):
                fn(Tc[r], Yc[r])
            e1.record(stream)
            torch.cuda.synchronize()
            Ta.copy_(Tc[-1])
            Ya.copy_(Yc[-1])
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        res = {"n_cells": m}
        ms = timed(lambda T_, Y_: gm.chem_step(T_, p0, Y_, DT, status=sta, n_steps=nsa, workspace=cwa, stream=stream))
        at = int(nsa.cpu().numpy().sum())
        tf = 2.0 * ops["per_attempt"] * at / (ms * 1e-3) / 1e12
        res["integrator"] = {"ms": ms, "cells_per_s": m / (ms * 1e-3), "attempts": at, "tflops": tf,
                             "fp64_frac": tf / PEAK_FP64_TFLOPS,
                             "status_counts": np.bincount(sta.cpu().numpy(), minlength=5).tolist()}
        res["states_integrator"] = (Ta.cpu().numpy(), Ya.cpu().numpy())
        for key, opts in (("dnn_bf16", None), ("dnn_fp8", fp8_opts)):
            ms = timed(lambda T_, Y_: dnn.step(T_, p0, Y_, DT, status=sta, workspace=wsa, stream=stream, opts=opts))
            tf = dnn_cell_flops * m / (ms * 1e-3) / 1e12
            res[key] = {"ms": ms, "cells_per_s": m / (ms * 1e-3), "tflops": tf,
                        "mfma_frac": tf / (PEAK_BF16_TFLOPS if key == "dnn_bf16" else PEAK_FP8_TFLOPS),
                        "fallback_frac": float((sta == 4).float().mean())}
            res[f"states_{key}"] = (Ta.cpu().numpy(), Ya.cpu().numpy(), sta.cpu().numpy())
        # the DNN without renormalisation, for the error statement
        Ta.copy_(T0)
        Ya.copy_(Y0)
        dnn.step(Ta, p0, Ya, DT, status=sta, workspace=wsa, stream=stream, opts=df.dnn_opts(renormalise=0))
        torch.cuda.synchronize()
        res["states_dnn_bf16_norenorm"] = (Ta.cpu().numpy(), Ya.cpu().numpy(), sta.cpu().numpy())
        return res

    fS = fields.snapshot_s()
    f1 = fields.ignition_cells(mech_h)
    alone = {"snapshot_0": forms_alone(f, a.steps), "snapshot_s": forms_alone(fS, a.steps),
             "ignition_1024": forms_alone(f1, a.steps)}

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cpu, err = None, None
    if not a.no_cpu:
        tim, ora = run_cpu_leg(threads)
        t_int, t_dnn = tim["s0_integrator_s"], tim["s0_dnn_s"] * n / tim["s0_dnn_cells"]
        t_int1 = tim["s0_integrator_1core_s"] * n / tim["s0_integrator_1core_cells"]
        t_dnn1 = tim["s0_dnn_1core_s"] * n / tim["s0_dnn_1core_cells"]
        cpu = {"value": n / (t_int + t_dnn), "unit": "cells/s", "cores": threads, "kind": "oracle",
               "sample": f"snapshot 0: integrator on all {n} cells ({t_int:.2f} s) + BF16-emulated DNN step on every "
                         f"16th cell ({tim['s0_dnn_cells']} cells, {tim['s0_dnn_s']:.2f} s, scaled to {n}); 1 core: "
                         f"every 64th / 256th cell, scaled",
               "build": "gcc -O3 -march=native, OpenMP over cells", "cpu_model": cpu_model(),
               "integrator_cells_per_s": n / t_int, "dnn_cells_per_s": n / t_dnn,
               "integrator_cells_per_s_1core": n / t_int1, "dnn_cells_per_s_1core": n / t_dnn1,
               "snapshot_s_integrator_cells_per_s": tim["sS_cells"] / tim["sS_integrator_s"],
               "ignition_1024_integrator_cells_per_s": tim["c1_cells"] / tim["c1_integrator_s"]}
        err = {}
        for key, fld, tag in (("snapshot_0", f, "s0"), ("snapshot_s", fS, "sS")):
            To, Yo = ora[f"{tag}_T"], ora[f"{tag}_Y"]
            al = alone[key]
            err[key] = {
                "renormalised": dnn_error(fld["T"], fld["Y"], al["states_dnn_bf16"][0], al["states_dnn_bf16"][1],
                                          To, Yo, al["states_dnn_bf16"][2]),
                "not_renormalised": dnn_error(fld["T"], fld["Y"], al["states_dnn_bf16_norenorm"][0],
                                              al["states_dnn_bf16_norenorm"][1], To, Yo,
                                              al["states_dnn_bf16_norenorm"][2]),
                "fp8_renormalised": dnn_error(fld["T"], fld["Y"], al["states_dnn_fp8"][0], al["states_dnn_fp8"][1],
                                              To, Yo, al["states_dnn_fp8"][2])}
            Tg, Yg = al["states_integrator"]
            relT = np.abs(Tg - To) / To
            mask = Yo > 1e-10
            relY = np.where(mask, np.abs(Yg - Yo) / np.where(mask, Yo, 1.0), 0.0)
            err[key]["integrator_max_rel_vs_oracle"] = float(max(relT.max(), relY.max()))
        To, Yo = ora["c1_T"], ora["c1_Y"]
        Tg, Yg = alone["ignition_1024"]["states_integrator"]
        err["ignition_1024_integrator_max_rel_vs_oracle"] = float(max(
            (np.abs(Tg - To) / To).max(),
            np.where(Yo > 1e-10, np.abs(Yg - Yo) / np.where(Yo > 1e-10, Yo, 1.0), 0.0).max()))
    for v in alone.values():
        for k in [k for k in v if k.startswith("states_")]:
            del v[k]

    batching = None if a.no_batching else batching_study(gm, mech_h, dev)
    adjoint = None if a.no_adjoint else adjoint_study(gm, mech_h, dev, not a.no_cpu, threads)
    training = None if a.no_training else training_study(gm, DNN_W, mech_h, dev)
    rollouts = None if a.no_rollout else rollout_study(gm, dnn, mech_h, dev)
    large = None if a.no_large else large_mechanism_study(dev, not a.no_cpu, threads, n=262144)

    s0 = alone["snapshot_0"]
    summary = {
        "value_is": "cells/s of one step = the 65,536-cell field through both forms (integrator and DNN "
                    "overlapped on two streams)",
        "integrator_cells_per_s": n / (chem_ms.mean() * 1e-3), "integrator_fp64_frac": chem_tflops / PEAK_FP64_TFLOPS,
        "integrator_alone_cells_per_s": s0["integrator"]["cells_per_s"],
        "dnn_bf16_alone_cells_per_s": s0["dnn_bf16"]["cells_per_s"], "dnn_bf16_mfma_frac": s0["dnn_bf16"]["mfma_frac"],
        "dnn_fp8_alone_cells_per_s": s0["dnn_fp8"]["cells_per_s"], "dnn_fp8_mfma_frac": s0["dnn_fp8"]["mfma_frac"],
        "snapshot_s_integrator_cells_per_s": alone["snapshot_s"]["integrator"]["cells_per_s"],
        "snapshot_s_dnn_bf16_cells_per_s": alone["snapshot_s"]["dnn_bf16"]["cells_per_s"],
        "ignition_1024_integrator_cells_per_s": alone["ignition_1024"]["integrator"]["cells_per_s"],
        "ignition_1024_dnn_bf16_cells_per_s": alone["ignition_1024"]["dnn_bf16"]["cells_per_s"],
        "dnn_max_abs_dT_K": None if err is None else {k: err[k]["renormalised"]["max_abs_dT_K"]
                                                      for k in ("snapshot_0", "snapshot_s")},
    }
    out = {
        "metric": "cells/s per chemistry step: FP64 stiff integrator vs BF16 DNN at stated error",
        "value": n / (ms_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+bf16",
        "data": "synthetic",
        "config": {"workload": "both forms per step: FP64 RODAS4 integrator + BF16 DNN 11-1600-800-400-9 (FP64 "
                               "fallback), overlapped on 2 streams; hot-kernel field 256x256=65536 cells, snapshot 0, "
                               "H2/air phi=1, 9 species/24 reactions (seeded), p=1 atm, dt=1e-6 s",
                   "n_cells": n, "dt": DT, "rtol": 1e-8, "mechanism": os.path.basename(MECH),
                   "dnn": os.path.basename(DNN_W), "snapshot": "0 (as generated)"},
        "roofline": {"bound": "alu", "kernel": "chem_coop_head_kernel<9, 2> (FP64 VALU, 32 lanes per cell for the 512 hottest cells, 16 for the rest)",
                     "achieved": chem_tflops,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": chem_tflops / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(), "lane_ops_per_attempt": ops["per_attempt"],
                     "forms": {"integrator_in_step": {"ms": float(chem_ms.mean()),
                                                      "cells_per_s": n / (chem_ms.mean() * 1e-3),
                                                      "fp64_frac": chem_tflops / PEAK_FP64_TFLOPS,
                                                      "attempts": attempts},
                               "dnn_bf16_in_step": {"ms": float(dnn_ms.mean()),
                                                    "cells_per_s": n / (dnn_ms.mean() * 1e-3),
                                                    "mfma_frac": dnn_cell_flops * n / (dnn_ms.mean() * 1e-3) / 1e12 /
                                                    PEAK_BF16_TFLOPS},
                               **{k: {f: {kk: (round(vv, 6) if isinstance(vv, float) else vv)
                                          for kk, vv in v[f].items() if kk != "status_counts"}
                                      for f in ("integrator", "dnn_bf16", "dnn_fp8")}
                                  for k, v in alone.items()}}},
        "cpu_baseline": cpu,
        "dnn_error_vs_oracle_integrator": err,
        "step_status_counts": {"integrator": np.bincount(stc, minlength=5).tolist(),
                               "dnn_bf16": np.bincount(std, minlength=5).tolist()},
        "forms_alone": alone,
        "batching_mixing_layer": batching,
        "adjoint": adjoint,
        "dnn_training": training,
        "rollouts_0d": rollouts,
        "large_mechanism": large,
        "summary": summary,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
