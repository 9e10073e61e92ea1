#!/usr/bin/env python3
"""Throughput benchmark of the gfx950 Lagrange-flux library on one GPU.

Workload: the periodic Kelvin-Helmholtz shear layer at 16384^2 cells (rho 2
with u = 0.5 inside |y - 1/2| < 1/4, rho 1 with u = -0.5 outside, p = 2.5,
v = 0.01 sin(4 pi x)), synthetic inputs built on the device.  A step is one
full Heun step of the scheme (predictor, corrector, the CFL reduction of
the new state and the device-side dt update) through lf_advance, which runs
it as one single-pass kernel per step.

Prints ONE JSON line on stdout: the FP64 cell-updates/s as ``value``; the
roofline of the dominant kernel (the single-pass step, bound by VALU issue)
and of the two-stage design's corrector against HBM, each from HIP events
on the stream the kernel runs on; the FP32 path, the two-stage path, the
mass-fraction runs, the four-quadrant problem at 8192^2, the isentropic
vortex at 4096^2 (rate and error against the exact solution), one strip
of the 16384^2 grid split into 8 (lf_step_halo with its ghost rows: one
GPU's share) and the adjoint (lf_adjoint_step and the checkpointed full
gradient at 4096^2) as extra objects; a plain device copy's bandwidth beside the rooflines; and
the FP64 CPU oracle timed on a bounded sample on this host (all threads,
and one thread).

  python bench.py [--gpus 1] [--steps K] [--warmup W]
  python bench.py --profile-pass kernels   # short fixed sequence for rocprofv3
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s
# (FP64 add/mul/fma, FP32 unpacked, DPP moves and selects all issue at this
# rate; FP64 vector FMA peak 78.6 TFLOP/s = 2 x this)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
BYTES_PER_CELL = {               # algorithmic (compulsory) bytes per cell
    ("corrector", 8): 96, ("predictor", 8): 64, ("step", 8): 160,
    ("corrector", 4): 48, ("predictor", 4): 32, ("step", 4): 80,
    ("single_pass", 8): 64, ("single_pass", 4): 32,
    ("adjoint_step", 8): 288, ("adjoint_step", 4): 144,
}
# VALU instructions per cell and step of the single-pass kernel: its main
# loop's trip of three rows (each a predictor row, a corrector row and the
# CFL reduction, per lane) in the gfx950 assembly of fused_step_kernel<T,
# periodic, periodic, no fractions>, divided by 3; tests/test_valu_count.py
# recounts it from a fresh build.
VALU_OPS_PER_CELL = {8: 1612 / 3, 4: 1186 / 3}
KERNEL_SOURCES = ["paper_1607_08710_amd/csrc/lf_forward.hip", "paper_1607_08710_amd/csrc/lf_fused.hip",
                  "paper_1607_08710_amd/csrc/lf_device.h", "paper_1607_08710_amd/csrc/lf_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage_kh16384.json")
ADJ_SOURCES = KERNEL_SOURCES + ["paper_1607_08710_amd/csrc/lf_adjoint.hip"]
ADJ_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_adjoint_kh4096.json")
# Bytes per cell of a full gradient step (forward step + its recompute +
# lf_adjoint_step, each at the two-pass design's compulsory traffic)
FULL_GRADIENT_BYTES = {8: 608, 4: 304}
METRIC = "cell-updates/s per step (FP64 vs FP32, % HBM roofline) + adjoint step/s at 4096^2"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_solver(L, cfg, dtype):
    return L.Solver(L.Params(cfg["nx"], cfg["ny"], cfg["dx"], cfg["dy"], cfg["gamma"], cfg["cfl"],
                             cfg["beta"], cfg["bc_x"], cfg["bc_y"], dtype, cfg.get("ns", 0),
                             cfg.get("recon", 0)))


def time_advance(S, U, steps, warmup):
    """Warm up, then time `steps` full steps of lf_advance between events."""
    import torch
    if warmup:
        S.advance(U, 0.0, math.inf, max_steps=warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    t, n, _ = S.advance(U, 0.0, math.inf, max_steps=steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert n == steps, (n, steps)
    return e0.elapsed_time(e1) / 1e3, wall


def time_stages(S, U, reps):
    """Average duration of the predictor and corrector kernels, each launch
    bracketed by HIP events on the stream the library launches on."""
    import torch
    dt = S.dt(U)
    Us = S.empty_state()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2 * reps)]
    for k in range(reps):
        a, b = ev[2 * k]
        a.record()
        S.stage(1, U, Us, dt)
        b.record()
        a, b = ev[2 * k + 1]
        a.record()
        S.stage(2, Us, U, dt, base=U, reduce=True)  # in place, as in lf_advance
        b.record()
    torch.cuda.synchronize()
    pred = sum(ev[2 * k][0].elapsed_time(ev[2 * k][1]) for k in range(reps)) / reps
    corr = sum(ev[2 * k + 1][0].elapsed_time(ev[2 * k + 1][1]) for k in range(reps)) / reps
    del Us
    return pred / 1e3, corr / 1e3


def time_single_pass(S, U, reps):
    """Average duration of the single-pass step kernel (lf_step into a
    separate buffer), each launch bracketed by HIP events on the stream the
    library launches on."""
    import torch
    dt = S.dt(U)
    out = S.empty_state()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        S.step(U, out, dt)
        b.record()
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / reps
    del out
    return ms / 1e3


def forward_leg(L, W, n, dtype_flag, steps, warmup, reps, fractions=0, recon=0):
    import torch
    tdt = torch.float64 if dtype_flag == L.LF_F64 else torch.float32
    esz = 8 if dtype_flag == L.LF_F64 else 4
    U, cfg = W.kelvin_helmholtz_torch(n, device="cuda", dtype=tdt, fractions=fractions)
    cfg["recon"] = recon
    S = make_solver(L, cfg, dtype_flag)
    tot0 = S.totals(U)
    sec, wall = time_advance(S, U, steps, warmup)
    tot1 = S.totals(U)
    cells = n * n
    cups = cells * steps / sec
    pred, corr = time_stages(S, U, reps)
    drift = [float(b - a) for a, b in zip(tot0, tot1)]
    # algorithmic bytes scale with the number of fields (4 Euler + fractions)
    fw = (4 + fractions) / 4
    res = {
        "value": cups, "ms_per_step": 1e3 * sec / steps, "wall_s": wall,
        "predictor_ms": 1e3 * pred, "corrector_ms": 1e3 * corr,
        "predictor_GBps": fw * BYTES_PER_CELL[("predictor", esz)] * cells / pred / 1e9,
        "corrector_GBps": fw * BYTES_PER_CELL[("corrector", esz)] * cells / corr / 1e9,
        "totals_initial": [float(a) for a in tot0], "totals_drift": drift,
    }
    if recon:
        res["reconstruction"] = "conservative (rho, rho u, rho v, rho E)"
    if fractions:
        res["fractions"] = fractions
    sp = time_single_pass(S, U, reps)
    res["path"] = "single pass (one kernel per step, U* on chip)"
    res["single_pass_kernel_ms"] = 1e3 * sp
    # per-step time of the timed lf_advance region: one single-pass launch
    # (with the CFL reduction) and the dt-update kernel
    res["single_pass_GBps"] = fw * BYTES_PER_CELL[("single_pass", esz)] * cells * steps / sec / 1e9
    if not fractions and not recon:
        res["single_pass_valu_TOPs"] = VALU_OPS_PER_CELL[esz] * cells * steps / sec / 1e12
    res["two_stage"] = {"value": cells / (pred + corr), "step_ms": 1e3 * (pred + corr),
                        "step_effective_GBps": fw * BYTES_PER_CELL[("step", esz)] * cells / (pred + corr) / 1e9}
    del U, S
    torch.cuda.empty_cache()
    return res


def four_quadrant_leg(L, W, n, steps):
    """The four-quadrant Riemann problem at n^2 (transmissive), `steps` steps
    in FP64 and in FP32 from the same initial state: cell-updates/s of each
    and the FP32 state's per-field relative L1 / L-infinity error against the
    FP64 one (the FP64 path itself matches the oracle to 1e-12)."""
    import torch
    U64, cfg = W.four_quadrant(n)
    d64 = torch.from_numpy(U64).cuda()
    del U64
    d32 = d64.to(torch.float32)
    d32_init = d32.clone()
    res = {"n": n, "steps": steps}
    dts64 = None
    for name, flag, d in (("f64", L.LF_F64, d64), ("f32", L.LF_F32, d32)):
        S = make_solver(L, cfg, flag)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        t, k, dts = S.advance(d, 0.0, math.inf, max_steps=steps, dts_capacity=steps)
        e1.record()
        torch.cuda.synchronize()
        assert k == steps
        if flag == L.LF_F64:
            dts64 = dts
        sec = e0.elapsed_time(e1) / 1e3
        esz = 8 if flag == L.LF_F64 else 4
        res[name] = {"value": n * n * steps / sec, "ms_per_step": 1e3 * sec / steps, "t": t,
                     "single_pass_GBps": BYTES_PER_CELL[("single_pass", esz)] * n * n * steps / sec / 1e9}
        del S
    # error of the FP32 path at the FP64 run's times: replay its dt sequence
    # (untimed) from the same float initial state
    S = make_solver(L, cfg, L.LF_F32)
    x, y = d32_init, torch.empty_like(d32_init)
    for dt in dts64:
        S.step(x, y, float(dt))
        x, y = y, x
    torch.cuda.synchronize()
    del S, y, d32_init
    d32 = x
    a = d32.to(torch.float64)
    l1, linf = [], []
    for f in range(4):
        den1 = d64[f].abs().sum().item() or d64[1].abs().sum().item()
        deni = d64[f].abs().max().item() or d64[1].abs().max().item()
        diff = (a[f] - d64[f]).abs()
        l1.append(diff.sum().item() / den1)
        linf.append(diff.max().item() / deni)
    res["fp32_vs_fp64_rel_l1"] = l1
    res["fp32_vs_fp64_rel_linf"] = linf
    del a, d32, d64
    torch.cuda.empty_cache()
    return res


def vortex_leg(L, W, n, t_end=2.0):
    """The isentropic vortex (periodic [0,10]^2, advected by (1, 1)) at n^2
    up to t_end, in FP64 and in FP32 from the same initial state: the
    cell-updates/s of each lf_advance run (dt on the device) and the L1
    error of the density against the exact solution, the initial vortex
    translated by (t_end, t_end)."""
    import torch
    U, cfg = W.vortex(n, t_end=t_end)
    exact, _ = W.vortex(n, t=t_end)
    rho_exact = torch.from_numpy(exact[0]).cuda()
    del exact
    res = {"n": n, "t_end": t_end}
    for name, flag, tdt in (("f64", L.LF_F64, torch.float64), ("f32", L.LF_F32, torch.float32)):
        d = torch.from_numpy(U).to(device="cuda", dtype=tdt)
        S = make_solver(L, cfg, flag)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        t, k, _ = S.advance(d, 0.0, t_end)
        e1.record()
        torch.cuda.synchronize()
        assert t == t_end, (t, t_end)
        sec = e0.elapsed_time(e1) / 1e3
        err = (d[0].to(torch.float64) - rho_exact).abs().mean().item()
        res[name] = {"value": n * n * k / sec, "steps": k, "ms_per_step": 1e3 * sec / k, "rho_l1_error": err}
        del d, S
    del rho_exact
    torch.cuda.empty_cache()
    return res


def shard_leg(L, W, n, shards, steps, warmup):
    """One GPU's share of the n^2 Kelvin-Helmholtz grid split into `shards`
    strips of rows: lf_step_halo on the first strip (n x n/shards cells),
    each step preceded by the refresh of its ghost rows, 4 below and 4
    above, copied on the device from the neighbouring strips' rows (in
    place of the exchange between GPUs).  Reports the strip's step time,
    the ghost-row copy time and cell-updates/s of the strip; and checks
    that the strips stepped this way give the whole grid's lf_step bit for
    bit."""
    import torch
    U, cfg = W.kelvin_helmholtz_torch(n)
    h = n // shards
    S_all = make_solver(L, cfg, L.LF_F64)
    dt = S_all.dt(U)
    S = make_solver(L, dict(cfg, ny=h), L.LF_F64)
    G = L.GHOST_ROWS
    glo = torch.empty((4, G, n), dtype=U.dtype, device=U.device)
    ghi = torch.empty_like(glo)
    a = U[:, :h].contiguous()
    b = torch.empty_like(a)

    def refresh():
        glo.copy_(U[:, n - G:])      # the strip below, across the periodic wrap
        ghi.copy_(U[:, h:h + G])     # the strip above

    for _ in range(warmup):
        refresh()
        S.step_halo(a, glo, ghi, b, dt)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(steps):
        refresh()
    ev[1].record()
    for _ in range(steps):
        S.step_halo(a, glo, ghi, b, dt)
        a, b = b, a
    ev[2].record()
    torch.cuda.synchronize()
    copy_ms = ev[0].elapsed_time(ev[1]) / steps
    step_ms = ev[1].elapsed_time(ev[2]) / steps
    # every strip from the same U^n against the whole grid's step
    ref = torch.empty_like(U)
    S_all.step(U, ref, dt)
    same = True
    for k in range(shards):
        y0 = k * h
        rows = torch.arange(y0, y0 + h, device=U.device)
        lo = torch.arange(y0 - G, y0, device=U.device) % n
        hi = torch.arange(y0 + h, y0 + h + G, device=U.device) % n
        S.step_halo(U.index_select(1, rows).contiguous(), U.index_select(1, lo).contiguous(),
                    U.index_select(1, hi).contiguous(), b, dt)
        same = same and torch.equal(b, ref[:, y0:y0 + h])
    del U, ref, a, b, glo, ghi, S, S_all
    torch.cuda.empty_cache()
    return {"n": n, "shards": shards, "strip": [h, n], "steps": steps,
            "step_ms": step_ms, "value": n * h / (step_ms / 1e3),
            "ghost_copy_ms": copy_ms, "ghost_bytes_per_step": 2 * 4 * G * n * 8,
            "strips_equal_whole_grid_step": bool(same)}


def copy_bandwidth(nbytes=4 << 30, reps=10):
    """HBM bandwidth of a plain device-to-device copy (torch's copy kernel),
    bytes read + written per second: what a streaming kernel reaches on
    this GPU, next to the nominal 8 TB/s."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / sec / 1e9


def add_bandwidth(nbytes=2 << 30, reps=10):
    """HBM bandwidth of a plain element-wise c = a + b over float64 arrays of
    nbytes each (torch's add kernel): two streams read and one written per
    element, the read-heavy pattern of a corrector stage (which reads two
    states and writes one).  Bytes read + written per second."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    torch.add(a, b, out=c)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(a, b, out=c)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b, c
    torch.cuda.empty_cache()
    return 3 * nbytes / sec / 1e9


def adjoint_leg(L, W, n, dtype_flag, steps, ckpt, reps):
    """Bare lf_adjoint_step rate, and the full gradient (forward + recompute
    + adjoint) of a steps-long rollout with checkpoints every ckpt steps."""
    import torch
    from paper_1607_08710_amd import rollout
    tdt = torch.float64 if dtype_flag == L.LF_F64 else torch.float32
    U0, cfg = W.kelvin_helmholtz_torch(n, device="cuda", dtype=tdt)
    S = make_solver(L, cfg, dtype_flag)
    dt = S.dt(U0)
    lam = torch.randn_like(U0)
    out = torch.empty_like(U0)
    S.adjoint_step(U0, dt, lam, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        S.adjoint_step(U0, dt, lam, out)
    e1.record()
    torch.cuda.synchronize()
    bare = e0.elapsed_time(e1) / 1e3 / reps
    # the same adjoint step with the step's U* supplied (as the rollout's
    # recompute keeps it), i.e. without the predictor pass
    us = torch.empty_like(U0)
    S.stage(1, U0, us, dt)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        S.adjoint_step_ustar(U0, us, dt, lam, out)
    e1.record()
    torch.cuda.synchronize()
    bare_us = e0.elapsed_time(e1) / 1e3 / reps
    del us
    # full gradient of J = 1/2 dx dy sum (rho_N - rho_0)^2 w.r.t. U0; one
    # untimed rollout first, so that the timed one finds the allocator's
    # pool (10 checkpoints, a segment of 20 states and 20 U*: ~27 GB in
    # FP64 at 4096^2) already grown
    rho_t = U0[0].clone()
    for timed in (False, True):
        x = U0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        e0.record()
        UN = rollout(x, S, [dt] * steps, ckpt_every=ckpt)
        J = 0.5 * cfg["dx"] * cfg["dy"] * ((UN[0] - rho_t) ** 2).sum()
        J.backward()
        e1.record()
        torch.cuda.synchronize()
        if not timed:
            del x, UN, J
    full = e0.elapsed_time(e1) / 1e3
    g_ckpt = x.grad
    del x, UN, J
    torch.cuda.empty_cache()
    # the same gradient with every state and U* of the run kept in HBM
    # (ckpt_every = steps: no recompute), when they fit with a margin
    state_bytes = U0.numel() * U0.element_size()
    need = 2 * steps * state_bytes
    resident = None
    same = None
    if torch.cuda.mem_get_info()[0] > 1.15 * need:
        try:
            for timed in (False, True):
                x = U0.clone().requires_grad_(True)
                torch.cuda.synchronize()
                e0.record()
                UN = rollout(x, S, [dt] * steps, ckpt_every=steps)
                J = 0.5 * cfg["dx"] * cfg["dy"] * ((UN[0] - rho_t) ** 2).sum()
                J.backward()
                e1.record()
                torch.cuda.synchronize()
                if timed:
                    resident = e0.elapsed_time(e1) / 1e3
                    same = bool(torch.equal(x.grad, g_ckpt))
                del x, UN, J
        except torch.cuda.OutOfMemoryError:
            log("resident full gradient: out of device memory, not measured")
            resident = same = None
        torch.cuda.empty_cache()
    esz = 8 if dtype_flag == L.LF_F64 else 4
    res = {
        "lf_adjoint_step_per_s": 1.0 / bare,
        "lf_adjoint_step_ms": 1e3 * bare,
        "lf_adjoint_step_GBps": BYTES_PER_CELL[("adjoint_step", esz)] * n * n / bare / 1e9,
        "lf_adjoint_step_ustar_per_s": 1.0 / bare_us,
        "full_gradient_steps_per_s": steps / full,
        "full_gradient_s": full,
        "grad_finite": bool(torch.isfinite(g_ckpt).all().item()),
        # every state and U* of the run resident (2 x steps states, GB):
        # no recompute; the gradient equals the checkpointed one bit for bit
        "full_gradient_resident_steps_per_s": steps / resident if resident else None,
        "full_gradient_resident_GB": need / 1e9,
        "full_gradient_resident_equal": same,
    }
    del U0, S, lam, out, g_ckpt
    torch.cuda.empty_cache()
    return res


def _host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return model


def oracle_rate(U, cfg, min_seconds, min_steps=1, max_steps=400):
    """FP64 oracle Heun steps of state U at its fixed CFL dt, as many as fit
    in ~min_seconds (at least min_steps): (cell-updates/s, steps, seconds)."""
    import oracle
    P = oracle.Params(cfg["nx"], cfg["ny"], cfg["dx"], cfg["dy"], cfg["gamma"], cfg["cfl"], cfg["beta"],
                      cfg["bc_x"], cfg["bc_y"])
    rc, dt = oracle.dt(P, U)
    t0 = time.perf_counter()
    steps = 0
    while steps < min_steps or (time.perf_counter() - t0 < min_seconds and steps < max_steps):
        U = oracle.step(P, U, dt)
        steps += 1
    sec = time.perf_counter() - t0
    return cfg["nx"] * cfg["ny"] * steps / sec, steps, sec


def cpu_baseline(W, n=16384, rows=None, min_seconds=10.0):
    """The FP64 oracle on the benchmark's own workload, the Kelvin-Helmholtz
    state at n^2 (or its bottom `rows` rows), at least one full step, as
    many as fit in ~min_seconds, on this host's OpenMP threads."""
    U, cfg = W.kelvin_helmholtz(n, rows=rows)
    rate, steps, sec = oracle_rate(U, cfg, min_seconds)
    del U
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    what = f"{n}^2 (full grid)" if rows is None else f"{n} x {rows} (its bottom {rows} rows, periodic)"
    return {"value": rate, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "host_cpu": _host_cpu(), "host_logical_cpus": os.cpu_count(),
            "sample": f"Kelvin-Helmholtz {what}, {steps} FP64 Heun step(s) at fixed dt ({sec:.1f} s), "
                      f"OMP_NUM_THREADS={cores}"}


def cpu_planned(W, vortex_n=4096, quadrant_n=8192, min_seconds=3.0):
    """The oracle on bounded samples of the isentropic vortex at 4096^2 and
    the four-quadrant problem at 8192^2 (the timing workloads of the
    oracle's plan), all threads: a few full-grid steps of each."""
    out = {}
    U, cfg = W.vortex(vortex_n)
    rate, steps, sec = oracle_rate(U, cfg, min_seconds)
    out["vortex"] = {"value": rate, "n": vortex_n, "steps": steps, "seconds": sec}
    del U
    U, cfg = W.four_quadrant(quadrant_n)
    rate, steps, sec = oracle_rate(U, cfg, min_seconds)
    out["four_quadrant"] = {"value": rate, "n": quadrant_n, "steps": steps, "seconds": sec}
    del U
    out["unit"] = "cell-updates/s"
    out["cores"] = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    return out


def cpu_per_core(n=16384, rows=1024, min_seconds=4.0):
    """The oracle on one thread (the per-core figure the paper compares
    with) on the bottom `rows` rows of the benchmark grid, in a child
    process started with OMP_NUM_THREADS=1 (OpenMP reads it at start-up);
    the child touches no GPU."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-only", "--cpu-n", str(n),
                          "--cpu-rows", str(rows), "--cpu-seconds", str(min_seconds)], env=env,
                         capture_output=True, text=True, timeout=900, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def traffic_entry(n, key, path=TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """A per-launch figure of one kernel (key in a committed counter record,
    e.g. corrector_f64_bytes) from the rocprofv3 counter summary at path,
    or None when absent, taken at another grid size or from other kernel
    sources."""
    if not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash(sources):
        return None, "kernel changed since the counters were taken"
    if rec.get("n") != n:
        return None, "counters taken at another size"
    if rec.get(key) is None:
        return None, "not in the counter summary"
    return rec.get(key), "rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel"


def adjoint_rooflines(n, adj64, adj32):
    """lf_adjoint_step (288 / 144 B per cell: U* recomputed, then the two
    adjoint stages) and the full gradient step (608 / 304 B per cell:
    forward step, its recompute and the adjoint step) against HBM, from the
    timed rates; traffic per lf_adjoint_step from the committed counters of
    its three kernels."""
    cells = n * n
    out = {}
    for name, r, esz in (("f64", adj64, 8), ("f32", adj32, 4)):
        if r is None:
            continue
        b = BYTES_PER_CELL[("adjoint_step", esz)]
        ach = b * cells * r["lf_adjoint_step_per_s"] / 1e9
        traffic, src = traffic_entry(n, f"adjoint_step_{name}_bytes", ADJ_TRAFFIC_FILE, ADJ_SOURCES)
        issued, _ = traffic_entry(n, f"adjoint_step_{name}_valu_wave_instructions", ADJ_TRAFFIC_FILE, ADJ_SOURCES)
        step = {"bound": "hbm",
                "kernel": f"lf_adjoint_step (FP{esz * 8}): stage_kernel predictor (U* recomputed) + "
                          f"adjoint_kernel modes 1 and 2",
                "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS,
                "traffic": traffic, "traffic_source": src, "algorithmic_bytes_per_cell": b,
                "cells_per_launch": cells, "avg_launch_ms": r["lf_adjoint_step_ms"]}
        if issued:
            step["issued_valu_lane_instructions_per_cell"] = issued * 64 / cells
            step["valu_issue_frac"] = issued * 64 * r["lf_adjoint_step_per_s"] / 1e12 / VALU_PEAK_TOPS
        bf = FULL_GRADIENT_BYTES[esz]
        achf = bf * cells * r["full_gradient_steps_per_s"] / 1e9
        full = {"bound": "hbm", "achieved": achf, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achf / HBM_PEAK_GBPS, "algorithmic_bytes_per_cell_step": bf,
                "steps_per_s": r["full_gradient_steps_per_s"],
                "steps_per_s_at_roofline": HBM_PEAK_GBPS * 1e9 / (bf * cells)}
        out[name] = {"lf_adjoint_step": step, "full_gradient": full}
    return out


def _calibration_copies():
    """Plain copies of known size for the counter calibration: 1 GiB read +
    1 GiB written per launch, by torch's copy kernel and by the runtime's
    device-to-device memcpy."""
    import ctypes
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(3):
        rc = hip.hipMemcpyAsync(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), 1 << 30, 3, stream)
        assert rc == 0, rc
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def _adjoint_profile_steps(L, W, n):
    """lf_adjoint_step three times in each precision at n^2 (its three
    kernels: the predictor recompute and the two adjoint stages)."""
    import torch
    for flag, tdt in ((L.LF_F64, torch.float64), (L.LF_F32, torch.float32)):
        U, cfg = W.kelvin_helmholtz_torch(n, device="cuda", dtype=tdt)
        S = make_solver(L, cfg, flag)
        dt = S.dt(U)
        lam, out = torch.ones_like(U), torch.empty_like(U)
        for _ in range(3):
            S.adjoint_step(U, dt, lam, out)
        torch.cuda.synchronize()
        del U, S, lam, out
        torch.cuda.empty_cache()


def profile_pass(L, W, n, which="kernels", adj_n=4096):
    """Fixed short sequences for rocprofv3.  "kernels": each stage kernel of
    both precisions (and the FP64 one with one mass fraction) a few times,
    the single-pass kernel through lf_advance and lf_step, the adjoint step
    at 4096^2 in both precisions, then plain device copies of known size.
    "adjoint": the adjoint steps and the copies only."""
    import torch
    if which == "kernels":
        for flag, tdt, k in ((L.LF_F64, torch.float64, 0), (L.LF_F32, torch.float32, 0),
                             (L.LF_F64, torch.float64, 1)):
            U, cfg = W.kelvin_helmholtz_torch(n, device="cuda", dtype=tdt, fractions=k)
            S = make_solver(L, cfg, flag)
            S.advance(U, 0.0, math.inf, max_steps=4)  # even: no copy back from the workspace
            time_stages(S, U, 5)
            if k == 0:
                time_single_pass(S, U, 5)
            torch.cuda.synchronize()
            del U, S
            torch.cuda.empty_cache()
    _adjoint_profile_steps(L, W, adj_n)
    _calibration_copies()
    log("profile pass done")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=16384, help="grid cells per side")
    ap.add_argument("--adj-n", type=int, default=4096)
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--adj-ckpt", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="forward,species,quadrant,vortex,shard,adjoint,cpu",
                    help="comma list of legs to run: forward, species, quadrant, vortex, shard, adjoint, cpu "
                         "(profiling runs use one leg so that each kernel runs at one grid size)")
    ap.add_argument("--shards", type=int, default=8)
    ap.add_argument("--vortex-n", type=int, default=4096)
    ap.add_argument("--cpu-n", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-rows", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--oracle-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--quadrant-n", type=int, default=8192)
    ap.add_argument("--quadrant-steps", type=int, default=1000)
    ap.add_argument("--species-steps", type=int, default=200)
    ap.add_argument("--profile-pass", choices=["none", "kernels", "adjoint"], default="none")
    args = ap.parse_args()

    if args.oracle_only:  # child of cpu_per_core(): the oracle alone, no GPU
        import workloads as W
        print(json.dumps(cpu_baseline(W, n=args.cpu_n, rows=args.cpu_rows or None,
                                      min_seconds=args.cpu_seconds)), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the Lagrange-flux path is built and measured on a single "
              "MI355X (one GPU's strip of a split grid, lf_step_halo, is timed by the shard leg; the "
              "exchange between GPUs is not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1607_08710_amd as L
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    L.lib()

    if args.profile_pass != "none":
        profile_pass(L, W, args.n, args.profile_pass, args.adj_n)
        return

    legs = set(x.strip() for x in args.legs.split(",") if x.strip())
    f64 = f32 = adj64 = adj32 = roofline = cpu = hbm_roofline = roofline_adjoint = None
    species = roofline_two_stage = recon64 = quadrant = vortex = shard = None
    if "forward" in legs:
        log(f"FP64 Kelvin-Helmholtz {args.n}^2: {args.warmup} warm-up + {args.steps} timed steps")
        f64 = forward_leg(L, W, args.n, L.LF_F64, args.steps, args.warmup, args.kernel_reps)
        log(f"FP64 {f64['value'] / 1e9:.2f} G cell-updates/s, {f64['ms_per_step']:.3f} ms/step")
        log(f"FP32 Kelvin-Helmholtz {args.n}^2")
        f32 = forward_leg(L, W, args.n, L.LF_F32, args.steps, args.warmup, args.kernel_reps)
        f32["ratio_vs_fp64"] = f32["value"] / f64["value"]
        f32["two_stage"]["ratio_vs_fp64"] = f32["two_stage"]["value"] / f64["two_stage"]["value"]
        log(f"FP32 {f32['value'] / 1e9:.2f} G cell-updates/s, {f32['ms_per_step']:.3f} ms/step")
        cells = args.n * args.n
        # the timed steps run the single-pass kernel: bound by VALU issue; its
        # launch time is the per-step time of the timed region (which also
        # holds the few-microsecond dt-update kernel)
        sp_s = f64["ms_per_step"] / 1e3
        achieved = VALU_OPS_PER_CELL[8] * cells / sp_s / 1e12
        traffic, traffic_src = traffic_entry(args.n, "single_pass_f64_bytes")
        issued, _ = traffic_entry(args.n, "single_pass_f64_lf_advance_valu_wave_instructions")
        copy_gbps = copy_bandwidth()
        add_gbps = add_bandwidth()
        log(f"device copy {copy_gbps:.0f} GB/s, two-read one-write probe {add_gbps:.0f} GB/s")
        roofline = {"bound": "alu",
                    "kernel": "lf::fused_step_kernel<double, 0, 0, 0, false> (FP64 single-pass step, periodic)",
                    "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                    "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic, "traffic_source": traffic_src,
                    "algorithmic_ops_per_cell": VALU_OPS_PER_CELL[8],
                    "ops": "VALU lane-instructions per OUTPUT cell-step: the main loop's instructions per row "
                           "and lane, counted from the kernel's gfx950 assembly, on the 56 output lanes of "
                           "each 64-lane wave (halo lanes and strip prologues not counted)",
                    "peak_definition": "256 CUs x 4 SIMD16 x 16 lanes x 2.4 GHz lane-instructions/s (FP64 "
                                       "add/mul/fma, DPP moves, selects issue at this rate)",
                    "algorithmic_bytes_per_cell": BYTES_PER_CELL[("single_pass", 8)],
                    "hbm_GBps": BYTES_PER_CELL[("single_pass", 8)] * cells / sp_s / 1e9,
                    "hbm_frac": BYTES_PER_CELL[("single_pass", 8)] * cells / sp_s / 1e9 / HBM_PEAK_GBPS,
                    "cells_per_launch": cells, "avg_launch_ms": f64["ms_per_step"],
                    "measured_copy_GBps": copy_gbps, "measured_two_read_one_write_GBps": add_gbps}
        if issued:
            # all lanes, halo columns and strip prologues included (SQ_INSTS_VALU x 64)
            roofline["issued_ops_per_cell"] = issued * 64 / cells
            roofline["issued_frac"] = issued * 64 / sp_s / 1e12 / VALU_PEAK_TOPS
        # the metric's "% HBM roofline": cell-updates/s x the compulsory bytes
        # of the two-pass design (160 B FP64, 80 B FP32 per cell-step) against
        # 8 TB/s; the single-pass kernel moves 64 / 32 of those bytes
        hbm_roofline = {"definition": "cell-updates/s x bytes per cell-step of the two-pass design "
                                      "(predictor R 32 + W 32, corrector R 64 + W 32 in FP64; half in FP32) / "
                                      "8 TB/s",
                        "note": "the single pass keeps U* on chip and moves 64 (FP64) / 32 (FP32) of those "
                                "bytes per cell-step, so its fraction can exceed 1; the two-stage path "
                                "moves them all",
                        "peak_GBps": HBM_PEAK_GBPS}
        for name, r, esz in (("f64", f64, 8), ("f32", f32, 4)):
            b = BYTES_PER_CELL[("step", esz)]
            hbm_roofline[name] = {
                "bytes_per_cell_step": b,
                "single_pass": {"cell_updates_per_s": r["value"], "GBps": r["value"] * b / 1e9,
                                "frac": r["value"] * b / 1e9 / HBM_PEAK_GBPS},
                "two_stage": {"cell_updates_per_s": r["two_stage"]["value"],
                              "GBps": r["two_stage"]["value"] * b / 1e9,
                              "frac": r["two_stage"]["value"] * b / 1e9 / HBM_PEAK_GBPS},
            }
        # the two-stage design (one kernel per stage) against HBM
        corr_s = f64["corrector_ms"] / 1e3
        ach2 = BYTES_PER_CELL[("corrector", 8)] * cells / corr_s / 1e9
        traffic2, traffic_src2 = traffic_entry(args.n, "corrector_f64_bytes")
        roofline_two_stage = {"bound": "hbm",
                              "kernel": "lf::stage_kernel<double, 2, 0, 0, 0, false> (FP64 corrector, periodic)",
                              "achieved": ach2, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                              "frac": ach2 / HBM_PEAK_GBPS, "traffic": traffic2, "traffic_source": traffic_src2,
                              "algorithmic_bytes_per_cell": BYTES_PER_CELL[("corrector", 8)],
                              "cells_per_launch": cells, "avg_launch_ms": f64["corrector_ms"],
                              "measured_copy_GBps": copy_gbps, "frac_of_measured_copy": ach2 / copy_gbps,
                              "measured_two_read_one_write_GBps": add_gbps,
                              "frac_of_two_read_one_write": ach2 / add_gbps}
    if "species" in legs:
        species = {}
        for k in (1, 2):
            log(f"FP64 Kelvin-Helmholtz {args.n}^2 with {k} mass fraction(s): {args.species_steps} steps")
            r = forward_leg(L, W, args.n, L.LF_F64, args.species_steps, args.warmup, args.kernel_reps,
                            fractions=k)
            species[f"f64_ns{k}"] = r
            log(f"  {r['value'] / 1e9:.2f} G cell-updates/s (two stages: {r['two_stage']['value'] / 1e9:.2f} G, "
                f"corrector {r['corrector_GBps']:.0f} GB/s)")
    if "species" in legs:
        log(f"FP64 Kelvin-Helmholtz {args.n}^2, conservative-variable reconstruction: {args.species_steps} steps")
        recon64 = forward_leg(L, W, args.n, L.LF_F64, args.species_steps, args.warmup, args.kernel_reps, recon=1)
        log(f"  {recon64['value'] / 1e9:.2f} G cell-updates/s")
    if "quadrant" in legs:
        log(f"four-quadrant Riemann problem {args.quadrant_n}^2, {args.quadrant_steps} steps, FP64 and FP32")
        quadrant = four_quadrant_leg(L, W, args.quadrant_n, args.quadrant_steps)
        log(f"  FP64 {quadrant['f64']['value'] / 1e9:.2f} G, FP32 {quadrant['f32']['value'] / 1e9:.2f} G "
            f"cell-updates/s; FP32 vs FP64 rel L1 {max(quadrant['fp32_vs_fp64_rel_l1']):.2e}")
    if "vortex" in legs:
        log(f"isentropic vortex {args.vortex_n}^2 to t = 2, FP64 and FP32")
        vortex = vortex_leg(L, W, args.vortex_n)
        log(f"  FP64 {vortex['f64']['value'] / 1e9:.2f} G cell-updates/s over {vortex['f64']['steps']} steps, "
            f"rho L1 error {vortex['f64']['rho_l1_error']:.3e}; FP32 {vortex['f32']['value'] / 1e9:.2f} G, "
            f"{vortex['f32']['rho_l1_error']:.3e}")
    if "shard" in legs:
        log(f"one strip of {args.n}^2 in {args.shards}: lf_step_halo on {args.n // args.shards} x {args.n} cells")
        shard = shard_leg(L, W, args.n, args.shards, args.steps // 2, args.warmup)
        log(f"  {shard['step_ms']:.3f} ms/step ({shard['value'] / 1e9:.2f} G cell-updates/s), ghost rows "
            f"{shard['ghost_copy_ms'] * 1e3:.1f} us/step; strips equal the whole-grid step: "
            f"{shard['strips_equal_whole_grid_step']}")
    if "adjoint" in legs:
        log(f"adjoint {args.adj_n}^2, {args.adj_steps} steps, checkpoints every {args.adj_ckpt}")
        adj64 = adjoint_leg(L, W, args.adj_n, L.LF_F64, args.adj_steps, args.adj_ckpt, 10)
        log(f"adjoint FP64: {adj64['lf_adjoint_step_per_s']:.1f} lf_adjoint_step/s, "
            f"{adj64['full_gradient_steps_per_s']:.1f} full-gradient steps/s")
        adj32 = adjoint_leg(L, W, args.adj_n, L.LF_F32, args.adj_steps, args.adj_ckpt, 10)
        log(f"adjoint FP32: {adj32['lf_adjoint_step_per_s']:.1f} lf_adjoint_step/s, "
            f"{adj32['full_gradient_steps_per_s']:.1f} full-gradient steps/s")
        roofline_adjoint = adjoint_rooflines(args.adj_n, adj64, adj32)
    if "cpu" in legs and not args.no_cpu_baseline:
        log("CPU oracle baseline")
        cpu_n = args.cpu_n or args.n
        cpu = cpu_baseline(W, n=cpu_n, min_seconds=args.cpu_seconds)
        log(f"oracle {cpu['value'] / 1e6:.2f} M cell-updates/s on {cpu['cores']} threads ({cpu['sample']})")
        cpu["one_thread"] = cpu_per_core(n=cpu_n, rows=min(1024, cpu_n))
        log(f"oracle on one thread {cpu['one_thread']['value'] / 1e6:.2f} M cell-updates/s")
        cpu["planned_workloads"] = cpu_planned(W)
        log(f"oracle: vortex {cpu['planned_workloads']['vortex']['value'] / 1e6:.2f} M, four-quadrant "
            f"{cpu['planned_workloads']['four_quadrant']['value'] / 1e6:.2f} M cell-updates/s")

    line = {
        "metric": METRIC,
        "value": f64["value"] if f64 else None,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"] if f64 else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Kelvin-Helmholtz shear layer, periodic, {args.n}^2 cells, gamma 1.4, "
                               f"CFL 0.5, Sweby beta 1.5, Heun steps via lf_advance",
                   "nx": args.n, "ny": args.n, "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_two_stage": roofline_two_stage,
        "hbm_roofline": hbm_roofline,
        "roofline_adjoint": roofline_adjoint,
        "cpu_baseline": cpu,
        "fp64": f64,
        "fp32": f32,
        "species": species,
        "conservative_reconstruction": recon64,
        "four_quadrant": quadrant,
        "vortex": vortex,
        "shard": shard,
        "adjoint": {"n": args.adj_n, "steps": args.adj_steps, "ckpt_every": args.adj_ckpt,
                    "f64": adj64, "f32": adj32},
        "paper_context": {"value": 81.0e6, "unit": "cell-updates/s",
                          "hardware": "2 x 8-core Intel Sandy Bridge E5-2670, AVX, OpenMP",
                          "workload": "mesh unspecified (fine meshes in DRAM)"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
