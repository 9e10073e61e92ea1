"""Multi-step oracle parity at the benchmark sizes, in the launch
configuration the benchmark times (the single-pass step kernel).

The oracle cannot step a 16384^2 grid ten times in a test, but it does not
need to: after k Heun steps a cell depends only on the (8k+1)^2 block of
the initial state around it (each step reads 4 cells along each axis, two
per stage, Sec. 5 items 2-11).  So the GPU runs k steps of the whole grid
and the oracle steps, for each sampled cell, the patch of radius 4k around
it (gpu_util.oracle_steps_at); the centre values must agree.

Two parts per workload:
  * lf_step chained k times at the oracle's time step of the initial state
    (frozen), against the oracle's patches: FP64 within 1e-12 relative
    L-infinity per field (the FP32 path within 2e-5 relative L1 over the
    sampled cells);
  * lf_advance over the same k steps, with dt and t on the device: its
    state equals the lf_step chain driven by the time steps it recorded, bit
    for bit, its first time step equals the oracle's, and every recorded
    time step is the CFL time step (Heun list, item 1) of the chain's state
    before that step, evaluated with plain torch float64 operations.

Sampled cells include the structure of each problem: the shear layers of
the Kelvin-Helmholtz state, the vortex core, and for the four-quadrant
problem the lines x = 1/2 and y = 1/2 where its shocks and contacts start,
so that most samples are not free-stream cells.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import (cfl_dt_torch, oracle_params, oracle_steps_at, solver_for, to_dev,
                      values_at)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _release():
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def _chain(S, U0, dts):
    """lf_step applied len(dts) times from U0 (single-pass kernel, separate
    buffers); returns the final state."""
    x = U0
    a, b = S.empty_state(), S.empty_state()
    for k, dt in enumerate(dts):
        y = a if k % 2 == 0 else b
        S.step(x, y, float(dt))
        x = y
    return x


def _advance_matches_chain(S, U0, cfg, k, dt0_oracle, dt_tol):
    """lf_advance for k steps on a copy of U0 vs the lf_step chain at the
    recorded time steps (bitwise); the first dt vs the oracle's and each dt
    vs the CFL time step of the state it was taken from, both within
    dt_tol relative."""
    import torch
    Ua = U0.clone()
    t, n, dts = S.advance(Ua, 0.0, math.inf, max_steps=k, dts_capacity=k)
    assert n == k and len(dts) == k
    assert abs(dts[0] - dt0_oracle) <= dt_tol * dt0_oracle, (dts[0], dt0_oracle)
    x = U0
    a, b = S.empty_state(), S.empty_state()
    worst = 0.0
    for q, dt in enumerate(dts):
        ref = cfl_dt_torch(x, cfg)
        worst = max(worst, abs(dt - ref) / ref)
        y = a if q % 2 == 0 else b
        S.step(x, y, float(dt))
        x = y
    same = bool(torch.equal(x, Ua))
    del Ua, a, b, x
    _release()
    print(f"lf_advance: {k} steps, dt relative gap to the CFL property {worst:.1e}, equal to the chain: {same}")
    assert worst <= dt_tol, worst
    assert same


def _rel_err_linf(got, ref, scale):
    return np.abs(got - ref).max(axis=0) / scale


# ---- Kelvin-Helmholtz 16384^2, the first 10 steps ---------------------------------

def _kh_cells(n, rng, count):
    cells = [(int(i), int(j)) for i, j in rng.integers(0, n, size=(count, 2))]
    # across both shear layers (y = 1/4 and 3/4: rows n/4 and 3n/4)
    for i in (0, 3001, 9002, n - 1):
        for j0 in (n // 4, 3 * n // 4):
            cells += [(i, j0 + d) for d in (-2, -1, 0, 1)]
    cells += [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0)]
    return cells


def test_kh_16384_ten_steps_f64():
    import torch
    n, k = 16384, 10
    U0, cfg = workloads.kelvin_helmholtz_torch(n, device="cuda")
    P = oracle_params(cfg)
    Uh = U0.cpu().numpy()
    rc, dt0 = oracle.dt(P, Uh)
    assert rc == 0
    del Uh
    S = solver_for(cfg)
    Uk = _chain(S, U0, [dt0] * k)
    cells = _kh_cells(n, np.random.default_rng(16385), 48)
    ref = oracle_steps_at(U0, cfg, [dt0] * k, cells)
    got = values_at(Uk, cells)
    scale = U0.abs().amax(dim=(1, 2)).cpu().numpy()
    moved = (np.abs(got - values_at(U0, cells)) / scale).max(axis=1) > 1e-6
    err = _rel_err_linf(got, ref, scale)
    print(f"KH {n}^2, {k} steps vs oracle patches ({len(cells)} cells, {moved.sum()} changed): rel Linf {err}")
    assert np.all(err <= TOL64), err
    assert moved.sum() >= len(cells) // 2
    del Uk
    _release()
    _advance_matches_chain(S, U0, cfg, k, dt0, 1e-14)


def test_kh_16384_f32_one_and_ten_steps():
    """The FP32 single-pass kernel (periodic, five waves per SIMD) at its
    launch shape: FP32 state, FP64 oracle on the same rounded initial
    state; relative L1 over the sampled cells <= 2e-5 per field, L-infinity
    reported."""
    import torch
    n = 16384
    U0, cfg = workloads.kelvin_helmholtz_torch(n, device="cuda", dtype=torch.float32)
    P = oracle_params(cfg)
    Uh = U0.to(torch.float64).cpu().numpy()
    rc, dt0 = oracle.dt(P, Uh)
    assert rc == 0
    del Uh
    S = solver_for(cfg, "f32")
    cells = _kh_cells(n, np.random.default_rng(32768), 40)
    for k in (1, 10):
        Uk = _chain(S, U0, [dt0] * k)
        ref = oracle_steps_at(U0, cfg, [dt0] * k, cells)
        got = values_at(Uk, cells)
        l1 = np.abs(got - ref).sum(axis=0) / np.abs(ref).sum(axis=0)
        linf = np.abs(got - ref).max(axis=0) / np.abs(ref).max(axis=0)
        print(f"KH {n}^2 FP32, {k} step(s) vs oracle patches: rel L1 {l1}, rel Linf {linf}")
        assert np.all(l1 <= 2e-5), (k, l1)
        del Uk
        _release()
    # FP32 CFL sums are formed in float, reduced and divided in FP64
    _advance_matches_chain(S, U0, cfg, 10, dt0, 1e-6)


def test_kh_16384_f32_single_pass_equals_two_stages():
    """At 16384^2 the FP32 single-pass kernel (lf_step into a separate
    buffer) and the two stage kernels (lf_step in place) give the same bits,
    one step and three steps in a row."""
    import torch
    n = 16384
    U0, cfg = workloads.kelvin_helmholtz_torch(n, device="cuda", dtype=torch.float32)
    S = solver_for(cfg, "f32")
    dt = S.dt(U0)
    x = U0.clone()
    y = S.empty_state()
    z = S.empty_state()
    for step in range(3):
        S.step(x, y, dt)      # single pass
        S.step(x, x, dt)      # two stages, in place
        assert torch.equal(x, y), step
        if step == 0:
            z.copy_(x)
    assert not torch.equal(z, U0)


# ---- four-quadrant Riemann problem 8192^2, 25 steps -----------------------------

def test_four_quadrant_8192_25_steps_f64():
    import torch
    n, k = 8192, 25
    U, cfg = workloads.four_quadrant(n)
    P = oracle_params(cfg)
    rc, dt0 = oracle.dt(P, U)
    assert rc == 0
    U0 = to_dev(U)
    del U
    S = solver_for(cfg)
    Uk = _chain(S, U0, [dt0] * k)
    h = n // 2
    rng = np.random.default_rng(8193)
    cells = []
    # across the line x = 1/2 (columns h-1 | h) at seeded rows, and across
    # y = 1/2 at seeded columns: the initial discontinuities
    for j in rng.integers(0, n, size=6):
        cells += [(h + d, int(j)) for d in (-6, -2, -1, 0, 1, 5)]
    for i in rng.integers(0, n, size=6):
        cells += [(int(i), h + d) for d in (-6, -2, -1, 0, 1, 5)]
    # the centre, where the four waves meet
    cells += [(h + a, h + b) for a in (-8, -3, 0, 2, 7) for b in (-8, -3, 0, 2, 7)]
    # the lines' ends at the transmissive boundaries, and corners
    cells += [(h - 1, 0), (h, n - 1), (0, h), (n - 1, h - 1), (0, 0), (n - 1, n - 1)]
    ref = oracle_steps_at(U0, cfg, [dt0] * k, cells)
    got = values_at(Uk, cells)
    scale = U0.abs().amax(dim=(1, 2)).cpu().numpy()
    moved = (np.abs(got - values_at(U0, cells)) / scale).max(axis=1) > 1e-3
    err = _rel_err_linf(got, ref, scale)
    print(f"four-quadrant {n}^2, {k} steps vs oracle patches ({len(cells)} cells, {moved.sum()} changed by "
          f"more than 1e-3): rel Linf {err}")
    assert np.all(err <= TOL64), err
    assert moved.sum() >= len(cells) // 2, moved.sum()
    # the x <-> y mirror symmetry of the problem holds on the GPU state too
    t = Uk.transpose(1, 2)
    assert torch.equal(t[0], Uk[0]) and torch.equal(t[1], Uk[2]) and torch.equal(t[3], Uk[3])
    del Uk, t
    _release()
    _advance_matches_chain(S, U0, cfg, k, dt0, 1e-14)


# ---- isentropic vortex 4096^2, 10 steps -----------------------------------------

def test_vortex_4096_ten_steps_f64():
    n, k = 4096, 10
    U, cfg = workloads.vortex(n)
    P = oracle_params(cfg)
    rc, dt0 = oracle.dt(P, U)
    assert rc == 0
    U0 = to_dev(U)
    del U
    S = solver_for(cfg)
    Uk = _chain(S, U0, [dt0] * k)
    rng = np.random.default_rng(4097)
    cells = [(int(i), int(j)) for i, j in rng.integers(0, n, size=(24, 2))]
    c = n // 2
    cells += [(c + a, c + b) for a in (-300, -41, -1, 0, 40, 301) for b in (-300, -2, 0, 39, 300)]
    cells += [(0, 0), (n - 1, n - 1), (0, c), (c, n - 1)]
    ref = oracle_steps_at(U0, cfg, [dt0] * k, cells)
    got = values_at(Uk, cells)
    scale = U0.abs().amax(dim=(1, 2)).cpu().numpy()
    err = _rel_err_linf(got, ref, scale)
    print(f"vortex {n}^2, {k} steps vs oracle patches ({len(cells)} cells): rel Linf {err}")
    assert np.all(err <= TOL64), err
    del Uk
    _release()
    _advance_matches_chain(S, U0, cfg, k, dt0, 1e-14)
