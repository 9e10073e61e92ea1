"""GPU: the single-pass step kernel against the two-stage path.

lf_step with a separate output buffer (and lf_advance) run the predictor
and the corrector in one kernel, keeping U* on chip.  The arithmetic is
that of the stage kernels, so the result must be bit for bit that of
lf_stage(1) followed by lf_stage(2), on every shape (tile edges at 56
columns, block edges at 224 / 448 columns, strip edges, grids smaller than
the stencil), both boundary conditions per axis, both precisions and every
limiter.  The oracle parity of lf_step and lf_advance is covered by the
other GPU test files, which now run this kernel.
"""
import math

import numpy as np
import pytest

import workloads
from gpu_util import solver_for, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 9), (9, 1), (3, 2), (5, 7), (56, 9), (57, 33), (113, 70), (224, 17), (225, 40),
          (448, 5), (449, 66), (130, 129)]
BCS = [(0, 0), (1, 1), (0, 1), (1, 0)]


def _cfg(nx, ny, bcx, bcy, beta=1.5):
    d = 1.0 / max(nx, ny)
    return dict(nx=nx, ny=ny, dx=d, dy=d * 1.25, gamma=1.4, cfl=0.5, beta=beta, bc_x=bcx, bc_y=bcy)


def _two_stage(S, U, dt):
    Us, out = S.empty_state(), S.empty_state()
    S.stage(1, U, Us, dt)
    S.stage(2, Us, out, dt, base=U)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_single_pass_step_bitwise(shape, bc, dtype):
    nx, ny = shape
    cfg = _cfg(nx, ny, *bc)
    U = workloads.random_state(nx, ny, seed=nx * 7 + ny * 3 + bc[0] + 2 * bc[1])
    S = solver_for(cfg, dtype)
    d = to_dev(U, dtype)
    dt = S.dt(d)
    out = S.empty_state()
    S.step(d, out, dt)
    ref = _two_stage(S, d, dt)
    assert np.array_equal(to_host(out), to_host(ref))


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_pass_step_bitwise_limiters(beta, dtype):
    cfg = _cfg(300, 75, 1, 0, beta)
    U = workloads.random_state(300, 75, seed=int(10 * beta) + 1)
    S = solver_for(cfg, dtype)
    d = to_dev(U, dtype)
    dt = S.dt(d)
    out = S.empty_state()
    S.step(d, out, dt)
    assert np.array_equal(to_host(out), to_host(_two_stage(S, d, dt)))


@pytest.mark.parametrize("rows", ["4", "5", "8", "37", "64", "4096"])
def test_single_pass_strip_heights(rows, monkeypatch):
    """The strip height changes the launch shape only."""
    monkeypatch.setenv("LF_FUSED_ROWS", rows)
    cfg = _cfg(131, 77, 1, 1)
    U = workloads.random_state(131, 77, seed=5)
    S = solver_for(cfg)
    d = to_dev(U)
    dt = S.dt(d)
    out = S.empty_state()
    S.step(d, out, dt)
    assert np.array_equal(to_host(out), to_host(_two_stage(S, d, dt)))


@pytest.mark.parametrize("steps", [7, 8])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_advance_matches_stage_loop(steps, bc):
    """lf_advance (single pass, alternating buffers, odd and even step
    counts) against a host loop of lf_dt and the two stages."""
    cfg = _cfg(197, 61, *bc)
    U = workloads.random_state(197, 61, seed=11, rough=False)
    S = solver_for(cfg)
    d = to_dev(U)
    t, n, dts = S.advance(d, 0.0, math.inf, max_steps=steps, dts_capacity=steps)
    assert n == steps
    e = to_dev(U)
    for k in range(steps):
        dt = S.dt(e)
        assert dt == dts[k]
        e = _two_stage(S, e, dt)
    assert np.array_equal(to_host(d), to_host(e))


def test_advance_clamped_end_and_totals():
    """Runs ending on the clamped step with an odd and an even count keep
    the result in the caller's buffer, and conservation holds."""
    U, cfg = workloads.vortex(128)
    S = solver_for(cfg)
    for t_end in (0.05, 0.06):
        d = to_dev(U)
        tot0 = S.totals(d)
        t, n, dts = S.advance(d, 0.0, t_end, dts_capacity=1000)
        assert t == t_end and abs(dts.sum() - t_end) < 1e-15
        e = to_dev(U)
        for k in range(n):
            e = _two_stage(S, e, dts[k])
        assert np.array_equal(to_host(d), to_host(e))
        tot1 = S.totals(d)
        assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(tot0))


def test_single_pass_full_size_bitwise():
    """Kelvin-Helmholtz at 16384^2, the benchmark's launch: one step of
    each path, compared bit for bit on the whole grid (on the device)."""
    import torch
    U, cfg = workloads.kelvin_helmholtz_torch(16384)
    S = solver_for(cfg)
    dt = S.dt(U)
    out = S.empty_state()
    S.step(U, out, dt)
    ref = _two_stage(S, U, dt)
    assert torch.equal(out, ref)


@pytest.mark.parametrize("ns", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (9, 1), (57, 33), (225, 40), (449, 66)])
def test_single_pass_step_bitwise_fractions(shape, bc, dtype, ns):
    """With mass fractions the single pass carries them through the same
    window and lane shifts as the stage kernel: bitwise the same."""
    nx, ny = shape
    cfg = dict(_cfg(nx, ny, *bc), ns=ns)
    U = workloads.random_state_fractions(nx, ny, ns, seed=nx * 5 + ny + ns + bc[0] + 2 * bc[1])
    S = solver_for(cfg, dtype)
    d = to_dev(U, dtype)
    dt = S.dt(d)
    out = S.empty_state()
    S.step(d, out, dt)
    assert np.array_equal(to_host(out), to_host(_two_stage(S, d, dt)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (9, 1), (57, 33), (225, 40)])
def test_step_save_and_adjoint_ustar_bitwise(shape, bc, dtype):
    """lf_step_save writes lf_step's U^{n+1} and lf_stage(1)'s U*, and
    lf_adjoint_step_ustar on that U* gives lf_adjoint_step's result."""
    import torch
    nx, ny = shape
    cfg = _cfg(nx, ny, *bc)
    U = workloads.random_state(nx, ny, seed=nx + 3 * ny + bc[0])
    S = solver_for(cfg, dtype)
    d = to_dev(U, dtype)
    dt = S.dt(d)
    out, us = S.empty_state(), S.empty_state()
    S.step_save(d, out, us, dt)
    ref_out, ref_us = S.empty_state(), S.empty_state()
    S.step(d, ref_out, dt)
    S.stage(1, d, ref_us, dt)
    assert torch.equal(out, ref_out) and torch.equal(us, ref_us)
    lam = to_dev(np.random.default_rng(3).standard_normal(U.shape), dtype)
    a, b = S.empty_state(), S.empty_state()
    S.adjoint_step(d, dt, lam, a)
    S.adjoint_step_ustar(d, us, dt, lam, b)
    assert torch.equal(a, b)
