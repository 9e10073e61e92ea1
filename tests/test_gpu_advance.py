"""GPU: the time loop of lf_advance at its edges, against the oracle's
lfo_advance (the same loop: dt from the state, clamped to t_end, stop on a
non-physical state).

  * empty loops (t0 >= t_end, max_steps = 0) leave the state untouched;
  * a non-physical initial state is refused before any step;
  * a run that turns non-physical stops at the same step as the oracle and
    reports it;
  * a dt record shorter than the run keeps the first steps' dts;
  * a run longer than the device's dt ring (4096 steps, several host
    batches, an odd step count so the result comes back from the second
    buffer) matches the oracle step for step.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import oracle_params, rel_linf, solver_for, to_dev, to_host

pytestmark = pytest.mark.gpu


def _cfg(n, bc=0, cfl=0.5):
    return dict(nx=n, ny=n, dx=1.0 / n, dy=1.0 / n, gamma=1.4, cfl=cfl, beta=1.5, bc_x=bc, bc_y=bc)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_empty_loops_leave_state(dtype):
    cfg = _cfg(40)
    U = workloads.random_state(40, 40, seed=2, rough=False)
    S = solver_for(cfg, dtype)
    d = to_dev(U, dtype)
    before = to_host(d)
    t, n, _ = S.advance(d, 0.5, 0.5)
    assert n == 0 and t == 0.5
    t, n, _ = S.advance(d, 0.0, 1.0, max_steps=0)
    assert n == 0 and t == 0.0
    assert np.array_equal(to_host(d), before)


def test_nonphysical_initial_state_refused():
    import paper_1607_08710_amd as L
    cfg = _cfg(40)
    U = workloads.random_state(40, 40, seed=3)
    U[3, 7, 9] = 0.5 * (U[1, 7, 9] ** 2 + U[2, 7, 9] ** 2) / U[0, 7, 9] - 1e-3  # p < 0
    S = solver_for(cfg)
    d = to_dev(U)
    with pytest.raises(L.NonPhysicalState):
        S.advance(d, 0.0, 1.0, max_steps=5)
    assert np.array_equal(to_host(d), U)


def test_run_that_turns_nonphysical_stops_there():
    """The two-rarefaction tube at CFL 2.5 (far above its stable range)
    loses positivity in its first step, whatever the rounding; the loop
    stops after that step and reports it, with the state it produced."""
    import paper_1607_08710_amd as L
    U, cfg = workloads.paper_tube("two_rarefaction", 200, cfl=2.5)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, cfg["t_end"])
    assert rco == oracle.ERR_NONPHYSICAL and no == 1
    S = solver_for(cfg)
    d = to_dev(U)
    with pytest.raises(L.NonPhysicalState) as info:
        S.advance(d, 0.0, cfg["t_end"], dts_capacity=100)
    assert info.value.steps == 1 and info.value.t == to
    # the state left is the one the step produced (an odd count: it came
    # back from the workspace buffer)
    rc, dt = oracle.dt(P, U)
    ref = S.empty_state()
    S.step(to_dev(U), ref, dt)
    assert np.array_equal(to_host(d), to_host(ref), equal_nan=True)
    Ug = to_host(d)
    rho, p = Ug[0], 0.4 * (Ug[3] - 0.5 * (Ug[1] ** 2 + Ug[2] ** 2) / Ug[0])
    assert not np.all(np.isfinite(Ug) & (rho > 0) & (p > 0))


def test_short_dt_record():
    cfg = _cfg(48)
    U = workloads.random_state(48, 48, seed=4, rough=False)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, 1.0, max_steps=30)
    S = solver_for(cfg)
    d = to_dev(U)
    t, n, dts = S.advance(d, 0.0, 1.0, max_steps=30, dts_capacity=7)
    assert n == 30 and len(dts) == 7
    np.testing.assert_allclose(dts, dto[:7], rtol=1e-12)


def test_run_longer_than_dt_ring():
    """5001 steps on a smooth periodic 24^2 state (odd count: the result
    comes back from the workspace buffer)."""
    cfg = _cfg(24, cfl=0.4)
    U = workloads.random_state(24, 24, seed=6, rough=False)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, math.inf, max_steps=5001)
    assert rco == 0 and no == 5001
    S = solver_for(cfg)
    d = to_dev(U)
    t, n, dts = S.advance(d, 0.0, math.inf, max_steps=5001, dts_capacity=6000)
    assert n == 5001 and len(dts) == 5001
    np.testing.assert_allclose(dts, dto, rtol=1e-10)
    assert np.all(rel_linf(to_host(d), Uo) <= 1e-10)
