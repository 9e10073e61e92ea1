"""GPU parity of the conservative-variable reconstruction (the ablation of
Sec. 5's primitive reconstruction) through the C ABI against the FP64
oracle: residual and step on rough random states (every limiter branch
and both upwind sides) over wave tiles, ragged tails and all boundary
pairs; the single-pass kernel bitwise against the two stages; whole runs
of Sod (long-run bar, as for the primitive scheme) and the vortex; FP32.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import oracle_params, rel_l1, rel_linf, solver_for, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(130, 70), (61, 5), (1, 9), (9, 1), (121, 33), (225, 40)]
BCS = [(0, 0), (1, 1), (0, 1), (1, 0)]


def _cfg(nx, ny, bcx, bcy, beta=1.5):
    d = 1.0 / max(nx, ny)
    return dict(nx=nx, ny=ny, dx=d, dy=d, gamma=1.4, cfl=0.5, beta=beta, bc_x=bcx, bc_y=bcy, recon=1)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", BCS)
def test_residual_conservative_f64(shape, bc):
    nx, ny = shape
    cfg = _cfg(nx, ny, *bc)
    U = workloads.random_state(nx, ny, seed=nx * 1000 + ny + 7 * bc[0] + 13 * bc[1] + 5)
    S = solver_for(cfg)
    R = S.empty_state()
    S.residual(to_dev(U), R)
    err = rel_linf(to_host(R), oracle.residual(oracle_params(cfg), U))
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("beta", [0.0, 1.0, 1.5, 2.0])
@pytest.mark.parametrize("bc", BCS)
def test_step_conservative_f64(beta, bc):
    cfg = _cfg(130, 70, *bc, beta)
    U = workloads.random_state(130, 70, seed=int(9 + 10 * beta + bc[0] + 2 * bc[1]))
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U)
    S = solver_for(cfg)
    d = to_dev(U)
    out = S.empty_state()
    S.step(d, out, dt)  # single pass
    err = rel_linf(to_host(out), oracle.step(P, U, dt))
    assert np.all(err <= 1e-12), err
    Us, ref = S.empty_state(), S.empty_state()
    S.stage(1, d, Us, dt)
    S.stage(2, Us, ref, dt, base=d)
    assert np.array_equal(to_host(out), to_host(ref))


@pytest.mark.parametrize("beta", [0.0, 1.5, 2.0])
def test_step_conservative_f32(beta):
    """FP32, the limiter's end points included: for beta = 0 the FP32
    limiter returns minmod, and only the zero weight of the slopes in the
    face values makes the step first order."""
    cfg = _cfg(130, 70, 1, 0, beta)
    U = workloads.random_state(130, 70, seed=71 + int(10 * beta))
    U32 = U.astype(np.float32).astype(np.float64)
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U32)
    S = solver_for(cfg, "f32")
    out = S.empty_state()
    S.step(to_dev(U32, "f32"), out, dt)
    err = rel_l1(to_host(out), oracle.step(P, U32, dt))
    assert np.all(err <= 2e-6), err


def test_sod_conservative_advance_f64():
    U, cfg = workloads.sod()
    cfg = dict(cfg, recon=1)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, cfg["t_end"])
    S = solver_for(cfg)
    d = to_dev(U)
    t, n, dts = S.advance(d, 0.0, cfg["t_end"], dts_capacity=10000)
    assert rco == 0 and n == no and t == to
    Ug = to_host(d)
    assert np.all(rel_linf(Ug, Uo) <= 1e-11), rel_linf(Ug, Uo)
    assert np.all(rel_l1(Ug, Uo) <= 3e-13), rel_l1(Ug, Uo)


def test_vortex_conservative_advance_f64():
    U, cfg = workloads.vortex(128)
    cfg = dict(cfg, recon=1)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, cfg["t_end"])
    S = solver_for(cfg)
    d = to_dev(U)
    t, n, _ = S.advance(d, 0.0, cfg["t_end"], dts_capacity=10000)
    assert n == no and t == to
    assert np.all(rel_linf(to_host(d), Uo) <= 1e-11)


def test_adjoint_refuses_conservative():
    import paper_1607_08710_amd as L
    cfg = _cfg(64, 32, 0, 0)
    S = solver_for(cfg)
    U = to_dev(workloads.random_state(64, 32, seed=1))
    out = S.empty_state()
    with pytest.raises(L.LFError):
        S.adjoint_step(U, 1e-3, U, out)
