"""GPU parity for the passive mass fractions (conservative transport of
rho y_k, Sec. 7) through the C ABI against the FP64 oracle.

Bars as for the Euler fields: FP64 within 1e-12 relative L-infinity per
field for single steps and short runs, 1e-11 / 3e-13 (L-infinity / L1) for
the 555-step Sod run (its rounding floor, measured on the oracle, is ~6e-12);
FP32 within 2e-6 relative L1 per step.  Every species count the library
instantiates (1..4) is exercised, with wave tiles, ragged tails and both
boundary conditions on each axis.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import (oracle_params, oracle_step_at, rel_l1, rel_linf, solver_for, to_dev,
                      to_host)

pytestmark = pytest.mark.gpu


def _cfg(nx, ny, bcx, bcy, ns, beta=1.5):
    d = 1.0 / max(nx, ny)
    return dict(nx=nx, ny=ny, dx=d, dy=d, gamma=1.4, cfl=0.5, beta=beta, bc_x=bcx, bc_y=bcy, ns=ns)


SHAPES = [(130, 70), (61, 5), (1, 9), (9, 1), (121, 33)]
BCS = [(0, 0), (1, 1), (0, 1), (1, 0)]


@pytest.mark.parametrize("ns", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", BCS)
def test_residual_species_f64(ns, shape, bc):
    nx, ny = shape
    cfg = _cfg(nx, ny, *bc, ns)
    U = workloads.random_state_fractions(nx, ny, ns, seed=nx * 100 + ny + ns + 7 * bc[0] + 13 * bc[1])
    S = solver_for(cfg)
    R = S.empty_state()
    S.residual(to_dev(U), R)
    ref = oracle.residual(oracle_params(cfg), U)
    err = rel_linf(to_host(R), ref)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("ns", [1, 2, 4])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("beta", [0.0, 1.0, 1.5, 2.0])
def test_step_species_f64(ns, bc, beta):
    cfg = _cfg(130, 70, *bc, ns, beta)
    U = workloads.random_state_fractions(130, 70, ns, seed=int(3 + ns + 10 * beta + bc[0] + 2 * bc[1]))
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U)
    S = solver_for(cfg)
    out = S.empty_state()
    S.step(to_dev(U), out, dt)
    err = rel_linf(to_host(out), oracle.step(P, U, dt))
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("ns", [1, 3])
@pytest.mark.parametrize("beta", [0.0, 1.5, 2.0])
def test_step_species_f32(ns, beta):
    """FP32, the limiter's end points included: for beta = 0 the FP32
    limiter returns minmod, and only the zero weight of the slopes in the
    face values (the fractions' as well) makes the step first order."""
    cfg = _cfg(130, 70, 1, 0, ns, beta)
    U = workloads.random_state_fractions(130, 70, ns, seed=50 + ns + int(10 * beta))
    U32 = U.astype(np.float32).astype(np.float64)
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U32)
    S = solver_for(cfg, "f32")
    out = S.empty_state()
    S.step(to_dev(U32, "f32"), out, dt)
    err = rel_l1(to_host(out), oracle.step(P, U32, dt))
    assert np.all(err <= 2e-6), err


def test_euler_fields_bitwise_independent_of_species():
    """The Euler fields of a state with fractions come out bit for bit as
    without them (the fractions never feed back)."""
    cfg2 = _cfg(130, 70, 1, 0, 2)
    cfg0 = _cfg(130, 70, 1, 0, 0)
    U = workloads.random_state_fractions(130, 70, 2, seed=77)
    S2, S0 = solver_for(cfg2), solver_for(cfg0)
    d2, d0 = to_dev(U), to_dev(U[:4])
    t2, n2, _ = S2.advance(d2, 0.0, 1.0, max_steps=10)
    t0, n0, _ = S0.advance(d0, 0.0, 1.0, max_steps=10)
    assert n2 == n0 == 10 and t2 == t0
    assert np.array_equal(to_host(d2)[:4], to_host(d0))


def test_uniform_fraction_stays_uniform():
    cfg = _cfg(130, 70, 1, 0, 1)
    U = workloads.with_fractions(workloads.random_state(130, 70, seed=3), [0.3])
    S = solver_for(cfg)
    d = to_dev(U)
    S.advance(d, 0.0, 1.0, max_steps=5)
    Ug = to_host(d)
    assert np.abs(Ug[4] / Ug[0] - 0.3).max() <= 1e-14


def test_sod_interface_advance_f64():
    """Sod 400x4 carrying two complementary materials, 555 steps to t = 0.2."""
    U, cfg = workloads.sod_interface()
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, cfg["t_end"])
    S = solver_for(cfg)
    d = to_dev(U)
    t, n, dts = S.advance(d, 0.0, cfg["t_end"], dts_capacity=10000)
    assert rco == 0 and n == no and t == to
    Ug = to_host(d)
    assert np.all(rel_linf(Ug, Uo) <= 1e-11), rel_linf(Ug, Uo)
    assert np.all(rel_l1(Ug, Uo) <= 3e-13), rel_l1(Ug, Uo)
    y1 = Ug[4] / Ug[0]
    assert y1.min() >= -1e-12 and y1.max() <= 1 + 1e-12


@pytest.mark.parametrize("u,v,bc", [(0.7, -0.4, (0, 0)), (-0.5, 0.3, (1, 1))])
def test_advected_fraction_f64(u, v, bc):
    U, cfg = workloads.advected_fraction(190, 75, u, v, seed=11, bc=bc)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, 1.0, max_steps=40)
    S = solver_for(cfg)
    d = to_dev(U)
    t, n, _ = S.advance(d, 0.0, 1.0, max_steps=40)
    assert n == no == 40
    assert np.all(rel_linf(to_host(d), Uo) <= 1e-12)


def test_kelvin_helmholtz_fraction_totals():
    """KH 256^2 with a material marker, 100 steps: parity, and every field
    (the marker's rho y included) conserved to FP64 rounding."""
    U, cfg = workloads.kelvin_helmholtz_fraction(256)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, 10.0, max_steps=100)
    S = solver_for(cfg)
    d = to_dev(U)
    tot0 = S.totals(d)
    assert tot0.shape == (5,)
    np.testing.assert_allclose(tot0, oracle.totals(P, U), rtol=1e-15)
    S.advance(d, 0.0, 10.0, max_steps=100)
    Ug = to_host(d)
    assert np.all(rel_linf(Ug, Uo) <= 1e-11), rel_linf(Ug, Uo)
    tot1 = S.totals(d)
    scale = np.abs(U).sum(axis=(1, 2)) * cfg["dx"] * cfg["dy"]
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * scale), (tot1 - tot0) / scale


def test_sampled_step_species_full_size():
    """Kelvin-Helmholtz at 8192^2 with two fractions (a marker and a seeded
    rough field), one step against the oracle cell by cell."""
    import torch
    n = 8192
    U, cfg = workloads.kelvin_helmholtz_torch(n)
    rng = np.random.default_rng(8193)
    x = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) / n
    marker = (torch.abs(x - 0.5) < 0.25).to(torch.float64)[:, None].expand(n, n)
    g = torch.Generator(device="cuda").manual_seed(5)
    rough = torch.rand((n, n), generator=g, device="cuda", dtype=torch.float64)
    d = torch.empty((6, n, n), dtype=torch.float64, device="cuda")
    d[:4] = U
    d[4] = U[0] * marker
    d[5] = U[0] * rough
    del U
    cfg = dict(cfg, ns=2)
    S = solver_for(cfg)
    dt = S.dt(d)
    out = S.empty_state()
    S.step(d, out, dt)
    cells = [(int(i), int(j)) for i, j in rng.integers(0, n, size=(200, 2))]
    cells += [(100, n // 4 + k) for k in range(-3, 3)] + [(0, 0), (n - 1, n - 1), (59, 3 * n // 4), (60, 5)]
    Uh = d.cpu().numpy()
    ref = oracle_step_at(Uh, cfg, dt, cells)
    Og = out.cpu().numpy()
    got = np.array([Og[:, j, i] for i, j in cells])
    scale = np.abs(Uh).reshape(6, -1).max(axis=1)
    err = np.abs(got - ref).max(axis=0) / scale
    assert np.all(err <= 1e-12), err
