"""Invariants of the oracle's grid operators that the scheme fixes exactly.

  * free-stream preservation: a uniform state is a bitwise fixed point
    (every face computes identical bits, so the flux balance of eq. (11)
    vanishes exactly);
  * conservation under periodic boundaries (telescoping flux balance);
  * x/y transpose symmetry, bitwise, with dx = dy;
  * the 400x4 Sod problem stays one-dimensional (identical rows, rho v == 0);
  * the four-quadrant problem keeps its diagonal mirror symmetry;
  * the non-physical flag of the CFL reduction.
"""
import numpy as np
import pytest

import oracle
import workloads
from conftest import params_from


def _P(nx, ny, bcx=oracle.PERIODIC, bcy=oracle.PERIODIC, d=0.01, **kw):
    return oracle.Params(nx, ny, d, d, bc_x=bcx, bc_y=bcy, **kw)


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_free_stream_bitwise(oracle_lib, bcx, bcy):
    rng = np.random.default_rng(bcx * 2 + bcy)
    for _ in range(3):
        rho, u, v, p = rng.uniform(0.2, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 2)
        U = workloads.prim_to_cons(1.4, np.full((7, 9), rho), u, v, p)
        P = _P(9, 7, bcx, bcy)
        assert np.array_equal(oracle_lib.residual(P, U), np.zeros_like(U))
        rc, dt = oracle_lib.dt(P, U)
        U2 = oracle_lib.step(P, U, dt)
        assert np.array_equal(U2, U)


@pytest.mark.parametrize("rough", [True, False])
def test_conservation_periodic(oracle_lib, rough):
    U = workloads.random_state(40, 24, seed=5, rough=rough)
    P = _P(40, 24)
    t0 = oracle_lib.totals(P, U)
    Uf, t, n, dts, rc = oracle_lib.advance(P, U, 0.0, 1.0, max_steps=25)
    assert rc == 0 and n == 25
    t1 = oracle_lib.totals(P, Uf)
    scale = np.abs(U).sum(axis=(1, 2)) * P.dx * P.dy
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t1 - t0) / scale


def test_residual_sums_to_zero_periodic(oracle_lib):
    U = workloads.random_state(33, 17, seed=8)
    R = oracle_lib.residual(_P(33, 17), U)
    scale = np.abs(R).sum(axis=(1, 2))
    assert np.all(np.abs(R.sum(axis=(1, 2))) <= 1e-12 * scale)


def _transpose_state(U):
    T = np.ascontiguousarray(np.transpose(U, (0, 2, 1)))
    T[[1, 2]] = T[[2, 1]]  # swap x and y momentum
    return T


@pytest.mark.parametrize("bc", [oracle.PERIODIC, oracle.TRANSMISSIVE])
def test_transpose_symmetry_bitwise(oracle_lib, bc):
    U = workloads.random_state(24, 24, seed=13)
    P = _P(24, 24, bc, bc)
    rc, dt = oracle_lib.dt(P, U)
    U1 = oracle_lib.step(P, U, dt)
    U1t = oracle_lib.step(P, _transpose_state(U), dt)
    assert np.array_equal(_transpose_state(U1), U1t)


def test_transpose_symmetry_rectangular(oracle_lib):
    """Sod along x on 400x4 equals Sod along y on 4x400, transposed."""
    Ux, cx = workloads.sod(axis="x")
    Uy, cy = workloads.sod(axis="y")
    assert np.array_equal(_transpose_state(Ux), Uy)
    Px, Py = params_from(cx), params_from(cy)
    fx, tx, nx_, dtx, rcx = oracle_lib.advance(Px, Ux, 0.0, 0.05)
    fy, ty, ny_, dty, rcy = oracle_lib.advance(Py, Uy, 0.0, 0.05)
    assert rcx == rcy == 0 and nx_ == ny_ and np.array_equal(dtx, dty)
    assert np.array_equal(_transpose_state(fx), fy)


def test_sod_stays_one_dimensional(oracle_lib):
    U, cfg = workloads.sod()
    Uf, t, n, dts, rc = oracle_lib.advance(params_from(cfg), U, 0.0, cfg["t_end"])
    assert rc == 0 and t == cfg["t_end"]
    for j in range(1, cfg["ny"]):
        assert np.array_equal(Uf[:, j], Uf[:, 0])
    assert np.all(Uf[2] == 0.0)


def test_four_quadrant_diagonal_symmetry(oracle_lib):
    U, cfg = workloads.four_quadrant(64)
    assert np.array_equal(_transpose_state(U), U)
    Uf, t, n, dts, rc = oracle_lib.advance(params_from(cfg), U, 0.0, 1.0, max_steps=40)
    assert rc == 0 and n == 40
    assert np.array_equal(_transpose_state(Uf), Uf)
    assert np.all(Uf[0] > 0)


def test_nonphysical_flag(oracle_lib):
    U = workloads.random_state(8, 8, seed=2)
    P = _P(8, 8)
    assert oracle_lib.dt(P, U)[0] == 0
    bad = U.copy()
    bad[3, 4, 5] = 0.5 * (bad[1, 4, 5] ** 2 + bad[2, 4, 5] ** 2) / bad[0, 4, 5] - 1e-3  # p < 0
    assert oracle_lib.dt(P, bad)[0] == oracle.ERR_NONPHYSICAL
    bad = U.copy()
    bad[0, 1, 1] = -1.0
    assert oracle_lib.dt(P, bad)[0] == oracle.ERR_NONPHYSICAL
    bad = U.copy()
    bad[2, 7, 0] = np.nan
    assert oracle_lib.dt(P, bad)[0] == oracle.ERR_NONPHYSICAL


def test_advance_clamps_to_t_end(oracle_lib):
    U = workloads.random_state(16, 16, seed=4, rough=False)
    P = _P(16, 16, d=1.0 / 16)
    Uf, t, n, dts, rc = oracle_lib.advance(P, U, 0.0, 0.05)
    assert rc == 0 and t == 0.05
    assert np.all(dts[:-1] > 0) and dts[-1] <= dts[-2] * 1.5
    assert abs(dts.sum() - 0.05) < 1e-15


def test_totals_against_exact_sum(oracle_lib):
    """lfo_totals is a compensated sum times dx*dy: against math.fsum (the
    correctly rounded sum) it agrees to one rounding of the product, also
    on data built to cancel."""
    import math
    rng = np.random.default_rng(12)
    U = rng.standard_normal((4, 37, 53)) * 10.0 ** rng.integers(-8, 8, size=(4, 37, 53))
    P = _P(53, 37, d=0.25)
    got = oracle_lib.totals(P, U)
    for f in range(4):
        exact = math.fsum(U[f].ravel()) * 0.25 * 0.25
        assert got[f] == pytest.approx(exact, rel=4e-16, abs=1e-300)
