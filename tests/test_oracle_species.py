"""Passive mass fractions in the oracle: the conservative transport
d(rho y_k)/dt + div(rho y_k u) = 0 that the paper prefers to the advective
form for multimaterial flow (Sec. 7), discretised like the mass flux of
eq. (12) with the reconstruction of Sec. 5.

Pins, each independent of the oracle's own formulas:
  * special case: with uniform rho, p and velocity the Euler fields are a
    fixed point and the fraction follows the textbook upwind MUSCL scheme
    for linear advection (minmod / superbee / first order, Heun in time),
    written out below from its textbook definition;
  * consistency with mass: a uniform fraction stays uniform on any flow,
    and two complementary fractions keep summing to rho;
  * conservation of every rho y_k under periodic boundaries;
  * the Euler fields are untouched by the extra fields (bitwise);
  * the material interface of Sod travels with the exact contact speed,
    and the fractions stay in [0, 1] (the scheme is TVD for the fraction).
"""
import numpy as np
import pytest

import oracle
import workloads
from conftest import params_from


# ---- textbook linear advection (independent of the oracle) ------------------

def _limited_slope(a, b, beta):
    """Textbook limited slopes: 0 (first order), minmod, superbee."""
    s = 0.5 * (np.sign(a) + np.sign(b))
    if beta == 0.0:
        return np.zeros_like(a)
    if beta == 1.0:
        return s * np.minimum(np.abs(a), np.abs(b))
    if beta == 2.0:
        return s * np.maximum(np.minimum(2 * np.abs(a), np.abs(b)),
                              np.minimum(np.abs(a), 2 * np.abs(b)))
    raise ValueError(beta)


def _upwind_flux_1d(y, vel, beta, bc):
    """Flux vel * y_face through the faces of a 1D row (face k between cells
    k-1 and k, k = 0..n), the face value reconstructed on the upwind side."""
    n = y.size
    idx = np.arange(-2, n + 2)
    idx = idx % n if bc == oracle.PERIODIC else np.clip(idx, 0, n - 1)
    e = y[idx]                       # e[m] = cell m - 2
    sl = _limited_slope(e[1:-1] - e[:-2], e[2:] - e[1:-1], beta)  # cells -1 .. n
    if vel > 0:
        yf = e[1:-2] + 0.5 * sl[:-1]    # from cell k-1, k = 0..n
    else:
        yf = e[2:-1] - 0.5 * sl[1:]     # from cell k
    return vel * yf


def _advection_rate(q, u, v, dx, dy, beta, bcx, bcy):
    """d q / dt = -(div of the upwind MUSCL fluxes) for q = rho0 * y."""
    ny, nx = q.shape
    out = np.zeros_like(q)
    for j in range(ny):
        F = _upwind_flux_1d(q[j], u, beta, bcx)
        out[j] -= (F[1:] - F[:-1]) / dx
    for i in range(nx):
        G = _upwind_flux_1d(q[:, i], v, beta, bcy)
        out[:, i] -= (G[1:] - G[:-1]) / dy
    return out


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
@pytest.mark.parametrize("u,v,bc", [(0.7, -0.4, (0, 0)), (-0.5, 0.3, (1, 1)), (0.6, 0.0, (0, 1))])
def test_reduces_to_textbook_advection(oracle_lib, beta, u, v, bc):
    U, cfg = workloads.advected_fraction(37, 23, u, v, seed=int(10 * beta) + 3, bc=bc, beta=beta)
    P = params_from(cfg)
    rho0 = U[0, 0, 0]
    q = U[4].copy()
    rc, dt = oracle_lib.dt(P, U)
    assert rc == 0
    for _ in range(6):
        U = oracle_lib.step(P, U, dt)
        # textbook Heun on q
        k1 = _advection_rate(q, u, v, cfg["dx"], cfg["dy"], beta, *bc)
        qs = q + dt * k1
        k2 = _advection_rate(qs, u, v, cfg["dx"], cfg["dy"], beta, *bc)
        q = q + 0.5 * dt * (k1 + k2)
    assert np.all(U[0] == rho0)  # the Euler fields stay a fixed point
    err = np.abs(U[4] - q).max() / np.abs(q).max()
    assert err <= 1e-13, err


def test_uniform_fraction_stays_uniform(oracle_lib):
    U = workloads.random_state(31, 19, seed=3)
    U = workloads.with_fractions(U, [0.3])
    P = oracle.Params(31, 19, 0.02, 0.02, bc_x=1, bc_y=0, ns=1)
    for _ in range(5):
        rc, dt = oracle_lib.dt(P, U)
        U = oracle_lib.step(P, U, dt)
    assert np.abs(U[4] / U[0] - 0.3).max() <= 1e-14


def test_complementary_fractions_sum_to_density(oracle_lib):
    U = workloads.random_state_fractions(29, 17, 1, seed=9)
    U = np.concatenate([U, (U[0] - U[4])[None]], axis=0)
    P = oracle.Params(29, 17, 0.02, 0.03, bc_x=0, bc_y=1, ns=2)
    for _ in range(5):
        rc, dt = oracle_lib.dt(P, U)
        U = oracle_lib.step(P, U, dt)
    assert np.abs(U[4] + U[5] - U[0]).max() <= 1e-13 * np.abs(U[0]).max()


def test_fraction_conservation_periodic(oracle_lib):
    U = workloads.random_state_fractions(40, 24, 3, seed=5)
    P = oracle.Params(40, 24, 0.01, 0.01, ns=3)
    t0 = oracle_lib.totals(P, U)
    assert t0.shape == (7,)
    Uf, t, n, dts, rc = oracle_lib.advance(P, U, 0.0, 1.0, max_steps=20)
    assert rc == 0 and n == 20
    t1 = oracle_lib.totals(P, Uf)
    scale = np.abs(U).sum(axis=(1, 2)) * P.dx * P.dy
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t1 - t0) / scale


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1)])
def test_euler_fields_unchanged(oracle_lib, bc):
    U = workloads.random_state_fractions(26, 21, 2, seed=12)
    P2 = oracle.Params(26, 21, 0.02, 0.02, bc_x=bc[0], bc_y=bc[1], ns=2)
    P0 = P2.with_(ns=0)
    assert np.array_equal(oracle_lib.residual(P2, U)[:4], oracle_lib.residual(P0, U[:4]))
    rc, dt = oracle_lib.dt(P2, U)
    assert np.array_equal(oracle_lib.step(P2, U, dt)[:4], oracle_lib.step(P0, U[:4], dt))


def test_sod_interface_follows_contact(oracle_lib):
    U, cfg = workloads.sod_interface()
    P = params_from(cfg)
    Uf, t, n, dts, rc = oracle_lib.advance(P, U, 0.0, cfg["t_end"])
    assert rc == 0
    y1 = Uf[4, 0] / Uf[0, 0]
    y2 = Uf[5, 0] / Uf[0, 0]
    # TVD for the fraction: no new extrema (up to rounding)
    assert y1.min() >= -1e-12 and y1.max() <= 1 + 1e-12
    # complementary to rounding, accumulated over the 555 steps
    assert np.abs(y1 + y2 - 1.0).max() <= 1e-11
    # the interface (y = 1/2) sits at the exact contact position
    *_, us = oracle_lib.exact_riemann(1.4, workloads.SOD_LEFT, workloads.SOD_RIGHT, np.zeros(1))
    x = workloads.cell_centres(cfg["nx"], 0.0, 1.0)
    k = int(np.argmax(y1 < 0.5))
    xi = x[k - 1] + (y1[k - 1] - 0.5) / (y1[k - 1] - y1[k]) * (x[k] - x[k - 1])
    assert abs(xi - (0.5 + us * cfg["t_end"])) < 1.0 * cfg["dx"], (xi, 0.5 + us * cfg["t_end"])


def test_linearisations_refuse_fractions(oracle_lib):
    U = workloads.random_state_fractions(8, 8, 1, seed=1)
    P = oracle.Params(8, 8, 0.1, 0.1, ns=1)
    with pytest.raises(RuntimeError):
        oracle_lib.residual_vjp(P, U, U)
    with pytest.raises(RuntimeError):
        oracle_lib.adjoint_step(P, U, 1e-3, U)
