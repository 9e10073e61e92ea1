"""The conservative-variable reconstruction (the ablation of the primitive
reconstruction of Sec. 5): limited slopes of (rho, rho u, rho v, rho E),
face states converted to primitive variables for eqs. (13)-(14), and the
reconstructed conservative vector of the upwind side in eq. (12).

Pins, independent of the oracle's formulas:
  * linear conservative data: with beta >= 1 the limited slope of a linear
    profile is its difference, so both face states are the midpoint state
    and the face flux is the Euler flux of that state, written out below
    from its definition (this distinguishes it from the primitive
    reconstruction, whose face state of the same data differs);
  * uniform velocity and pressure with varying density: rho u and rho E
    are affine in rho, the slopes scale with them, and the scheme equals
    the primitive one to rounding (itself pinned elsewhere);
  * free-stream preservation (bitwise), conservation under periodic
    boundaries, accuracy on Sod against the exact solution, second-order
    convergence on the isentropic vortex.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import params_from

G = 1.4


def _euler_flux_x(q):
    rho, mx, my, E = q
    u, v = mx / rho, my / rho
    p = (G - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    return np.array([mx, mx * u + p, my * u, (E + p) * u])


@pytest.mark.parametrize("beta", [1.0, 1.5, 2.0])
def test_linear_data_gives_midpoint_euler_flux(oracle_lib, beta):
    nx, ny, dx = 24, 3, 0.05
    x = workloads.cell_centres(nx, 0.0, nx * dx)
    q = np.array([1.0 + 0.1 * x, 0.2 + 0.05 * x, 0.1 - 0.02 * x, 3.0 + 0.1 * x])  # linear in x
    U = np.ascontiguousarray(np.repeat(q[:, None, :], ny, axis=1))
    P = oracle.Params(nx, ny, dx, dx, beta=beta, bc_x=oracle.TRANSMISSIVE, bc_y=oracle.PERIODIC,
                      recon=oracle.RECON_CONSERVATIVE)
    R = oracle_lib.residual(P, U)
    # interior faces i+1/2 with two cells of data on each side: midpoint state
    for i in range(2, nx - 3):
        fe = _euler_flux_x(0.5 * (q[:, i] + q[:, i + 1]))
        fw = _euler_flux_x(0.5 * (q[:, i - 1] + q[:, i]))
        ref = (fe - fw) / dx
        assert np.allclose(R[:, 0, i], ref, rtol=0, atol=1e-12 * np.abs(fe).max() / dx), (i, R[:, 0, i], ref)
    # the primitive reconstruction of the same data does not give it
    Rp = oracle_lib.residual(P.with_(recon=oracle.RECON_PRIMITIVE), U)
    assert np.abs(Rp[3, 0, 5:15] - R[3, 0, 5:15]).max() > 1e-6


@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_uniform_velocity_pressure_equals_primitive(oracle_lib, bc):
    rng = np.random.default_rng(3)
    nx, ny = 30, 22
    rho = rng.uniform(0.5, 2.0, (ny, nx))
    U = workloads.prim_to_cons(G, rho, 0.7, -0.4, 1.3)
    P = oracle.Params(nx, ny, 0.03, 0.04, bc_x=bc[0], bc_y=bc[1], recon=oracle.RECON_CONSERVATIVE)
    Rc = oracle_lib.residual(P, U)
    Rp = oracle_lib.residual(P.with_(recon=oracle.RECON_PRIMITIVE), U)
    scale = np.abs(Rp).reshape(4, -1).max(axis=1)
    assert np.all(np.abs(Rc - Rp).reshape(4, -1).max(axis=1) <= 1e-12 * scale)


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1)])
def test_free_stream_and_conservation(oracle_lib, bc):
    U = workloads.prim_to_cons(G, np.full((9, 11), 1.2), 0.3, -0.6, 0.8)
    P = oracle.Params(11, 9, 0.1, 0.1, bc_x=bc[0], bc_y=bc[1], recon=oracle.RECON_CONSERVATIVE)
    assert np.array_equal(oracle_lib.residual(P, U), np.zeros_like(U))
    if bc == (0, 0):
        V = workloads.random_state(40, 24, seed=6, rough=False)
        Pp = oracle.Params(40, 24, 0.01, 0.01, recon=oracle.RECON_CONSERVATIVE)
        t0 = oracle_lib.totals(Pp, V)
        Vf, t, n, dts, rc = oracle_lib.advance(Pp, V, 0.0, 1.0, max_steps=20)
        assert rc == 0 and n == 20
        scale = np.abs(V).sum(axis=(1, 2)) * 0.01 * 0.01
        assert np.all(np.abs(oracle_lib.totals(Pp, Vf) - t0) <= 1e-13 * scale)


def test_sod_against_exact(oracle_lib):
    U, cfg = workloads.paper_tube("sod", 400)
    P = params_from(cfg, recon=oracle.RECON_CONSERVATIVE)
    Uf, t, n, dts, rc = oracle_lib.advance(P, U, 0.0, cfg["t_end"])
    assert rc == 0
    w = np.array([oracle_lib.cons_to_prim(G, Uf[:, 0, i]) for i in range(400)])
    assert np.all(w[:, 0] > 0) and np.all(w[:, 3] > 0)
    x = workloads.cell_centres(400, 0.0, 1.0)
    er, eu, ep, _, _ = oracle_lib.exact_riemann(G, cfg["left"], cfg["right"], (x - 0.5) / cfg["t_end"])
    err = [np.mean(np.abs(w[:, 0] - er)) / er.max(), np.mean(np.abs(w[:, 3] - ep)) / ep.max()]
    assert max(err) < 0.01, err


def test_vortex_second_order(oracle_lib):
    """Density L1 error at t = 0.5 on 128^2 and 256^2 (coarser grids do not
    resolve the unit-radius core: the limiter clips its extremum and both
    reconstructions converge irregularly there)."""
    errs = []
    for n in (128, 256):
        U, cfg = workloads.vortex(n)
        t_end = 0.5
        P = params_from(cfg, recon=oracle.RECON_CONSERVATIVE)
        Uf, t, steps, dts, rc = oracle_lib.advance(P, U, 0.0, t_end)
        assert rc == 0
        Ue, _ = workloads.vortex(n, t=t_end)
        errs.append(np.abs(Uf[0] - Ue[0]).mean())
    order = math.log2(errs[0] / errs[1])
    assert order > 1.7, (errs, order)


def test_linearisations_refuse_conservative(oracle_lib):
    U = workloads.random_state(8, 8, seed=1)
    P = oracle.Params(8, 8, 0.1, 0.1, recon=oracle.RECON_CONSERVATIVE)
    with pytest.raises(RuntimeError):
        oracle_lib.residual_vjp(P, U, U)
    with pytest.raises(RuntimeError):
        oracle_lib.residual_jvp(P, U, U)
