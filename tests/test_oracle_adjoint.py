"""Pins of the oracle's linearisation at frozen dt.

  * brute force: on a 6x6 grid over 3 steps the full Jacobian of the step
    map from central finite differences of the (pinned) forward oracle
    matches every column of the tangent-linear model and every row of the
    adjoint;
  * dot-product identity <J v, w> = <v, J^T w> between the tangent-linear
    and adjoint steps, and between the residual JVP and VJP;
  * the misfit gradient of the adjoint workload (smooth density, uniform
    velocity and pressure) against central differences along seeded
    directions;
  * the reach of one adjoint step: a patch of radius 7 around a cell gives
    the full-grid value at its centre, radius 6 does not.
"""
import numpy as np
import pytest

import oracle
import workloads


def _P(nx, ny, bcx, bcy, d=0.1):
    return oracle.Params(nx, ny, d, d, bc_x=bcx, bc_y=bcy)


def _forward(P, U, dt, steps):
    for _ in range(steps):
        U = oracle.step(P, U, dt)
    return U


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 1), (0, 1)])
def test_bruteforce_jacobian_6x6(oracle_lib, bcx, bcy):
    P = _P(6, 6, bcx, bcy)
    U0 = workloads.random_state(6, 6, seed=21 + bcx + 2 * bcy)
    rc, dt = oracle_lib.dt(P, U0)
    dt *= 0.8
    steps = 3
    n = U0.size
    # FD Jacobian
    Jfd = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        h = 1e-6 * max(1.0, abs(U0.flat[k]))
        e[k] = h
        fp = _forward(P, U0 + e.reshape(U0.shape), dt, steps)
        fm = _forward(P, U0 - e.reshape(U0.shape), dt, steps)
        Jfd[:, k] = ((fp - fm) / (2 * h)).ravel()
    # tangent-linear columns
    states = [U0]
    for _ in range(steps - 1):
        states.append(oracle_lib.step(P, states[-1], dt))
    Jtl = np.empty((n, n))
    for k in range(n):
        d = np.zeros(n)
        d[k] = 1.0
        d = d.reshape(U0.shape)
        for s in range(steps):
            d = oracle_lib.tlm_step(P, states[s], dt, d)
        Jtl[:, k] = d.ravel()
    # adjoint rows
    Jad = np.empty((n, n))
    for r in range(n):
        lam = np.zeros(n)
        lam[r] = 1.0
        lam = lam.reshape(U0.shape)
        for s in reversed(range(steps)):
            lam = oracle_lib.adjoint_step(P, states[s], dt, lam)
        Jad[r, :] = lam.ravel()
    scale = np.abs(Jtl).max()
    assert np.abs(Jtl - Jfd).max() <= 2e-7 * scale, np.abs(Jtl - Jfd).max() / scale
    assert np.abs(Jad - Jtl).max() <= 1e-13 * scale


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 1), (1, 0)])
def test_dot_product_step(oracle_lib, bcx, bcy):
    P = _P(31, 20, bcx, bcy, d=0.05)
    U = workloads.random_state(31, 20, seed=40 + bcx)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(U.shape)
    w = rng.standard_normal(U.shape)
    rc, dt = oracle_lib.dt(P, U)
    Jv = oracle_lib.tlm_step(P, U, dt, v)
    JTw = oracle_lib.adjoint_step(P, U, dt, w)
    a, b = np.vdot(Jv, w), np.vdot(v, JTw)
    assert abs(a - b) <= 1e-13 * (np.abs(Jv).sum() * np.abs(w).max()), (a, b)
    # residual pair
    Rv = oracle_lib.residual_jvp(P, U, v)
    RTw = oracle_lib.residual_vjp(P, U, w)
    a, b = np.vdot(Rv, w), np.vdot(v, RTw)
    assert abs(a - b) <= 1e-13 * (np.abs(Rv).sum() * np.abs(w).max()), (a, b)


def test_residual_jvp_matches_fd(oracle_lib):
    P = _P(12, 10, 0, 1, d=0.05)
    U = workloads.random_state(12, 10, seed=77)
    d = np.random.default_rng(0).standard_normal(U.shape)
    h = 1e-6
    fd = (oracle_lib.residual(P, U + h * d) - oracle_lib.residual(P, U - h * d)) / (2 * h)
    jv = oracle_lib.residual_jvp(P, U, d)
    assert np.abs(fd - jv).max() <= 1e-6 * np.abs(jv).max()


def _misfit_gradient(P, U0, rho_tgt, dt, steps, uvp):
    states = [U0]
    for _ in range(steps):
        states.append(oracle.step(P, states[-1], dt))
    rhoN = states[-1][0]
    J = 0.5 * P.dx * P.dy * np.sum((rhoN - rho_tgt) ** 2)
    lam = np.zeros_like(U0)
    lam[0] = P.dx * P.dy * (rhoN - rho_tgt)
    for s in reversed(range(steps)):
        lam = oracle.adjoint_step(P, states[s], dt, lam)
    u, v, _p = uvp
    # d U0 / d rho0 at fixed (u, v, p) = (1, u, v, (u^2+v^2)/2)
    g = lam[0] + u * lam[1] + v * lam[2] + 0.5 * (u * u + v * v) * lam[3]
    return J, g


def test_misfit_gradient_fd(oracle_lib):
    """The limited step map is only piecewise smooth: on smooth data the
    Sweby limiter sits next to its |a| = |b| kink, and a finite-difference
    pair that straddles a kink in any cell differs from the one-sided
    derivative the adjoint follows.  Central differences are therefore
    taken at four step sizes; a correct gradient agrees to 1e-6 at the
    step sizes that cross no kink, a wrong one at none."""
    n, steps = 48, 12
    U0, rho_tgt, cfg = workloads.adjoint_case(n)
    P = oracle.Params(n, n, cfg["dx"], cfg["dy"], bc_x=0, bc_y=0)
    rc, dt = oracle_lib.dt(P, U0)
    J, g = _misfit_gradient(P, U0, rho_tgt, dt, steps, (0.2, 0.2, 1.0))
    rho0 = U0[0]

    def Jof(r):
        U = workloads.prim_to_cons(1.4, r, 0.2, 0.2, 1.0)
        rN = _forward(P, U, dt, steps)[0]
        return 0.5 * P.dx * P.dy * np.sum((rN - rho_tgt) ** 2)

    for d in workloads.fd_directions(n, count=4):
        ad = np.sum(g * d)
        errs = []
        for eps in (1e-6, 1e-7, 3e-8, 1e-8):
            fd = (Jof(rho0 + eps * d) - Jof(rho0 - eps * d)) / (2 * eps)
            errs.append(abs(fd - ad) / abs(ad))
        assert min(errs) <= 1e-6, errs
        assert max(errs) <= 1e-4, errs


def test_adjoint_step_patch_locality(oracle_lib):
    """The reach of one adjoint step, which the full-size GPU check relies
    on: on a rough periodic 48^2 state, the adjoint step on a patch of
    radius 10 (or 7) gathered around a cell with the periodic wrap gives
    the full-grid value at the patch centre, to rounding, with transmissive
    patch edges; at radius 6 the edge reaches the centre."""
    n = 48
    U = workloads.random_state(n, n, seed=5)
    lam = np.random.default_rng(1).standard_normal(U.shape)
    P = oracle.Params(n, n, 1.0 / n, 1.0 / n, 1.4, 0.5, 1.5, oracle.PERIODIC, oracle.PERIODIC)
    rc, dt = oracle.dt(P, U)
    full = oracle.adjoint_step(P, U, dt, lam)
    scale = np.abs(full).max(axis=(1, 2))

    def worst(r):
        Pp = oracle.Params(2 * r + 1, 2 * r + 1, 1.0 / n, 1.0 / n, 1.4, 0.5, 1.5, oracle.TRANSMISSIVE,
                           oracle.TRANSMISSIVE)
        w = 0.0
        for i, j in [(0, 0), (5, 40), (47, 47), (20, 3), (33, 17)]:
            xs, ys = np.arange(i - r, i + r + 1) % n, np.arange(j - r, j + r + 1) % n
            ref = oracle.adjoint_step(Pp, np.ascontiguousarray(U[:, ys][:, :, xs]), dt,
                                      np.ascontiguousarray(lam[:, ys][:, :, xs]))[:, r, r]
            w = max(w, float(np.max(np.abs(ref - full[:, j, i]) / scale)))
        return w

    assert worst(10) <= 1e-15 and worst(7) <= 1e-15
    assert worst(6) > 1e-10
