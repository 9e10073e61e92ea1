"""Closed-form pin of the oracle's Heun combination on the Euler fields
(Sec. 5, items 6 and 11: U* = U^n - dt R(U^n), then U^{n+1} = U^n -
dt (R(U^n) + R(U*)) / 2).

With uniform velocity (u, v) and pressure p, the Euler system reduces to
linear advection of the density, and every conservative field is affine in
it: rho u, rho v and rho E = p/(gamma-1) + rho |u|^2 / 2.  Along such a
state the acoustic solve gives u* = u_n and p* = p on every face (eqs.
(13)-(14) with equal velocities and pressures), so the scheme's mass flux
is the upwind MUSCL flux of the density with the Sweby-limited slopes, and
one step is the textbook Heun step of that linear-advection scheme.  The
textbook scheme is written out independently of the oracle (the limiters
of the minmod and superbee special cases, beta = 1 and 2, and the first
order scheme, beta = 0).  A dropped 1/2, a corrector that uses R(U*) alone,
or a sign error in either stage changes the result by O(dt), far above the
rounding-level bar."""
import numpy as np
import pytest

import oracle
import workloads
from test_oracle_species import _advection_rate


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
@pytest.mark.parametrize("u,v,bc", [(0.3, -0.2, (0, 0)), (-0.45, 0.25, (1, 1)), (0.5, 0.1, (0, 1))])
def test_euler_heun_step_is_textbook_advection(beta, u, v, bc):
    nx, ny, gamma, p = 33, 26, 1.4, 1.0
    rng = np.random.default_rng(int(100 * beta) + 7 * bc[0] + 3 * bc[1])
    rho = rng.uniform(0.5, 1.5, size=(ny, nx))
    U = workloads.prim_to_cons(gamma, rho, u, v, p)
    P = oracle.Params(nx, ny, 1.0 / nx, 1.0 / nx, gamma, 0.5, beta, bc[0], bc[1])
    rc, dt = oracle.dt(P, U)
    assert rc == 0
    q = rho.copy()
    for _ in range(5):
        U = oracle.step(P, U, dt)
        k1 = _advection_rate(q, u, v, P.dx, P.dy, beta, *bc)
        qs = q + dt * k1
        k2 = _advection_rate(qs, u, v, P.dx, P.dy, beta, *bc)
        q = q + 0.5 * dt * (k1 + k2)
    expect = workloads.prim_to_cons(gamma, q, u, v, p)
    for f in range(4):
        err = np.abs(U[f] - expect[f]).max() / np.abs(expect[f]).max()
        assert err <= 1e-13, (f, err)


def test_wrong_combinations_are_far_off():
    """The bar separates the textbook step from its plausible misreadings:
    the corrector's residual alone, the mean without the 1/2, and the
    predictor alone all miss it by far more than 1e-13."""
    nx, ny, gamma, p, u, v, beta = 33, 26, 1.4, 1.0, 0.3, -0.2, 1.0
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.5, 1.5, size=(ny, nx))
    U = workloads.prim_to_cons(gamma, rho, u, v, p)
    P = oracle.Params(nx, ny, 1.0 / nx, 1.0 / nx, gamma, 0.5, beta, 0, 0)
    rc, dt = oracle.dt(P, U)
    got = oracle.step(P, U, dt)[0]
    k1 = _advection_rate(rho, u, v, P.dx, P.dy, beta, 0, 0)
    k2 = _advection_rate(rho + dt * k1, u, v, P.dx, P.dy, beta, 0, 0)
    scale = np.abs(rho).max()
    assert np.abs(got - (rho + 0.5 * dt * (k1 + k2))).max() / scale <= 1e-13
    for wrong in (rho + dt * k2, rho + dt * (k1 + k2), rho + dt * k1):
        assert np.abs(got - wrong).max() / scale > 1e-4
