"""GPU parity for the paper's one-dimensional shock tubes and its limiter
variants, through the C ABI against the FP64 oracle.

Shock tubes (Sec. 5.2): Sod (100, 400 cells, T = 0.23), two-rarefaction
near vacuum (200, 2000 cells, T = 0.16), sonic rarefaction (400 cells,
T = 0.16) and the Mach-40 shock-shock tube (400 cells, minmod), each a
single row at CFL 0.25 with transmissive boundaries, whole runs through
lf_advance (up to 3518 steps).  Their bar follows the oracle's own
rounding floor: one-ulp noise added after every step moves its final
state by up to 1.4e-11 relative L-infinity and 2.0e-12 relative L1 (pinned
below 2.5e-11 / 2.5e-12 by the CPU conditioning tests), so FP64 parity is
held to 1e-10 and 1e-11.  Both paths are then checked against the exact
Riemann solution.

Limiter variants (eq. (sweby)): beta = 0 (first order, all slopes zero),
1 (minmod), 1.5, 2 (superbee) for one step in FP64 and FP32, the adjoint
step, and a short two-dimensional run.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import oracle_params, rel_l1, rel_linf, solver_for, to_dev, to_host

pytestmark = pytest.mark.gpu

TUBES = [(name, n) for name, spec in workloads.PAPER_TUBES.items() for n in spec[3]]


def _exact_err(U, cfg):
    """Relative L1 error of (rho, u, p) against the exact Riemann solution,
    each over the largest magnitude the exact field takes."""
    n, g = cfg["nx"], cfg["gamma"]
    x = workloads.cell_centres(n, 0.0, 1.0)
    er, eu, ep, _, _ = oracle.exact_riemann(g, cfg["left"], cfg["right"], (x - 0.5) / cfg["t_end"])
    rho = U[0, 0]
    u = U[1, 0] / rho
    p = (g - 1.0) * (U[3, 0] - 0.5 * rho * u * u - 0.5 * U[2, 0] ** 2 / rho)
    return np.array([np.mean(np.abs(a - e)) / np.max(np.abs(e)) for a, e in ((rho, er), (u, eu), (p, ep))])


@pytest.mark.parametrize("name,n", TUBES)
def test_paper_tube_f64(name, n):
    U, cfg = workloads.paper_tube(name, n)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, cfg["t_end"])
    assert rco == 0
    S = solver_for(cfg)
    d = to_dev(U)
    t, steps, dts = S.advance(d, 0.0, cfg["t_end"], dts_capacity=10000)
    assert steps == no and t == to == cfg["t_end"]
    np.testing.assert_allclose(dts, dto, rtol=1e-10)
    Ug = to_host(d)
    assert np.all(Ug[0] > 0) and np.all(Ug[2] == 0.0)
    err = rel_linf(Ug, Uo)
    assert np.all(err <= 1e-10), err
    e1 = rel_l1(Ug, Uo)
    assert np.all(e1 <= 1e-11), e1
    eg, eo = _exact_err(Ug, cfg), _exact_err(Uo, cfg)
    assert np.all(eg < 0.02), eg
    np.testing.assert_allclose(eg, eo, rtol=1e-6)


@pytest.mark.parametrize("name,n", [("sod", 400), ("two_rarefaction", 2000), ("shock_shock", 400)])
def test_paper_tube_f32(name, n):
    """FP32 state, FP64 accumulation of the update, against the FP64
    oracle started from the same float-rounded state."""
    U, cfg = workloads.paper_tube(name, n)
    U32 = U.astype(np.float32).astype(np.float64)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U32, 0.0, cfg["t_end"])
    S = solver_for(cfg, "f32")
    d = to_dev(U32, "f32")
    t, steps, dts = S.advance(d, 0.0, cfg["t_end"], dts_capacity=10000)
    assert t == cfg["t_end"] and abs(steps - no) <= 1
    Ug = to_host(d)
    assert np.all(Ug[0] > 0)
    e1 = rel_l1(Ug, Uo)
    assert np.all(e1 <= 2e-5), e1
    assert np.all(_exact_err(Ug, cfg) < 0.02)


def _cfg(nx, ny, bcx, bcy, beta):
    d = 1.0 / max(nx, ny)
    return dict(nx=nx, ny=ny, dx=d, dy=d, gamma=1.4, cfl=0.5, beta=beta, bc_x=bcx, bc_y=bcy)


BETAS = [0.0, 1.0, 1.5, 2.0]


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_limiter_variant_step_f64(beta, bc):
    cfg = _cfg(130, 70, *bc, beta)
    U = workloads.random_state(130, 70, seed=int(40 + 10 * beta + bc[0]))
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U)
    S = solver_for(cfg)
    out = S.empty_state()
    S.step(to_dev(U), out, dt)
    err = rel_linf(to_host(out), oracle.step(P, U, dt))
    assert np.all(err <= 1e-12), err


def test_first_order_has_no_slopes():
    """beta = 0 zeroes every slope, so the step equals the first-order
    Lagrange-flux step, whose face states are the cell values: on a state
    whose only variation is along x the residual is the one-dimensional
    first-order residual in every row."""
    rng = np.random.default_rng(7)
    nx, ny = 75, 3
    rho = np.tile(rng.uniform(0.5, 2.0, nx), (ny, 1))
    u = np.tile(rng.uniform(-0.5, 0.5, nx), (ny, 1))
    p = np.tile(rng.uniform(0.5, 2.0, nx), (ny, 1))
    U = workloads.prim_to_cons(1.4, rho, u, 0.0, p)
    cfg = _cfg(nx, ny, 0, 0, 0.0)
    S = solver_for(cfg)
    R = S.empty_state()
    S.residual(to_dev(U), R)
    Rg = to_host(R)
    # first-order fluxes from the pointwise oracle solver, face by face
    F = np.empty((4, nx + 1))
    for i in range(nx + 1):
        wl = oracle.cons_to_prim(1.4, U[:, 0, (i - 1) % nx])
        wr = oracle.cons_to_prim(1.4, U[:, 0, i % nx])
        F[:, i] = oracle.face_flux(1.4, wl, wr)
    ref = (F[:, 1:] - F[:, :-1]) / cfg["dx"]
    assert np.all(Rg[2] == 0.0)
    scale = np.abs(ref).max(axis=1)
    for j in range(ny):
        assert np.all(np.abs(Rg[[0, 1, 3], j] - ref[[0, 1, 3]]).max(axis=1) <= 1e-12 * scale[[0, 1, 3]])


@pytest.mark.parametrize("beta", BETAS)
def test_limiter_variant_step_f32(beta):
    cfg = _cfg(130, 70, 1, 0, beta)
    U = workloads.random_state(130, 70, seed=int(60 + 10 * beta))
    U32 = U.astype(np.float32).astype(np.float64)
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U32)
    S = solver_for(cfg, "f32")
    out = S.empty_state()
    S.step(to_dev(U32, "f32"), out, dt)
    err = rel_l1(to_host(out), oracle.step(P, U32, dt))
    assert np.all(err <= 2e-6), err


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_limiter_variant_adjoint_f64(beta, bc):
    cfg = _cfg(70, 45, *bc, beta)
    U = workloads.random_state(70, 45, seed=int(80 + 10 * beta + bc[0]))
    lam = np.random.default_rng(5).standard_normal(U.shape)
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U)
    S = solver_for(cfg)
    out = S.empty_state()
    S.adjoint_step(to_dev(U), dt, to_dev(lam), out)
    err = rel_linf(to_host(out), oracle.adjoint_step(P, U, dt, lam))
    assert np.all(err <= 1e-11), err


@pytest.mark.parametrize("beta", BETAS)
def test_limiter_variant_four_quadrant_f64(beta):
    """Four-quadrant problem at 128^2 for 100 steps with each limiter; the
    diagonal mirror symmetry stays bitwise."""
    U, cfg = workloads.four_quadrant(128)
    cfg = dict(cfg, beta=beta)
    P = oracle_params(cfg)
    Uo, to, no, dto, rco = oracle.advance(P, U, 0.0, 1.0, max_steps=100)
    S = solver_for(cfg)
    d = to_dev(U)
    t, steps, dts = S.advance(d, 0.0, 1.0, max_steps=100)
    assert steps == no == 100
    Ug = to_host(d)
    err = rel_linf(Ug, Uo)
    assert np.all(err <= 1e-11), err
    assert np.all(rel_l1(Ug, Uo) <= 3e-13)
    T = np.ascontiguousarray(np.transpose(Ug, (0, 2, 1)))
    T[[1, 2]] = T[[2, 1]]
    assert np.array_equal(T, Ug)


# ---- the adjoint at the limiter's ties --------------------------------------------

# Differences (in units of 1/64) that put the limiter on each of its ties
# for beta = 1, 1.5 and 2: |a| = |b|, beta |a| = |b|, |a| = beta |b|, a sign
# change and a zero difference.
TIE_STEPS = {1.0: [2, 2, 3, 2, 2, 3, 3, -2, 0, 2, 4, 2],
             1.5: [2, 2, 3, 2, 2, 3, 3, -2, 0, 2, 4, 2],
             2.0: [2, 2, 4, 2, 2, 4, 4, -2, 0, 2, 3, 2]}


def _tie_profile(n, beta, shift):
    d = np.array(TIE_STEPS[beta], dtype=np.float64) / 64.0
    return np.concatenate([[0.0], np.cumsum(np.resize(np.roll(d, shift), n - 1))])


@pytest.mark.parametrize("beta", [1.0, 1.5, 2.0])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
@pytest.mark.parametrize("moving", [False, True])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_residual_vjp_at_limiter_ties(beta, bc, moving, dtype):
    """J_R(U)^T g where every primitive difference sits on a tie of the
    limiter (exact dyadic values, gamma = 1.5): the one-sided derivatives
    the adjoint takes there follow the conventions of eq. (sweby)'s max-min
    form (min follows its first argument, max its first, zero when ab <=
    0), on both sides; a different choice would change the result by O(1).
    Moving: rho = 1, and u, v, p carry the ties.  At rest: rho carries them
    and p = rho, so that c_L = c_R at every face as well (the sound speed's
    tie, which follows the left side).  Both forms of the perfect-gas law
    (the oracle's, through the specific energy, and the kernels') recover
    the primitive variables bit for bit, or the ties would not survive.
    The values are exact in FP32 too, so the FP32 kernel meets the same
    ties; it is held to 1e-5 (its rounding), far below the O(1) change a
    different one-sided derivative would make."""
    nx, ny = 70, 45
    cx = lambda s: _tie_profile(nx, beta, s)[None, :]
    cy = lambda s: _tie_profile(ny, beta, s)[:, None]
    if moving:
        rho = np.ones((ny, nx))
        u = 0.25 + cx(1) - cy(5)
        v = -0.25 + cx(7) + cy(2)
        p = 1.0 + cx(3) + cy(9)
    else:
        rho = 1.0 + cx(0) + cy(4)
        u = np.zeros((ny, nx))
        v = np.zeros((ny, nx))
        p = rho.copy()
    U = workloads.prim_to_cons(1.5, rho, u, v, p)
    w = np.array([oracle.cons_to_prim(1.5, U[:, j, i]) for j in range(ny) for i in range(nx)])
    assert np.array_equal(w, np.stack([rho, u, v, p], axis=-1).reshape(-1, 4))
    assert np.array_equal(0.5 * (U[3] - 0.5 * (U[1] * u + U[2] * v)), p)  # the kernels' form
    cfg = dict(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / nx, gamma=1.5, cfl=0.5, beta=beta, bc_x=bc[0], bc_y=bc[1])
    g = np.random.default_rng(int(10 * beta) + bc[0]).standard_normal(U.shape)
    S = solver_for(cfg, dtype)
    out = S.empty_state()
    S.residual_vjp(to_dev(U, dtype), to_dev(g, dtype), out)
    if dtype == "f32":
        g = g.astype(np.float32).astype(np.float64)  # the cotangent the kernel saw
    ref = oracle.residual_vjp(oracle_params(cfg), U, g)
    err = rel_linf(to_host(out), ref)
    assert np.all(err <= (1e-11 if dtype == "f64" else 1e-5)), err
