"""Pins of the oracle's pointwise pieces against closed forms.

Each test checks a property the paper's formulas or the mathematics fix,
chosen so that a dropped term, a wrong sign or a swapped operand in the
oracle fails at least one of them:
  * eq. (sweby): hand-tabulated values, symmetry, oddness, the minmod (beta=1)
    and superbee (beta=2) special cases, phi(a,a) = a;
  * eqs. (13)-(14): they solve the two acoustic jump relations with the
    impedances rho_L a and rho_R a; contact and linear-acoustic special cases;
  * eq. (12): physical Euler flux for a uniform state, tangential Galilean
    invariance, mirror symmetry, upwind side;
  * Sec. 3: EOS round trip against the input builder.
"""
import math

import numpy as np
import pytest

import workloads

pytestmark = []


# ---- eq. (sweby) ----------------------------------------------------------

@pytest.mark.parametrize("a,b,beta,expect", [
    (1.0, 3.0, 1.5, 1.5),    # max(min(1, 4.5), min(1.5, 3)) = 1.5
    (3.0, 1.0, 1.5, 1.5),    # max(min(3, 1.5), min(4.5, 1)) = 1.5
    (-2.0, -1.0, 2.0, -2.0), # -max(min(2, 2), min(4, 1))
    (2.0, 8.0, 1.0, 2.0),    # minmod
    (2.0, 8.0, 2.0, 4.0),    # superbee: max(min(2,16), min(4,8))
    (4.0, 1.0, 2.0, 2.0),    # superbee: max(min(4,2), min(8,1))
    (1.0, -1.0, 1.5, 0.0),   # opposite signs
    (0.0, 5.0, 1.5, 0.0),    # ab = 0
    (5.0, 0.0, 1.5, 0.0),
    (-3.0, -6.0, 1.5, -4.5), # -max(min(3, 9), min(4.5, 6))
])
def test_sweby_table(oracle_lib, a, b, beta, expect):
    assert oracle_lib.sweby(a, b, beta) == expect


def test_sweby_identities(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(2000):
        a, b = rng.normal(size=2) * 10 ** rng.uniform(-3, 3, size=2)
        beta = rng.uniform(1.0, 2.0)
        phi = oracle_lib.sweby(a, b, beta)
        assert phi == oracle_lib.sweby(b, a, beta)            # symmetric
        assert -phi == oracle_lib.sweby(-a, -b, beta)         # odd
        assert oracle_lib.sweby(a, a, beta) == a              # consistency, beta >= 1
        if a * b <= 0:
            assert phi == 0.0
        else:
            mm = math.copysign(min(abs(a), abs(b)), a)
            sb = math.copysign(max(min(abs(a), 2 * abs(b)), min(2 * abs(a), abs(b))), a)
            assert oracle_lib.sweby(a, b, 1.0) == mm          # minmod
            assert oracle_lib.sweby(a, b, 2.0) == sb          # superbee
            # TVD region: between minmod and superbee, same sign as a
            assert abs(mm) <= abs(phi) <= abs(sb) and phi * a > 0


# ---- eqs. (13)-(14) -------------------------------------------------------

def _c(gamma, rho, p):
    return math.sqrt(gamma * p / rho)


def test_acoustic_jump_relations(oracle_lib):
    """(p*, u*) solve p* - p_L + rho_L a (u* - u_L) = 0 and
    p* - p_R - rho_R a (u* - u_R) = 0 with a = max(c_L, c_R)."""
    rng = np.random.default_rng(11)
    g = 1.4
    for _ in range(2000):
        rl, rr = rng.uniform(0.1, 5, 2)
        pl, pr = rng.uniform(0.05, 5, 2)
        ul, ur = rng.uniform(-3, 3, 2)
        us, ps = oracle_lib.acoustic_solve(g, rl, ul, pl, rr, ur, pr)
        a = max(_c(g, rl, pl), _c(g, rr, pr))
        scale = max(abs(pl), abs(pr), rl * a * abs(ul), rr * a * abs(ur), rl * a * abs(us), 1.0)
        assert abs(ps - pl + rl * a * (us - ul)) <= 1e-13 * scale
        assert abs(ps - pr - rr * a * (us - ur)) <= 1e-13 * scale


def test_acoustic_special_cases(oracle_lib):
    g = 1.4
    # contact: equal u and p -> u* = u, p* = p
    us, ps = oracle_lib.acoustic_solve(g, 1.0, 0.3, 2.0, 0.2, 0.3, 2.0)
    assert us == pytest.approx(0.3, rel=1e-15, abs=1e-16) and ps == pytest.approx(2.0, rel=1e-15)
    # equal densities: textbook linear acoustic solver with impedance Z = rho a
    rho, ul, ur, pl, pr = 0.8, 0.4, -0.1, 1.3, 0.7
    a = max(_c(g, rho, pl), _c(g, rho, pr))
    Z = rho * a
    us, ps = oracle_lib.acoustic_solve(g, rho, ul, pl, rho, ur, pr)
    assert ps == pytest.approx(0.5 * (pl + pr) - 0.5 * Z * (ur - ul), rel=1e-14)
    assert us == pytest.approx(0.5 * (ul + ur) - (pr - pl) / (2 * Z), rel=1e-14)
    # mirror: swapping sides and negating velocities negates u*, keeps p*
    us2, ps2 = oracle_lib.acoustic_solve(g, rho, -ur, pr, rho, -ul, pl)
    assert us2 == pytest.approx(-us, rel=1e-14) and ps2 == pytest.approx(ps, rel=1e-14)


# ---- eq. (12) -------------------------------------------------------------

def test_flux_uniform_state_is_euler_flux(oracle_lib):
    rng = np.random.default_rng(3)
    g = 1.4
    for _ in range(500):
        rho, p = rng.uniform(0.1, 3, 2)
        un, ut = rng.uniform(-2, 2, 2)
        w = np.array([rho, un, ut, p])
        E = p / (g - 1) + 0.5 * rho * (un * un + ut * ut)
        expect = np.array([rho * un, rho * un * un + p, rho * un * ut, (E + p) * un])
        phi = oracle_lib.face_flux(g, w, w)
        np.testing.assert_allclose(phi, expect, rtol=1e-14, atol=1e-14 * (abs(E) + p))


def test_flux_tangential_galilean_invariance(oracle_lib):
    """A common tangential velocity V leaves u*, p* unchanged; the
    tangential-momentum flux gains V * mass flux and the energy flux gains
    V * (old tangential flux) + V^2/2 * mass flux."""
    rng = np.random.default_rng(5)
    g = 1.4
    for _ in range(500):
        wl = np.array([rng.uniform(0.2, 3), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 3)])
        wr = np.array([rng.uniform(0.2, 3), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 3)])
        V = rng.uniform(-2, 2)
        f0 = oracle_lib.face_flux(g, wl, wr)
        f1 = oracle_lib.face_flux(g, wl + [0, 0, V, 0], wr + [0, 0, V, 0])
        sc = 1 + np.abs(f0).max()
        assert abs(f1[0] - f0[0]) <= 1e-14 * sc
        assert abs(f1[1] - f0[1]) <= 1e-14 * sc
        assert abs(f1[2] - (f0[2] + V * f0[0])) <= 1e-13 * sc
        assert abs(f1[3] - (f0[3] + V * f0[2] + 0.5 * V * V * f0[0])) <= 1e-13 * sc * (1 + V * V)


def test_flux_mirror_and_upwind_side(oracle_lib):
    g = 1.4
    rng = np.random.default_rng(9)
    for _ in range(500):
        wl = np.array([rng.uniform(0.2, 3), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 3)])
        wr = np.array([rng.uniform(0.2, 3), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 3)])
        f = oracle_lib.face_flux(g, wl, wr)
        # mirror x -> -x: swap sides, negate normal velocity
        m = np.array([1, -1, 1, 1])
        fm = oracle_lib.face_flux(g, wr * m, wl * m)
        np.testing.assert_allclose(fm, -f * np.array([1, -1, 1, 1]), rtol=1e-13, atol=1e-13)
        us, ps = oracle_lib.acoustic_solve(g, wl[0], wl[1], wl[3], wr[0], wr[1], wr[3])
        side = wl if us > 0 else wr
        assert f[0] == pytest.approx(side[0] * us, rel=1e-15, abs=1e-300)
        assert f[2] == pytest.approx(side[0] * side[2] * us, rel=1e-15, abs=1e-300)
        assert f[1] == pytest.approx(side[0] * side[1] * us + ps, rel=1e-14, abs=1e-14)


# ---- Sec. 3 EOS --------------------------------------------------------------

def test_cons_prim_round_trip(oracle_lib):
    rng = np.random.default_rng(1)
    for g in (1.4, 1.67, 3.0, 1.05):
        rho, u, v, p = rng.uniform(0.1, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.1, 3)
        U = workloads.prim_to_cons(g, rho, u, v, p)
        w = oracle_lib.cons_to_prim(g, U)
        np.testing.assert_allclose(w, [rho, u, v, p], rtol=1e-13)
