"""Accuracy pins of the oracle against exact solutions.

  * Sod shock tube (the paper's first experiment, Sec. 5.2) at 400 cells,
    t = 0.2, CFL 0.5, against the exact Riemann solution, with the exact
    solver itself checked for the Rankine-Hugoniot and isentropic relations;
  * isentropic vortex convergence: the scheme is second order in space and
    time (Sec. 5), so the observed L1 order on smooth data approaches 2.
"""
import math

import numpy as np
import pytest

import workloads
from conftest import params_from


def test_exact_riemann_jump_relations(oracle_lib):
    """Sod: the right-moving shock satisfies Rankine-Hugoniot mass and
    momentum balance, the left rarefaction is isentropic (p/rho^gamma
    constant) with the Riemann invariant u + 2c/(gamma-1) constant."""
    g = 1.4
    L, R = workloads.SOD_LEFT, workloads.SOD_RIGHT
    xi = np.linspace(-2.0, 2.0, 40001)
    rho, u, p, ps, us = oracle_lib.exact_riemann(g, L, R, xi)
    # shock: where rho jumps from the star value to rho_R
    k = np.nonzero(np.abs(np.diff(rho)) > 0.05)[0]
    ks = k[-1]  # right-most jump = shock
    s = 0.5 * (xi[ks] + xi[ks + 1])
    r1, u1, p1 = rho[ks], u[ks], p[ks]
    r0, u0, p0 = R
    assert r1 * (u1 - s) == pytest.approx(r0 * (u0 - s), rel=2e-4)
    assert r1 * (u1 - s) ** 2 + p1 == pytest.approx(r0 * (u0 - s) ** 2 + p0, rel=2e-4)
    # fan: from the head u_L - c_L to the tail u* - c*_L, c*_L = c_L (p*/p_L)^((g-1)/(2g))
    tail = us - math.sqrt(g) * (ps / L[2]) ** ((g - 1) / (2 * g))
    fan = (xi > -math.sqrt(g) + 1e-3) & (xi < tail - 1e-3)
    assert fan.sum() > 100
    np.testing.assert_allclose(p[fan] / rho[fan] ** g, L[2] / L[0] ** g, rtol=1e-12)
    c = np.sqrt(g * p[fan] / rho[fan])
    np.testing.assert_allclose(u[fan] + 2 * c / (g - 1), 2 * math.sqrt(g) / (g - 1), rtol=1e-12)
    # in the fan the characteristic u - c passes through the origin
    np.testing.assert_allclose(u[fan] - c, xi[fan], atol=1e-12)


def test_sod_against_exact(oracle_lib):
    U, cfg = workloads.sod()
    Uf, t, n, dts, rc = oracle_lib.advance(params_from(cfg), U, 0.0, cfg["t_end"])
    assert rc == 0
    x = workloads.cell_centres(cfg["nx"], 0.0, 1.0)
    rho, u, p, ps, us = oracle_lib.exact_riemann(1.4, workloads.SOD_LEFT, workloads.SOD_RIGHT,
                                                 (x - 0.5) / cfg["t_end"])
    w = np.array([oracle_lib.cons_to_prim(1.4, Uf[:, 0, i]) for i in range(cfg["nx"])])
    e_rho = np.mean(np.abs(w[:, 0] - rho))
    e_u = np.mean(np.abs(w[:, 1] - u))
    e_p = np.mean(np.abs(w[:, 3] - p))
    assert e_rho < 3e-3 and e_u < 6e-3 and e_p < 3e-3, (e_rho, e_u, e_p)
    assert np.all(w[:, 0] > 0) and np.all(w[:, 3] > 0)
    # plateau values between the rarefaction tail and the contact
    plateau = (x > 0.5 + 0.2 * (us - 0.3 * us)) & (x < 0.5 + 0.2 * us - 0.03)
    np.testing.assert_allclose(w[plateau, 3], ps, rtol=2e-3)
    np.testing.assert_allclose(w[plateau, 1], us, rtol=3e-3)


def test_sod_error_falls_with_resolution(oracle_lib):
    errs = []
    for n in (100, 400):
        U, cfg = workloads.sod(n=n)
        Uf, t, _, _, rc = oracle_lib.advance(params_from(cfg), U, 0.0, cfg["t_end"])
        x = workloads.cell_centres(n, 0.0, 1.0)
        rho = oracle_lib.exact_riemann(1.4, workloads.SOD_LEFT, workloads.SOD_RIGHT, (x - 0.5) / 0.2)[0]
        errs.append(np.mean(np.abs(Uf[0, 0] - rho)))
    assert errs[1] < 0.45 * errs[0], errs


def _vortex_l1(oracle_lib, n):
    U, cfg = workloads.vortex(n)
    Uf, t, steps, dts, rc = oracle_lib.advance(params_from(cfg), U, 0.0, cfg["t_end"])
    assert rc == 0 and t == cfg["t_end"]
    Ue, _ = workloads.vortex(n, t=cfg["t_end"])
    return np.array([np.mean(np.abs(Uf[f] - Ue[f])) for f in range(4)])


@pytest.mark.slow
def test_vortex_second_order(oracle_lib):
    """Observed L1 orders of the four fields on 64 -> 128 -> 256 -> 512
    (measured: density 1.45, 1.60, 1.84; the other fields 1.59-1.87).  The
    order rises towards 2 with resolution: the Sweby limiter clips the
    smooth extrema of the vortex core to first order, on a region whose
    share of the L1 error falls as the grid refines.  So the bars are 1.8
    on the finest pair and 1.55 on 128 -> 256, and the order must grow
    from pair to pair."""
    e64 = _vortex_l1(oracle_lib, 64)
    e128 = _vortex_l1(oracle_lib, 128)
    e256 = _vortex_l1(oracle_lib, 256)
    e512 = _vortex_l1(oracle_lib, 512)
    o0 = np.log2(e64 / e128)
    o1 = np.log2(e128 / e256)
    o2 = np.log2(e256 / e512)
    assert np.all(o1 >= 1.55), o1
    assert np.all(o2 >= 1.8), o2
    assert np.all(o0 < o1) and np.all(o1 < o2), (o0, o1, o2)
    assert e512[0] < 4e-5


def test_vortex_conservation(oracle_lib):
    U, cfg = workloads.vortex(64)
    P = params_from(cfg)
    Uf, t, steps, dts, rc = oracle_lib.advance(P, U, 0.0, 2.0)
    t0, t1 = oracle_lib.totals(P, U), oracle_lib.totals(P, Uf)
    assert np.all(np.abs(t1 - t0) <= 1e-13 * np.abs(t0)), (t1 - t0) / t0
