"""The oracle against the hand-worked Sod first stage (tests/golden/
sod_first_stage.txt): eqs. (13)-(14), the flux of eq. (12), the CFL time
step and the predictor of the Heun list (Sec. 5), and the exact-Riemann
star states of Toro's five tests (tests/golden/toro_star_states.txt)."""
import numpy as np
import pytest

import workloads
from conftest import params_from, read_golden


def _golden():
    return {k: float(v) for k, v in read_golden("sod_first_stage.txt")}


def test_sod_first_stage_face(oracle_lib):
    G = _golden()
    g = 1.4
    us, ps = oracle_lib.acoustic_solve(g, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    assert us == pytest.approx(G["face_u_star"], rel=2e-16)
    assert ps == pytest.approx(G["face_p_star"], rel=2e-16)
    phi = oracle_lib.face_flux(g, [1.0, 0.0, 0.0, 1.0], [0.125, 0.0, 0.0, 0.1])
    np.testing.assert_allclose(
        phi, [G["face_F_mass"], G["face_F_momx"], G["face_F_momy"], G["face_F_energy"]],
        rtol=4e-16, atol=0)


def test_sod_first_stage_grid(oracle_lib):
    G = _golden()
    U, cfg = workloads.sod()
    P = params_from(cfg)
    rc, dt = oracle_lib.dt(P, U)
    assert rc == 0 and dt == pytest.approx(G["dt0"], rel=2e-16)
    R = oracle_lib.residual(P, U)
    Us = U - dt * R  # Heun list, item 6
    for j in range(cfg["ny"]):
        np.testing.assert_allclose(Us[:, j, 199], [G["c199_rho"], G["c199_mx"], G["c199_my"], G["c199_E"]],
                                   rtol=1e-15, atol=1e-17)
        np.testing.assert_allclose(Us[:, j, 200], [G["c200_rho"], G["c200_mx"], G["c200_my"], G["c200_E"]],
                                   rtol=1e-15, atol=1e-17)
    others = np.ones(cfg["nx"], bool)
    others[[199, 200]] = False
    assert np.array_equal(Us[:, :, others], U[:, :, others])


def test_toro_star_states(oracle_lib):
    for row in read_golden("toro_star_states.txt"):
        v = list(map(float, row[1:]))
        L, R = v[0:3], v[3:6]
        _, _, _, ps, us = oracle_lib.exact_riemann(1.4, L, R, np.array([0.0]))
        rl = oracle_lib.exact_riemann(1.4, L, R, np.array([us - 1e-9]))[0][0]
        rr = oracle_lib.exact_riemann(1.4, L, R, np.array([us + 1e-9]))[0][0]
        # printed to 5-6 significant digits
        assert ps == pytest.approx(v[6], rel=1e-5, abs=5e-6), row[0]
        assert us == pytest.approx(v[7], rel=1e-5, abs=5e-6), row[0]
        assert rl == pytest.approx(v[8], rel=1e-5, abs=5e-6), row[0]
        assert rr == pytest.approx(v[9], rel=1e-5, abs=5e-6), row[0]
