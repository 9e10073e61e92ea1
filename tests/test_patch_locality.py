"""CPU check of the patch evaluation behind the full-size multi-step GPU
parity tests (gpu_util.oracle_steps_at): k oracle Heun steps of the patch
of radius 4k around a cell give that cell's value after k steps of the
whole grid, bit for bit (the oracle's arithmetic per cell does not depend
on the grid around the stencil), for periodic and transmissive axes and
cells at the grid edges."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import oracle_params, oracle_steps_at


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_patches_reproduce_full_grid_steps(bc):
    nx, ny, k = 41, 37, 3
    cfg = dict(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / nx, gamma=1.4, cfl=0.5, beta=1.5, bc_x=bc[0], bc_y=bc[1])
    U = workloads.random_state(nx, ny, seed=77 + bc[0] + 2 * bc[1], rough=False)
    P = oracle_params(cfg)
    rc, dt = oracle.dt(P, U)
    dts = [dt, 0.9 * dt, 0.8 * dt]
    full = U
    for d in dts:
        full = oracle.step(P, full, d)
    cells = [(0, 0), (nx - 1, ny - 1), (1, ny - 2), (nx // 2, ny // 2), (nx - 3, 2), (13, 29)]
    got = oracle_steps_at(U, cfg, dts, cells)
    ref = np.array([full[:, j, i] for i, j in cells])
    assert np.array_equal(got, ref)
    # a patch one cell too small no longer does
    from gpu_util import sample_patch
    i, j = nx // 2, ny // 2
    patch, ic, jc = sample_patch(U, cfg, i, j, 4 * k - 1)
    Pp = oracle.Params(patch.shape[2], patch.shape[1], cfg["dx"], cfg["dy"], 1.4, 0.5, 1.5,
                       oracle.TRANSMISSIVE, oracle.TRANSMISSIVE)
    for d in dts:
        patch = oracle.step(Pp, patch, d)
    assert not np.array_equal(patch[:, jc, ic], full[:, j, i])
