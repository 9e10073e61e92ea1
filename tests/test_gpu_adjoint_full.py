"""GPU: lf_adjoint_step at 4096^2, the size and launch configuration the
adjoint benchmark times (Kelvin-Helmholtz, periodic, FP64, a seeded
cotangent), checked cell by cell against the oracle's adjoint step at
sampled cells; and lf_adjoint_step_ustar on the U* of lf_step_save, bit for
bit against it on the whole grid.

The state is the Kelvin-Helmholtz one with every conservative value scaled
by 1 + 1e-4 r (r uniform in [-1, 1], seeded).  On the exactly uniform
bands of the plain state the limiter sits on its kinks (zero differences,
or rounding noise of the recovered pressure), where the derivative
convention decides: there a one-ulp change of the input moves the
oracle's own lambda^n by up to 17%, so no two implementations that round
differently can agree pointwise.  The perturbation moves every difference
far from the kinks (one-ulp sensitivity ~5e-16).

lambda^n at a cell depends on U^n within at most 8 cells (U* reaches 2
cells, each transposed residual Jacobian at most 4 more in U and 2 in its
cotangent) and on lambda^{n+1} within 4.  The oracle's adjoint step on a
21 x 21 patch gathered around the cell with the periodic wrap therefore
reproduces the full-grid value at the patch centre: whatever boundary
condition the patch gets, its edge is 10 cells away, beyond that reach
(the oracle's own tests check this locality on a small periodic grid).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import solver_for

pytestmark = pytest.mark.gpu

N = 4096
R = 10  # patch radius


def _patch(T, i, j):
    import torch
    xs = torch.arange(i - R, i + R + 1, device=T.device) % N
    ys = torch.arange(j - R, j + R + 1, device=T.device) % N
    return np.ascontiguousarray(T.index_select(1, ys).index_select(2, xs).cpu().numpy())


def test_adjoint_step_4096_sampled_f64():
    import torch
    Uh, cfg = workloads.kelvin_helmholtz(N)
    Uh *= 1.0 + 1e-4 * np.random.default_rng(7).uniform(-1.0, 1.0, Uh.shape)
    U = torch.from_numpy(Uh).cuda()
    del Uh
    S = solver_for(cfg)
    dt = S.dt(U)
    lam = torch.from_numpy(np.random.default_rng(4096).standard_normal((4, N, N))).cuda()
    out = S.empty_state()
    S.adjoint_step(U, dt, lam, out)
    torch.cuda.synchronize()
    Pp = oracle.Params(2 * R + 1, 2 * R + 1, cfg["dx"], cfg["dy"], cfg["gamma"], cfg["cfl"], cfg["beta"],
                       oracle.TRANSMISSIVE, oracle.TRANSMISSIVE)
    rng = np.random.default_rng(40960)
    cells = [(int(i), int(j)) for i, j in rng.integers(0, N, size=(40, 2))]
    cells += [(0, 0), (N - 1, N - 1), (0, N - 1), (N - 1, 0), (N // 2, N - 2)]
    # across the two shear layers (y = 1/4 and 3/4), where the limiter is active
    cells += [(777, N // 4 + k) for k in range(-3, 3)] + [(3001, 3 * N // 4 + k) for k in range(-3, 3)]
    scale = out.abs().amax(dim=(1, 2)).cpu().numpy()
    for i, j in cells:
        ref = oracle.adjoint_step(Pp, _patch(U, i, j), dt, _patch(lam, i, j))[:, R, R]
        got = out[:, j, i].cpu().numpy()
        err = np.abs(got - ref) / scale
        assert np.all(err <= 1e-11), (i, j, err)
    # the rollout's path: U* kept by lf_step_save, then the adjoint step on it
    Un1, Us, out2 = S.empty_state(), S.empty_state(), S.empty_state()
    S.step_save(U, Un1, Us, dt)
    S.adjoint_step_ustar(U, Us, dt, lam, out2)
    assert torch.equal(out, out2)
