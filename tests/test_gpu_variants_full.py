"""GPU: the scheme's variants at 16384^2, in the launch configuration the
benchmark's variant runs time (Kelvin-Helmholtz, periodic, FP64, one
single-pass step): one and two mass fractions (the band marker, then a
smooth x profile), and the conservative-variable reconstruction.  Each is
checked against the oracle cell by cell at sampled cells, including the
grid corners and cells across the shear layers.

A cell of the new state depends on the old state within 4 cells, so the
oracle's step on a 9 x 9 patch gathered around the cell with the periodic
wrap (transmissive patch edges) gives the full-grid value at its centre.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import solver_for

pytestmark = pytest.mark.gpu

N = 16384
R = 4


def _cells():
    rng = np.random.default_rng(16385)
    cells = [(int(i), int(j)) for i, j in rng.integers(0, N, size=(60, 2))]
    cells += [(0, 0), (N - 1, N - 1), (0, N - 1), (N - 1, 0)]
    cells += [(4321, N // 4 + k) for k in range(-3, 3)] + [(55, 3 * N // 4 + k) for k in range(-3, 3)]
    return cells


def _check(U, out, cfg, dt):
    import torch
    P = oracle.Params(2 * R + 1, 2 * R + 1, cfg["dx"], cfg["dy"], cfg["gamma"], cfg["cfl"], cfg["beta"],
                      oracle.TRANSMISSIVE, oracle.TRANSMISSIVE, ns=cfg.get("ns", 0), recon=cfg.get("recon", 0))
    scale = U.abs().amax(dim=(1, 2)).cpu().numpy()
    for i, j in _cells():
        xs = torch.arange(i - R, i + R + 1, device=U.device) % N
        ys = torch.arange(j - R, j + R + 1, device=U.device) % N
        patch = np.ascontiguousarray(U.index_select(1, ys).index_select(2, xs).cpu().numpy())
        ref = oracle.step(P, patch, dt)[:, R, R]
        got = out[:, j, i].cpu().numpy()
        err = np.abs(got - ref) / scale
        assert np.all(err <= 1e-12), (i, j, err)


@pytest.mark.parametrize("fractions", [1, 2])
def test_sampled_step_fractions_16384(fractions):
    import torch
    U, cfg = workloads.kelvin_helmholtz_torch(N, fractions=fractions)
    S = solver_for(cfg)
    dt = S.dt(U)
    out = S.empty_state()
    S.step(U, out, dt)
    torch.cuda.synchronize()
    _check(U, out, cfg, dt)
    del U, out, S
    torch.cuda.empty_cache()


def test_sampled_step_conservative_reconstruction_16384():
    import torch
    U, cfg = workloads.kelvin_helmholtz_torch(N)
    cfg = dict(cfg, recon=1)
    S = solver_for(cfg)
    dt = S.dt(U)
    out = S.empty_state()
    S.step(U, out, dt)
    torch.cuda.synchronize()
    _check(U, out, cfg, dt)
    del U, out, S
    torch.cuda.empty_cache()
