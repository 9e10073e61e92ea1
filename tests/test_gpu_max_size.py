"""GPU: the largest grid the library accepts (FP32), and FP64 beyond 4 GB
per field plane.

nx * ny must stay below 2^31 (cell offsets are 32-bit inside a plane).
At 46340 x 46340 = 2 147 395 600 cells, the last cell offset is within
90 000 of that limit.  An FP32 state is 34 GB, and the state, the output
and the workspace (two more states) take ~137 GB of the 288 GB HBM.  One
step (the single-pass kernel) and the CFL reduction run at that size; the
new state is checked against the oracle cell by cell at sampled
positions, including the last rows and columns, with patches gathered on
the device.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import solver_for

pytestmark = pytest.mark.gpu

N = 46340


def _patch(U, i, j, r=4):
    """Transmissive (clipped) neighbourhood of cell (i, j), gathered on the
    device; returns (host float64 patch, ic, jc)."""
    import torch
    xs = torch.arange(max(0, i - r), min(N, i + r + 1), device=U.device)
    ys = torch.arange(max(0, j - r), min(N, j + r + 1), device=U.device)
    p = U.index_select(1, ys).index_select(2, xs).to(torch.float64).cpu().numpy()
    return np.ascontiguousarray(p), i - int(xs[0]), j - int(ys[0])


def test_max_size_step_f32():
    import torch
    assert N * N < 2**31 and (N + 1) * (N + 1) >= 2**31
    cfg = dict(nx=N, ny=N, dx=1.0 / N, dy=1.0 / N, gamma=1.4, cfl=0.5, beta=1.5, bc_x=1, bc_y=1)
    # a smooth seeded state (transmissive box): rho and p vary on the scale
    # of the box, velocities on a tenth of it
    x = (torch.arange(N, dtype=torch.float32, device="cuda") + 0.5) / N
    U = torch.empty((4, N, N), dtype=torch.float32, device="cuda")
    U[0] = 1.0 + 0.3 * torch.sin(2 * math.pi * x)[None, :] * torch.cos(2 * math.pi * x)[:, None]
    U[1] = U[0] * (0.4 * torch.sin(20 * math.pi * x))[:, None]
    U[2] = U[0] * (0.4 * torch.cos(20 * math.pi * x))[None, :]
    U[3] = 2.5 + 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]
    S = solver_for(cfg, "f32")
    dt = S.dt(U)
    assert dt > 0
    out = S.empty_state()
    S.step(U, out, dt)
    torch.cuda.synchronize()
    rng = np.random.default_rng(46340)
    cells = [(int(i), int(j)) for i, j in rng.integers(0, N, size=(40, 2))]
    cells += [(N - 1, N - 1), (0, N - 1), (N - 1, 0), (N - 3, N - 2), (N // 2, N - 1), (57, N - 1)]
    # each field's error is measured against its largest magnitude over the
    # grid (as in the other sampled tests): the float error of a momentum
    # is set by the pressure in its flux, not by the local momentum, which
    # crosses zero
    scale = U.abs().amax(dim=(1, 2)).to(torch.float64).cpu().numpy()
    for i, j in cells:
        patch, ic, jc = _patch(U, i, j)
        P = oracle.Params(patch.shape[2], patch.shape[1], cfg["dx"], cfg["dy"], 1.4, 0.5, 1.5,
                          oracle.TRANSMISSIVE, oracle.TRANSMISSIVE)
        ref = oracle.step(P, patch, dt)[:, jc, ic]
        got = out[:, j, i].to(torch.float64).cpu().numpy()
        err = np.abs(got - ref) / scale
        # float state and float flux arithmetic: a few float ulps per step
        assert np.all(err <= 2e-6), (i, j, err)
    del U, out, S
    torch.cuda.empty_cache()


def test_large_step_f64():
    """FP64 at 32768^2: each field plane is 8.6 GB, so plane offsets exceed
    32 bits in bytes (the state, the output and the workspace take ~137 GB).
    One single-pass step and the CFL reduction, checked against the oracle
    at sampled cells, including the last rows and columns (periodic: the
    patches wrap)."""
    import torch
    n = 32768
    cfg = dict(nx=n, ny=n, dx=1.0 / n, dy=1.0 / n, gamma=1.4, cfl=0.5, beta=1.5, bc_x=0, bc_y=0)
    x = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) / n
    U = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    U[0] = 1.0 + 0.3 * torch.sin(2 * math.pi * x)[None, :] * torch.cos(2 * math.pi * x)[:, None]
    U[1] = U[0] * (0.4 * torch.sin(20 * math.pi * x))[:, None]
    U[2] = U[0] * (0.4 * torch.cos(20 * math.pi * x))[None, :]
    U[3] = 2.5 + 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]
    S = solver_for(cfg)
    dt = S.dt(U)
    out = S.empty_state()
    S.step(U, out, dt)
    torch.cuda.synchronize()
    rng = np.random.default_rng(32768)
    cells = [(int(i), int(j)) for i, j in rng.integers(0, n, size=(30, 2))]
    cells += [(n - 1, n - 1), (0, n - 1), (n - 1, 0), (n - 3, n - 2), (n // 2, n - 1)]
    scale = U.abs().amax(dim=(1, 2)).cpu().numpy()
    r = 4
    P = oracle.Params(2 * r + 1, 2 * r + 1, cfg["dx"], cfg["dy"], 1.4, 0.5, 1.5, oracle.TRANSMISSIVE,
                      oracle.TRANSMISSIVE)
    for i, j in cells:
        xs = torch.arange(i - r, i + r + 1, device="cuda") % n
        ys = torch.arange(j - r, j + r + 1, device="cuda") % n
        patch = np.ascontiguousarray(U.index_select(1, ys).index_select(2, xs).cpu().numpy())
        ref = oracle.step(P, patch, dt)[:, r, r]
        got = out[:, j, i].cpu().numpy()
        err = np.abs(got - ref) / scale
        assert np.all(err <= 1e-12), (i, j, err)
    del U, out, S
    torch.cuda.empty_cache()
