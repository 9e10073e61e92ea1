"""GPU: lf_step_halo, one step of a horizontal strip of a larger grid with
its ghost rows given (the unit of work of one GPU when the grid is split
into strips of rows).

Every strip of a grid that is periodic in y, stepped with the 4 rows
below and above it taken from the whole grid across the wrap, must give
lf_step of the whole grid bit for bit: the same kernel arithmetic on the
same data.  Strip heights include strips shorter than the ghost rows
(whose ghost rows then reach into the strips beyond the neighbours), both
x-boundaries, both precisions, mass fractions and the conservative
reconstruction; and the benchmark's Kelvin-Helmholtz 16384^2 split into
the 8 strips of 2048 rows that 8 GPUs would own.
"""
import pytest

import workloads
from gpu_util import solver_for, to_dev

pytestmark = pytest.mark.gpu

G = 4  # ghost rows per end


def _strips_step(cfg, U, dt, heights, dtype):
    """Step U (device, whole grid) strip by strip; returns the assembled
    result."""
    import torch
    nf, ny, nx = U.shape
    out = torch.empty_like(U)
    y0 = 0
    for h in heights:
        S = solver_for(dict(cfg, ny=h), dtype)
        rows = torch.arange(y0, y0 + h, device=U.device)
        lo = torch.arange(y0 - G, y0, device=U.device) % ny
        hi = torch.arange(y0 + h, y0 + h + G, device=U.device) % ny
        Un = U.index_select(1, rows).contiguous()
        glo = U.index_select(1, lo).contiguous()
        ghi = U.index_select(1, hi).contiguous()
        o = S.empty_state()
        S.step_halo(Un, glo, ghi, o, dt)
        out[:, y0:y0 + h] = o
        y0 += h
    assert y0 == ny
    return out


def _cfg(nx, ny, bcx, **kw):
    d = 1.0 / max(nx, ny)
    return dict(nx=nx, ny=ny, dx=d, dy=d * 1.25, gamma=1.4, cfl=0.5, beta=1.5, bc_x=bcx, bc_y=0, **kw)


@pytest.mark.parametrize("heights", [[96], [48, 48], [17] * 5 + [11], [3] * 32, [1] * 96, [5, 60, 2, 29]])
@pytest.mark.parametrize("bcx", [0, 1])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_strips_equal_whole_grid(heights, bcx, dtype):
    import torch
    nx, ny = 130, 96
    cfg = _cfg(nx, ny, bcx)
    U = to_dev(workloads.random_state(nx, ny, seed=len(heights) * 7 + bcx), dtype)
    S = solver_for(cfg, dtype)
    dt = S.dt(U)
    ref = S.empty_state()
    S.step(U, ref, dt)
    assert torch.equal(_strips_step(cfg, U, dt, heights, dtype), ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ns", [1, 2, 4])
def test_strips_equal_whole_grid_fractions(ns, dtype):
    import torch
    nx, ny = 121, 40
    cfg = _cfg(nx, ny, 1, ns=ns)
    U = to_dev(workloads.random_state_fractions(nx, ny, ns, seed=ns), dtype)
    S = solver_for(cfg, dtype)
    dt = S.dt(U)
    ref = S.empty_state()
    S.step(U, ref, dt)
    assert torch.equal(_strips_step(cfg, U, dt, [13, 2, 25], dtype), ref)


def test_strips_equal_whole_grid_conservative_reconstruction():
    import torch
    nx, ny = 77, 50
    cfg = _cfg(nx, ny, 0, recon=1)
    U = to_dev(workloads.random_state(nx, ny, seed=31))
    S = solver_for(cfg)
    dt = S.dt(U)
    ref = S.empty_state()
    S.step(U, ref, dt)
    assert torch.equal(_strips_step(cfg, U, dt, [20, 30], "f64"), ref)


def test_strips_16384_eight_shards():
    import torch
    n = 16384
    U, cfg = workloads.kelvin_helmholtz_torch(n)
    S = solver_for(cfg)
    dt = S.dt(U)
    ref = S.empty_state()
    S.step(U, ref, dt)
    del S
    out = _strips_step(cfg, U, dt, [n // 8] * 8, "f64")
    assert torch.equal(out, ref)


def test_step_halo_argument_checks():
    import paper_1607_08710_amd as L
    import torch
    cfg = _cfg(64, 16, 0)
    S = solver_for(cfg)
    U = to_dev(workloads.random_state(64, 16, seed=2))
    g = U[:, :G].contiguous()  # physical ghost rows (any will do for these checks)
    out = S.empty_state()
    with pytest.raises(ValueError):
        S.step_halo(U, g[:, :3], g, out, 1e-3)           # ghost rows of the wrong shape
    with pytest.raises(L.LFError):
        S.step_halo(U, g, g, out, -1.0)                  # negative dt
    with pytest.raises(L.LFError):
        S.step_halo(U, g, g, U, 1e-3)                    # output is the input
    S.step_halo(U, g, g, out, 0.0)                       # ghost rows may alias each other
    assert torch.equal(out, U)                           # dt = 0 leaves the state
