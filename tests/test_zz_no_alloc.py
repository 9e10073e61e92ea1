"""lf_adjoint_step_noalloc, the adjoint step for callers that cannot
allocate (its U* and mu live in the library's fixed device scratch),
against lf_adjoint_step with a caller workspace: bit for bit, on calls in a
row on one GPU, each followed by one on a smaller grid (the scratch then
still holds the larger grid's data), in both precisions; the first case of
each precision is the largest grid the scratch admits.  Calls after the
first on the device allocate no device memory.  And it runs inside a
captured HIP graph (the callers it is for): replays with eager work and
synchronisations between them, and the inputs changed in place, each
equal to lf_adjoint_step run eagerly on the same inputs."""
import numpy as np
import pytest

import workloads
from gpu_util import solver_for

pytestmark = pytest.mark.gpu


def _cfg(nx, ny, bc_x, bc_y):
    return dict(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, gamma=1.4, cfl=0.5, beta=1.5, bc_x=bc_x, bc_y=bc_y)


def _one(nx, ny, bc, dtype, seed):
    import torch
    S = solver_for(_cfg(nx, ny, *bc), dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    U = torch.from_numpy(workloads.random_state(nx, ny, seed=seed)).to(device="cuda", dtype=tdt)
    lam = torch.from_numpy(np.random.default_rng(seed + 1).standard_normal((4, ny, nx))).to(device="cuda",
                                                                                              dtype=tdt)
    lam0 = lam.clone()
    dt = S.dt(U)
    ref = S.empty_state()
    S.adjoint_step(U, dt, lam, ref)
    got = torch.full_like(ref, float("nan"))
    S.adjoint_step_noalloc(U, dt, lam, got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref), (nx, ny, bc, dtype)
    assert torch.equal(lam, lam0)
    assert bool(torch.isfinite(got).all())
    # the scratch is resolved now: further calls allocate nothing
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(2):
        S.adjoint_step_noalloc(U, dt, lam, got)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert torch.equal(got, ref)
    print(f"lf_adjoint_step_noalloc {dtype} {nx}x{ny} bc {bc}: equal to lf_adjoint_step", flush=True)


@pytest.mark.parametrize("dtype,big,small", [
    ("f64", (1024, 1024, (0, 0)), (301, 77, (1, 0))),
    ("f32", (2048, 1024, (0, 1)), (129, 65, (1, 1))),
])
def test_noalloc_equals_workspace_entry(dtype, big, small):
    _one(big[0], big[1], big[2], dtype, seed=7)
    _one(small[0], small[1], small[2], dtype, seed=8)


def test_noalloc_refuses_oversize_grid():
    import paper_1607_08710_amd as L
    import torch
    S = solver_for(_cfg(1025, 1024, 0, 0), "f64")
    U = S.empty_state()
    lam, out = torch.zeros_like(U), torch.empty_like(U)
    with pytest.raises(L.LFError) as e:
        S.adjoint_step_noalloc(U, 1e-3, lam, out)
    assert e.value.status == L.LF_ERR_TOO_LARGE


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_adjoint_step_in_a_graph(dtype):
    import torch
    nx, ny = 257, 190
    cfg = dict(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / nx, gamma=1.4, cfl=0.5, beta=1.5, bc_x=0, bc_y=1)
    S = solver_for(cfg, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    U = torch.from_numpy(workloads.random_state(nx, ny, seed=41)).to(device="cuda", dtype=tdt)
    lam = torch.from_numpy(np.random.default_rng(42).standard_normal((4, ny, nx))).to(device="cuda", dtype=tdt)
    dt = S.dt(U)
    out = S.empty_state()
    S.adjoint_step_noalloc(U, dt, lam, out)  # first call on the device: outside capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        S.adjoint_step_noalloc(U, dt, lam, out)
    ref = S.empty_state()
    for rep in range(4):
        if rep:
            # change the inputs in place (the graph reads them where they are)
            U.mul_(1.0 + 1e-3 * rep)
            lam.copy_(torch.roll(lam, shifts=rep, dims=2))
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda", dtype=tdt).sum()  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        S.adjoint_step(U, dt, lam, ref)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        assert bool(torch.isfinite(junk))
