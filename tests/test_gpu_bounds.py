"""Every output of the library is written exactly over its own extent.

Outputs are views into a larger device buffer whose guard bands before and
after hold a sentinel bit pattern; after the call the guard bands must hold
it unchanged, and no element of the output may still hold it.  This covers
the stores the kernels drop by design (halo lanes, rows of a strip's
overlap, stores into an empty range), the ragged tails of tiles and
strips, both boundary kinds and both precisions.  Values are checked
elsewhere (the parity tests); here only where the writes land.
"""
import numpy as np
import pytest

import workloads
from gpu_util import solver_for, to_dev

pytestmark = pytest.mark.gpu

GUARD = 3000  # elements on each side: more than a row of any grid below
SENT = {8: 0x7FF4DEADBEEF1234, 4: 0x7FA5A5A5}  # NaN bit patterns, as integers


def _cfg(nx, ny, bcx, bcy, ns=0, recon=0):
    d = 1.0 / max(nx, ny)
    return dict(nx=nx, ny=ny, dx=d, dy=d, gamma=1.4, cfl=0.5, beta=1.5, bc_x=bcx, bc_y=bcy, ns=ns,
                recon=recon)


def _ints(t):
    import torch
    return t.view(torch.int64 if t.element_size() == 8 else torch.int32)


class Guarded:
    """A state-shaped output inside a sentinel-filled buffer."""

    def __init__(self, S):
        import torch
        self.n = int(np.prod(S.shape))
        self.flat = torch.empty(self.n + 2 * GUARD, dtype=S.torch_dtype, device=S.device)
        self.sent = SENT[self.flat.element_size()]
        _ints(self.flat).fill_(self.sent)
        self.out = self.flat[GUARD:GUARD + self.n].view(S.shape)

    def check(self, what):
        import torch
        torch.cuda.synchronize()
        bits = _ints(self.flat)
        assert bool((bits[:GUARD] == self.sent).all()), f"{what}: write before the output"
        assert bool((bits[GUARD + self.n:] == self.sent).all()), f"{what}: write past the output"
        missed = int((bits[GUARD:GUARD + self.n] == self.sent).sum())
        assert missed == 0, f"{what}: {missed} output elements not written"


SHAPES = [(61, 37), (300, 261), (1, 9), (9, 1), (5, 3), (130, 70)]
BCS = [(0, 0), (1, 1), (0, 1), (1, 0)]


def _inputs(S, cfg, seed):
    ns = cfg.get("ns", 0)
    U = workloads.random_state_fractions(cfg["nx"], cfg["ny"], ns, seed=seed) if ns \
        else workloads.random_state(cfg["nx"], cfg["ny"], seed=seed)
    dt = 0.2 * cfg["dx"]
    g = np.random.default_rng(seed + 1).standard_normal(U.shape)
    dtype = "f64" if S.torch_dtype.itemsize == 8 else "f32"
    return to_dev(U, dtype), dt, to_dev(g, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_forward_outputs_in_bounds(shape, bc, dtype):
    nx, ny = shape
    cfg = _cfg(nx, ny, *bc)
    S = solver_for(cfg, dtype)
    U, dt, _ = _inputs(S, cfg, 7 + nx)
    o = Guarded(S)
    S.step(U, o.out, dt)
    o.check("lf_step")
    o, us = Guarded(S), Guarded(S)
    S.step_save(U, o.out, us.out, dt)
    o.check("lf_step_save (U^{n+1})")
    us.check("lf_step_save (U*)")
    for stage in (1, 2):
        o = Guarded(S)
        S.stage(stage, U, o.out, dt, base=U if stage == 2 else None)
        o.check(f"lf_stage {stage}")
    o = Guarded(S)
    S.residual(U, o.out)
    o.check("lf_residual")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_outputs_in_bounds(shape, bc, dtype):
    nx, ny = shape
    cfg = _cfg(nx, ny, *bc)
    S = solver_for(cfg, dtype)
    U, dt, g = _inputs(S, cfg, 11 + nx)
    o = Guarded(S)
    S.residual_vjp(U, g, o.out)
    o.check("lf_residual_vjp")
    o = Guarded(S)
    S.adjoint_step(U, dt, g, o.out)
    o.check("lf_adjoint_step")
    us = S.empty_state()
    S.step_save(U, S.empty_state(), us, dt)
    o = Guarded(S)
    S.adjoint_step_ustar(U, us, dt, g, o.out)
    o.check("lf_adjoint_step_ustar")
    o = Guarded(S)
    S.adjoint_step_noalloc(U, dt, g, o.out)
    o.check("lf_adjoint_step_noalloc")


@pytest.mark.parametrize("variant", [dict(ns=2), dict(ns=1), dict(recon=1)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_variant_step_outputs_in_bounds(variant, bc):
    cfg = _cfg(97, 45, *bc, **variant)
    S = solver_for(cfg, "f64")
    U, dt, _ = _inputs(S, cfg, 5)
    o = Guarded(S)
    S.step(U, o.out, dt)
    o.check(f"lf_step {variant}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bcx", [0, 1])
@pytest.mark.parametrize("shape", [(61, 1), (61, 3), (130, 37), (9, 5)])
def test_strip_step_outputs_in_bounds(shape, bcx, dtype):
    """lf_step_halo (ghost rows given) on strips shorter and taller than
    the ghost rows: every output element written, nothing beyond."""
    import torch
    nx, ny = shape
    cfg = _cfg(nx, ny, bcx, 0)
    S = solver_for(cfg, dtype)
    U, dt, _ = _inputs(S, cfg, 3 + ny)
    gl = workloads.random_state(nx, 4, seed=100 + ny)
    gh = workloads.random_state(nx, 4, seed=200 + ny)
    glo, ghi = to_dev(gl, dtype).contiguous(), to_dev(gh, dtype).contiguous()
    assert tuple(glo.shape) == (4, 4, nx) and glo.dtype == S.torch_dtype
    o = Guarded(S)
    S.step_halo(U, glo, ghi, o.out, dt)
    torch.cuda.synchronize()
    o.check(f"lf_step_halo {shape}")
