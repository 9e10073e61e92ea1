"""CPU checks of the test harness and of the C ABI's host side.

  * the patch sampler used by the full-size GPU parity tests reproduces a
    full-grid oracle step exactly at every cell, for every boundary
    combination and for grids smaller than the patch;
  * liblagrangeflux.so loads and exports every function declared in
    include/lagrangeflux.h;
  * lf_init validates its parameters and every entry point rejects null
    pointers, bad time steps and aliasing before any HIP call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import oracle_step_at

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("shape", [(13, 11), (5, 3), (9, 9), (1, 6)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_patch_sampler_is_exact(shape, bc):
    nx, ny = shape
    cfg = dict(nx=nx, ny=ny, dx=0.1, dy=0.1, gamma=1.4, cfl=0.5, beta=1.5, bc_x=bc[0], bc_y=bc[1])
    U = workloads.random_state(nx, ny, seed=nx * ny + bc[0])
    P = oracle.Params(nx, ny, 0.1, 0.1, bc_x=bc[0], bc_y=bc[1])
    rc, dt = oracle.dt(P, U)
    full = oracle.step(P, U, dt)
    cells = [(i, j) for j in range(ny) for i in range(nx)]
    got = oracle_step_at(U, cfg, dt, cells)
    for k, (i, j) in enumerate(cells):
        assert np.array_equal(got[k], full[:, j, i]), (i, j)


def _header_functions():
    text = open(os.path.join(ROOT, "include", "lagrangeflux.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    import paper_1607_08710_amd as L
    names = _header_functions()
    assert set(names) == set(L.ABI_FUNCTIONS), names
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n


def _params(**kw):
    import paper_1607_08710_amd as L
    base = dict(nx=64, ny=32, dx=0.1, dy=0.1, gamma=1.4, cfl=0.5, beta=1.5, bc_x=0, bc_y=1,
                dtype=L.LF_F64)
    base.update(kw)
    return L.Params(**base)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-1), dict(dx=0.0), dict(dy=float("nan")),
                                 dict(gamma=1.0), dict(gamma=3.5), dict(beta=-0.1), dict(beta=2.5), dict(beta=0.5),
                                 dict(cfl=0.0), dict(bc_x=2), dict(bc_y=-1), dict(dtype=7),
                                 dict(nx=65536, ny=65536), dict(n_species=-1), dict(n_species=5),
                                 dict(reconstruction=2), dict(reconstruction=1, n_species=1)])
def test_init_rejects(bad):
    import paper_1607_08710_amd as L
    with pytest.raises(L.LFError) as e:
        L.init(_params(**bad))
    assert e.value.status == L.LF_ERR_ARG


def test_init_workspace_size():
    import paper_1607_08710_amd as L
    for dt, esz in ((L.LF_F64, 8), (L.LF_F32, 4)):
        ctx, ws = L.init(_params(dtype=dt))
        state = 4 * 64 * 32 * esz
        assert ws >= 2 * state  # U* and the adjoint intermediate
        assert ws % 256 == 0
        L.lib().lf_destroy(ctx)
    L.lib().lf_destroy(None)
    assert L.status_string(L.LF_ERR_NONPHYSICAL).startswith("non-physical")


def test_entry_points_validate_before_hip():
    """Every call below fails argument validation, so no HIP call is made."""
    import paper_1607_08710_amd as L
    lib = L.lib()
    ctx, ws_bytes = L.init(_params())
    vp = ctypes.c_void_p
    A, B, W = vp(0x100000), vp(0x400000), vp(0x10000000)  # never dereferenced
    state = 4 * 64 * 32 * 8
    d = ctypes.c_double()
    n = ctypes.c_int64()
    E = L.LF_ERR_ARG
    assert lib.lf_dt(ctx, None, W, None, ctypes.byref(d)) == E
    assert lib.lf_dt(ctx, A, W, None, None) == E
    assert lib.lf_step(ctx, A, B, -1.0, W, None) == E
    assert lib.lf_step(ctx, A, B, float("inf"), W, None) == E
    assert lib.lf_step(ctx, A, vp(0x100000 + 8), 0.1, W, None) == E  # partial overlap
    assert lib.lf_step(None, A, B, 0.1, W, None) == E
    assert lib.lf_step(ctx, A, B, 0.1, vp(0x100000 + state - 8), None) == E  # ws overlaps Un
    assert lib.lf_advance(ctx, A, 0.0, 1.0, -1, W, None, ctypes.byref(d), ctypes.byref(n), None, 0) == E
    assert lib.lf_advance(ctx, A, float("nan"), 1.0, 5, W, None, ctypes.byref(d), ctypes.byref(n), None, 0) == E
    assert lib.lf_advance(ctx, A, 0.0, 1.0, 5, W, None, None, ctypes.byref(n), None, 0) == E
    assert lib.lf_advance(ctx, A, 0.0, 1.0, 5, W, None, ctypes.byref(d), ctypes.byref(n), None, 3) == E
    assert lib.lf_residual(ctx, A, A, W, None) == E
    assert lib.lf_residual_vjp(ctx, A, B, A, W, None) == E
    assert lib.lf_residual_vjp(ctx, A, B, B, W, None) == E
    assert lib.lf_adjoint_step(ctx, A, 0.1, B, B, W, None) == E
    assert lib.lf_adjoint_step(ctx, A, 0.1, B, A, W, None) == E
    assert lib.lf_adjoint_step(ctx, A, -0.1, B, vp(0x800000), W, None) == E
    assert lib.lf_totals(ctx, A, W, None, None) == E
    C = vp(0x700000)
    assert lib.lf_step_save(ctx, A, B, None, 0.1, W, None) == E
    assert lib.lf_step_save(ctx, A, B, A, 0.1, W, None) == E          # U* overlaps Un
    assert lib.lf_step_save(ctx, A, B, C, -1.0, W, None) == E
    assert lib.lf_step_save(ctx, A, A, C, 0.1, W, None) == E          # no in-place form
    assert lib.lf_adjoint_step_ustar(ctx, A, B, 0.1, C, B, W, None) == E  # lam_n overlaps U*
    assert lib.lf_adjoint_step_ustar(ctx, A, None, 0.1, C, B, W, None) == E
    ghost = 4 * 4 * 64 * 8  # [4 fields][4 rows][64] doubles
    assert lib.lf_step_halo(ctx, A, None, C, B, 0.1, W, None) == E
    assert lib.lf_step_halo(ctx, A, C, C, B, float("nan"), W, None) == E
    assert lib.lf_step_halo(ctx, A, C, C, A, 0.1, W, None) == E                      # output is the input
    assert lib.lf_step_halo(ctx, A, C, vp(B.value + ghost // 2), B, 0.1, W, None) == E  # output overlaps ghost_hi
    assert lib.lf_step_halo(ctx, A, vp(W.value + 64), C, B, 0.1, W, None) == E     # ghost_lo inside ws
    lib.lf_destroy(ctx)


def test_species_context_validation():
    """With mass fractions the state holds 4 + n_species planes (the
    overlap checks use that size) and the adjoint entry points refuse the
    context; all of it is decided before any HIP call."""
    import paper_1607_08710_amd as L
    lib = L.lib()
    ctx0, ws0 = L.init(_params())
    ctx, ws = L.init(_params(n_species=3))
    assert ws >= ws0 + 3 * 64 * 32 * 8  # U* carries the fractions too
    L.lib().lf_destroy(ctx0)
    vp = ctypes.c_void_p
    state = 7 * 64 * 32 * 8
    A, B, C, W = vp(0x1000000), vp(0x2000000), vp(0x3000000), vp(0x10000000)
    E = L.LF_ERR_ARG
    # out starts inside the 7-plane input (it would not overlap a 4-plane one)
    assert lib.lf_step(ctx, A, vp(0x1000000 + 5 * 64 * 32 * 8), 0.1, W, None) == E
    assert lib.lf_residual(ctx, A, vp(0x1000000 + state - 8), W, None) == E
    assert lib.lf_residual_vjp(ctx, A, B, C, W, None) == E
    assert lib.lf_adjoint_step(ctx, A, 0.1, B, C, W, None) == E
    lib.lf_destroy(ctx)


def test_conservative_reconstruction_context_validation():
    """The conservative-reconstruction ablation has no adjoint: both
    adjoint entry points refuse the context before any HIP call."""
    import paper_1607_08710_amd as L
    lib = L.lib()
    ctx, ws = L.init(_params(reconstruction=L.LF_RECON_CONSERVATIVE))
    vp = ctypes.c_void_p
    A, B, C, W = vp(0x1000000), vp(0x2000000), vp(0x3000000), vp(0x10000000)
    assert lib.lf_residual_vjp(ctx, A, B, C, W, None) == L.LF_ERR_ARG
    assert lib.lf_adjoint_step(ctx, A, 0.1, B, C, W, None) == L.LF_ERR_ARG
    lib.lf_destroy(ctx)


def test_noalloc_entry_validates_before_hip():
    """lf_adjoint_step_noalloc refuses a grid whose U* and mu do not fit
    its fixed scratch (LF_ERR_TOO_LARGE: FP64 beyond 1024^2 cells, FP32
    beyond 2 x 1024^2) and bad arguments (LF_ERR_ARG), before any HIP
    call."""
    import paper_1607_08710_amd as L
    lib = L.lib()
    vp = ctypes.c_void_p
    A, B, C = vp(0x1000000), vp(0x40000000), vp(0x80000000)
    for dtype, nx, ny in ((L.LF_F64, 1025, 1024), (L.LF_F64, 1024, 1025), (L.LF_F32, 2049, 1024),
                          (L.LF_F32, 2048, 1025)):
        ctx, _ = L.init(_params(nx=nx, ny=ny, dtype=dtype))
        assert lib.lf_adjoint_step_noalloc(ctx, A, 0.1, B, C, None) == L.LF_ERR_TOO_LARGE
        lib.lf_destroy(ctx)
    assert L.status_string(L.LF_ERR_TOO_LARGE).startswith("grid too large")
    ctx, _ = L.init(_params(nx=1024, ny=1024))
    E = L.LF_ERR_ARG
    assert lib.lf_adjoint_step_noalloc(None, A, 0.1, B, C, None) == E
    assert lib.lf_adjoint_step_noalloc(ctx, None, 0.1, B, C, None) == E
    assert lib.lf_adjoint_step_noalloc(ctx, A, -0.1, B, C, None) == E
    assert lib.lf_adjoint_step_noalloc(ctx, A, float("nan"), B, C, None) == E
    assert lib.lf_adjoint_step_noalloc(ctx, A, 0.1, B, B, None) == E   # lam_n is lam_np1
    assert lib.lf_adjoint_step_noalloc(ctx, A, 0.1, B, A, None) == E   # lam_n is Un
    lib.lf_destroy(ctx)
    for kw in (dict(n_species=1), dict(reconstruction=L.LF_RECON_CONSERVATIVE)):
        ctx, _ = L.init(_params(**kw))
        assert lib.lf_adjoint_step_noalloc(ctx, A, 0.1, B, C, None) == E
        lib.lf_destroy(ctx)


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_1607_08710_amd as L
    with pytest.raises(ValueError):
        L.Solver(_params(), device="cpu")
