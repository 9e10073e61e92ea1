"""Seeded, synthetic inputs shared by the oracle tests, the GPU tests and
the benchmark.

This module holds none of the scheme's arithmetic: it only builds initial
conditions from their analytic definitions (point values at cell centres
x_i = x0 + (i + 1/2) dx) and turns primitive fields into the conservative
vector with the perfect-gas law of the Euler system.  It does not import
the oracle or the GPU library.

Every workload returns ``(U, cfg)``: ``U`` a float64 array of shape
(4, ny, nx) holding (rho, rho*u, rho*v, rho*E), ``cfg`` a dict of plain
grid / physics parameters (nx, ny, dx, dy, gamma, cfl, beta, bc_x, bc_y,
t_end, plus case-specific extras).
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC = 0
TRANSMISSIVE = 1


def prim_to_cons(gamma: float, rho, u, v, p) -> np.ndarray:
    """(rho, u, v, p) -> (rho, rho u, rho v, rho E), rho E = p/(gamma-1) + rho|u|^2/2."""
    rho, u, v, p = (np.asarray(a, dtype=np.float64) for a in np.broadcast_arrays(rho, u, v, p))
    U = np.empty((4,) + rho.shape)
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * v
    U[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return U


def cell_centres(n: int, lo: float, hi: float) -> np.ndarray:
    d = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * d


def _cfg(nx, ny, Lx, Ly, bc_x, bc_y, gamma=1.4, cfl=0.5, beta=1.5, **extra):
    c = dict(nx=int(nx), ny=int(ny), dx=Lx / nx, dy=Ly / ny, gamma=gamma, cfl=cfl,
             beta=beta, bc_x=bc_x, bc_y=bc_y)
    c.update(extra)
    return c


# ---- shock tubes ------------------------------------------------------------

SOD_LEFT = (1.0, 0.0, 1.0)      # (rho, u, p) for x < 0.5
SOD_RIGHT = (0.125, 0.0, 0.1)   # (rho, u, p) for x > 0.5


def shock_tube(n: int, left, right, *, ny: int = 4, axis: str = "x", gamma: float = 1.4,
               cfl: float = 0.5, beta: float = 1.5, t_end: float = 0.2, x0: float = 0.5):
    """1D Riemann problem on [0,1] along ``axis``, extruded to ``ny`` cells
    across (square cells: the cross extent is ny/n), transmissive on both
    axes."""
    x = cell_centres(n, 0.0, 1.0)
    lo = x < x0
    rho = np.where(lo, left[0], right[0])
    un = np.where(lo, left[1], right[1])
    p = np.where(lo, left[2], right[2])
    if axis == "x":
        shape = (ny, n)
        R, U_, V_, P_ = (np.broadcast_to(a[None, :], shape) for a in (rho, un, 0 * un, p))
        cfg = _cfg(n, ny, 1.0, ny / n, TRANSMISSIVE, TRANSMISSIVE, gamma, cfl, beta)
    else:
        shape = (n, ny)
        R, V_, U_, P_ = (np.broadcast_to(a[:, None], shape) for a in (rho, un, 0 * un, p))
        cfg = _cfg(ny, n, ny / n, 1.0, TRANSMISSIVE, TRANSMISSIVE, gamma, cfl, beta)
    cfg.update(t_end=t_end, x0=x0, left=tuple(left), right=tuple(right), axis=axis)
    return prim_to_cons(gamma, R, U_, V_, P_), cfg


def sod(n: int = 400, ny: int = 4, axis: str = "x", **kw):
    """Sod shock tube (1,0,1) | (0.125,0,0.1), 400x4 cells, CFL 0.5, t = 0.2."""
    return shock_tube(n, SOD_LEFT, SOD_RIGHT, ny=ny, axis=axis, **kw)


# ---- isentropic vortex -------------------------------------------------------

def vortex_prim(x, y, t: float = 0.0, *, gamma: float = 1.4, eps: float = 5.0,
                L: float = 10.0, xc: float = 5.0, yc: float = 5.0, u0=1.0, v0=1.0):
    """Isentropic vortex of strength eps advected by (u0, v0) on the
    periodic [0,L]^2: the exact solution is the initial field translated by
    (u0 t, v0 t), taken at the nearest periodic image of the centre."""
    cx = xc + u0 * t
    cy = yc + v0 * t
    dxp = x - cx
    dyp = y - cy
    dxp = dxp - L * np.round(dxp / L)
    dyp = dyp - L * np.round(dyp / L)
    r2 = dxp * dxp + dyp * dyp
    f = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = u0 - f * dyp
    v = v0 + f * dxp
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return rho, u, v, p


def vortex(n: int, *, t: float = 0.0, gamma: float = 1.4, cfl: float = 0.5, beta: float = 1.5,
           t_end: float = 2.0):
    x = cell_centres(n, 0.0, 10.0)
    X, Y = np.meshgrid(x, x)  # Y[j, i] = y_j, X[j, i] = x_i
    rho, u, v, p = vortex_prim(X, Y, t, gamma=gamma)
    cfg = _cfg(n, n, 10.0, 10.0, PERIODIC, PERIODIC, gamma, cfl, beta, t_end=t_end)
    return prim_to_cons(gamma, rho, u, v, p), cfg


# ---- four-quadrant Riemann problem --------------------------------------------

# (rho, u, v, p) for the quadrants NE (x>1/2, y>1/2), NW, SW, SE.
QUADRANTS = (
    (1.5, 0.0, 0.0, 1.5),
    (0.5323, 1.206, 0.0, 0.3),
    (0.138, 1.206, 1.206, 0.029),
    (0.5323, 0.0, 1.206, 0.3),
)


def four_quadrant(n: int, *, gamma: float = 1.4, cfl: float = 0.5, beta: float = 1.5,
                  steps: int = 1000):
    x = cell_centres(n, 0.0, 1.0)
    X, Y = np.meshgrid(x, x)
    east, north = X > 0.5, Y > 0.5
    q = np.where(north & east, 0, np.where(north & ~east, 1, np.where(~north & ~east, 2, 3)))
    S = np.array(QUADRANTS)
    rho, u, v, p = (S[:, k][q] for k in range(4))
    cfg = _cfg(n, n, 1.0, 1.0, TRANSMISSIVE, TRANSMISSIVE, gamma, cfl, beta, steps=steps)
    return prim_to_cons(gamma, rho, u, v, p), cfg


# ---- Kelvin-Helmholtz shear layer -------------------------------------------

def kelvin_helmholtz(n: int, *, gamma: float = 1.4, cfl: float = 0.5, beta: float = 1.5,
                     steps: int = 500, dtype=np.float64, rows: int | None = None):
    """rho = 2, u = 0.5 for |y - 1/2| < 1/4, else rho = 1, u = -0.5; p = 2.5;
    v = 0.01 sin(4 pi x); periodic [0,1]^2.  The perturbation is
    deterministic (no random draw).  With ``rows`` = m < n only the bottom
    m rows of the n^2 grid are built (an n x m state, cfg ny = m, same dx
    and dy, still periodic: a timing sample of the same rows)."""
    x = cell_centres(n, 0.0, 1.0)
    inner = np.abs(x - 0.5) < 0.25  # along y
    rho_y = np.where(inner, 2.0, 1.0)
    u_y = np.where(inner, 0.5, -0.5)
    v_x = 0.01 * np.sin(4.0 * math.pi * x)
    m = n if rows is None else int(rows)
    U = np.empty((4, m, n), dtype=dtype)
    # built row by row to keep peak host memory at one state
    for j in range(m):
        rho = np.full(n, rho_y[j])
        U[:, j, :] = prim_to_cons(gamma, rho, u_y[j], v_x, 2.5)
    cfg = _cfg(n, m, 1.0, m / n, PERIODIC, PERIODIC, gamma, cfl, beta, steps=steps)
    return U, cfg


# ---- seeded smooth random field (adjoint workload) --------------------------

def smooth_field(n: int, seed: int, kmax2: int = 64, dtype=np.float64) -> np.ndarray:
    """f = sum over integer (kx, ky), 0 < kx^2 + ky^2 <= kmax2, in the half
    plane (kx > 0, or kx = 0 and ky > 0), of cos(2 pi (kx x + ky y) + phi_k),
    with phases phi_k ~ U[0, 2 pi) drawn from numpy PCG64(seed) in the
    enumeration order below; normalised to max |f| = 1 on the grid.
    Evaluated at cell centres of [0,1]^2, periodic by construction."""
    modes = []
    k = int(math.isqrt(kmax2))
    for kx in range(0, k + 1):
        for ky in range(-k, k + 1):
            if kx * kx + ky * ky == 0 or kx * kx + ky * ky > kmax2:
                continue
            if kx == 0 and ky <= 0:
                continue
            modes.append((kx, ky))
    rng = np.random.Generator(np.random.PCG64(seed))
    phases = rng.uniform(0.0, 2.0 * math.pi, size=len(modes))
    x = cell_centres(n, 0.0, 1.0)
    # separable evaluation: cos(a + b + c) via complex exponentials per mode
    ex = {kx: np.exp(2j * math.pi * kx * x) for kx, _ in modes}
    ey = {ky: np.exp(2j * math.pi * ky * x) for _, ky in modes}
    f = np.zeros((n, n))
    for (kx, ky), ph in zip(modes, phases):
        f += np.real(np.exp(1j * ph) * np.outer(ey[ky], ex[kx]))
    f /= np.max(np.abs(f))
    return f.astype(dtype)


def adjoint_case(n: int = 1024, *, seed_ic: int = 1, seed_target: int = 2, gamma: float = 1.4,
                 cfl: float = 0.5, beta: float = 1.5, steps: int = 200, ckpt_every: int = 20):
    """rho0 = 1 + 0.1 f_1, u = v = 0.2, p = 1 on the periodic [0,1]^2;
    target density rho_tgt = 1 + 0.1 f_2."""
    f1 = smooth_field(n, seed_ic)
    rho0 = 1.0 + 0.1 * f1
    U = prim_to_cons(gamma, rho0, 0.2, 0.2, 1.0)
    rho_tgt = 1.0 + 0.1 * smooth_field(n, seed_target)
    cfg = _cfg(n, n, 1.0, 1.0, PERIODIC, PERIODIC, gamma, cfl, beta, steps=steps,
               ckpt_every=ckpt_every, u=0.2, v=0.2, p=1.0)
    return U, rho_tgt, cfg


def fd_directions(n: int, count: int = 8, first_seed: int = 101):
    """Finite-difference directions d_m = f_{100+m}, m = 1..count."""
    return [smooth_field(n, first_seed + m) for m in range(count)]


# ---- generic random states (parity tests) -----------------------------------

def random_state(nx: int, ny: int, seed: int, *, gamma: float = 1.4, rough: bool = True):
    """Positive random state.  ``rough`` draws independent cell values
    (every limiter branch and both upwind sides occur); otherwise a
    smooth field plus small noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if rough:
        rho = rng.uniform(0.5, 1.5, (ny, nx))
        u = rng.uniform(-1.0, 1.0, (ny, nx))
        v = rng.uniform(-1.0, 1.0, (ny, nx))
        p = rng.uniform(0.5, 1.5, (ny, nx))
    else:
        x = cell_centres(nx, 0.0, 1.0)[None, :]
        y = cell_centres(ny, 0.0, 1.0)[:, None]
        ph = rng.uniform(0, 2 * math.pi, 4)
        rho = 1.0 + 0.3 * np.sin(2 * math.pi * x + ph[0]) * np.cos(2 * math.pi * y + ph[1])
        u = 0.5 * np.sin(2 * math.pi * (x + y) + ph[2]) + 0.01 * rng.standard_normal((ny, nx))
        v = 0.5 * np.cos(2 * math.pi * (x - y) + ph[3]) + 0.01 * rng.standard_normal((ny, nx))
        p = 1.0 + 0.2 * np.cos(2 * math.pi * x) * np.sin(2 * math.pi * y)
    return prim_to_cons(gamma, rho, u, v, p)


def kelvin_helmholtz_torch(n: int, *, device="cuda", dtype=None, gamma: float = 1.4, fractions: int = 0):
    """The Kelvin-Helmholtz state of kelvin_helmholtz(), built with torch
    directly in device memory (for the large benchmark grids).  Computed in
    float64 and cast once to ``dtype``.  With ``fractions`` = K > 0 the
    state also carries K mass fractions: the band marker of
    kelvin_helmholtz_fraction() first, then (1 + sin(2 pi (k+1) x)) / 2."""
    import torch
    dtype = dtype or torch.float64
    x = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) / n
    inner = torch.abs(x - 0.5) < 0.25
    rho_y = torch.where(inner, 2.0, 1.0)
    u_y = torch.where(inner, 0.5, -0.5)
    v_x = 0.01 * torch.sin(4.0 * math.pi * x)
    U = torch.empty((4 + fractions, n, n), dtype=dtype, device=device)
    rho = rho_y[:, None].expand(n, n)
    u = u_y[:, None].expand(n, n)
    v = v_x[None, :].expand(n, n)
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * v
    U[3] = 2.5 / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    for k in range(fractions):
        if k == 0:
            y = inner.to(torch.float64)[:, None].expand(n, n)
        else:
            y = (0.5 * (1.0 + torch.sin(2.0 * math.pi * (k + 1) * x)))[None, :].expand(n, n)
        U[4 + k] = rho * y
    cfg = _cfg(n, n, 1.0, 1.0, PERIODIC, PERIODIC, gamma, 0.5, 1.5, steps=500)
    if fractions:
        cfg["ns"] = fractions
    return U, cfg


# ---- the paper's one-dimensional shock tubes ----------------------------------

# name: (left (rho,u,p), right (rho,u,p), final time, cells, Sweby beta)
# Sod, two-rarefaction near vacuum, sonic rarefaction with supersonic contact
# (the text gives T = 0.16, a caption 0.18; 0.16 is used), shock-shock with
# a Mach-40 right state and the minmod limiter (beta = 1).
PAPER_TUBES = {
    "sod": ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.23, (100, 400), 1.5),
    "two_rarefaction": ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 0.16, (200, 2000), 1.5),
    "sonic_rarefaction": ((5.0, 0.0, 5.0), (0.125, 0.0, 0.1), 0.16, (400,), 1.5),
    "shock_shock": ((1.0, 5.0, 1.0), (1.0, -5.0, 0.01), 0.16, (400,), 1.0),
}


def paper_tube(name: str, n: int, *, gamma: float = 1.4, cfl: float = 0.25):
    """One of the paper's shock tubes on [0,1] with n cells in a single row.
    The row's cell is very tall (dy = 1e3), so the CFL sum
    (|u|+c)/dx + (|v|+c)/dy is the one-dimensional (|u|+c)/dx to 1e-5
    relative and CFL 0.25 means what it means in one dimension."""
    left, right, t_end, _, beta = PAPER_TUBES[name]
    x = cell_centres(n, 0.0, 1.0)
    lo = x < 0.5
    rho = np.where(lo, left[0], right[0])[None, :]
    u = np.where(lo, left[1], right[1])[None, :]
    p = np.where(lo, left[2], right[2])[None, :]
    cfg = dict(nx=n, ny=1, dx=1.0 / n, dy=1.0e3, gamma=gamma, cfl=cfl, beta=beta,
               bc_x=TRANSMISSIVE, bc_y=TRANSMISSIVE, t_end=t_end, left=left, right=right)
    return prim_to_cons(gamma, rho, u, 0.0, p), cfg


# ---- passive mass fractions (conservative transport of rho*y_k, Sec. 7) -------

def with_fractions(U, ys):
    """State with the fields rho*y_k appended: U has the 4 Euler fields,
    ys is a list of mass-fraction arrays broadcastable to U[0]."""
    out = np.empty((4 + len(ys),) + U.shape[1:], dtype=U.dtype)
    out[:4] = U
    for k, y in enumerate(ys):
        out[4 + k] = U[0] * np.broadcast_to(y, U.shape[1:])
    return out


def sod_interface(n: int = 400, ny: int = 4, **kw):
    """Sod 400x4 (CFL 0.5, t = 0.2) carrying two materials: y_1 = 1 left of
    the diaphragm, y_2 = 1 - y_1, stored as rho*y_2 = rho - rho*y_1."""
    U, cfg = sod(n, ny, **kw)
    x = cell_centres(n, 0.0, 1.0)[None, :]
    y1 = np.where(x < 0.5, 1.0, 0.0) * np.ones((ny, 1))
    out = with_fractions(U, [y1])
    out = np.concatenate([out, (out[0] - out[4])[None]], axis=0)
    cfg = dict(cfg, ns=2)
    return out, cfg


def advected_fraction(nx: int, ny: int, u: float, v: float, seed: int, *, bc=(PERIODIC, PERIODIC),
                      beta: float = 1.5, rho: float = 1.3, p: float = 0.9, cfl: float = 0.4):
    """Uniform rho, p and velocity (u, v) carrying one rough mass fraction
    (independent uniform draws in [0, 1]): the Euler fields are a fixed
    point and the fraction is linearly advected."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y = rng.uniform(0.0, 1.0, (ny, nx))
    U = prim_to_cons(1.4, np.full((ny, nx), rho), u, v, p)
    cfg = _cfg(nx, ny, 1.0, ny / nx, bc[0], bc[1], 1.4, cfl, beta, ns=1)
    return with_fractions(U, [y]), cfg


def random_state_fractions(nx: int, ny: int, ns: int, seed: int, **kw):
    """random_state() plus ns rough mass fractions in [0, 1]."""
    U = random_state(nx, ny, seed, **kw)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    return with_fractions(U, [rng.uniform(0.0, 1.0, (ny, nx)) for _ in range(ns)])


def kelvin_helmholtz_fraction(n: int, **kw):
    """kelvin_helmholtz() with one material marker: y = 1 inside the band
    |y - 1/2| < 1/4, 0 outside."""
    U, cfg = kelvin_helmholtz(n, **kw)
    yc = cell_centres(n, 0.0, 1.0)
    marker = np.where(np.abs(yc - 0.5) < 0.25, 1.0, 0.0)[:, None]
    return with_fractions(U, [marker]), dict(cfg, ns=1)
