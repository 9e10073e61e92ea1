"""Helpers shared by the GPU tests: building solvers from workload
configs, moving states between the oracle (numpy) and the HIP library
(torch), and the per-field error norms used in the parity bars."""
import numpy as np

import oracle


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def solver_for(cfg, dtype="f64", **over):
    import paper_1607_08710_amd as L
    kw = dict(nx=cfg["nx"], ny=cfg["ny"], dx=cfg["dx"], dy=cfg["dy"], gamma=cfg["gamma"],
              cfl=cfg["cfl"], beta=cfg["beta"], bc_x=cfg["bc_x"], bc_y=cfg["bc_y"],
              dtype=L.LF_F64 if dtype == "f64" else L.LF_F32, n_species=cfg.get("ns", 0),
              reconstruction=cfg.get("recon", 0))
    kw.update(over)
    return L.Solver(L.Params(**kw))


def oracle_params(cfg, **over):
    kw = dict(nx=cfg["nx"], ny=cfg["ny"], dx=cfg["dx"], dy=cfg["dy"], gamma=cfg["gamma"],
              cfl=cfg["cfl"], beta=cfg["beta"], bc_x=cfg["bc_x"], bc_y=cfg["bc_y"],
              ns=cfg.get("ns", 0), recon=cfg.get("recon", 0))
    kw.update(over)
    return oracle.Params(**kw)


def to_dev(U, dtype="f64"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64))
    if dtype == "f32":
        t = t.to(torch.float32)
    return t.cuda()


def to_host(t):
    return t.detach().cpu().to(dtype=__import__("torch").float64).numpy()


def rel_linf(a, b, floor_fields=(1,)):
    """Per-field max|a-b| / max|b|.  A field that is identically zero in b
    is measured against max|b| of the fields in floor_fields (momentum)."""
    out = []
    for f in range(b.shape[0]):
        den = np.abs(b[f]).max()
        if den == 0:
            den = max(np.abs(b[k]).max() for k in floor_fields) or 1.0
        out.append(np.abs(a[f] - b[f]).max() / den)
    return np.array(out)


def rel_l1(a, b, floor_fields=(1,)):
    out = []
    for f in range(b.shape[0]):
        den = np.abs(b[f]).sum()
        if den == 0:
            den = max(np.abs(b[k]).sum() for k in floor_fields) or 1.0
        out.append(np.abs(a[f] - b[f]).sum() / den)
    return np.array(out)


def sample_patch(U, cfg, i, j, r=4):
    """The (2r+1)^2 neighbourhood of cell (i, j) as seen by the stencil:
    wrapped along periodic axes, clipped at transmissive edges (where the
    patch keeps the grid's own boundary).  Returns (patch, ic, jc): the
    patch and the position of (i, j) in it.  With r = 4 one Heun step of
    the patch with transmissive boundaries reproduces the full-grid value
    of the centre cell exactly (the step reads 4 cells along each axis)."""
    nx, ny = cfg["nx"], cfg["ny"]
    if cfg["bc_x"] == oracle.PERIODIC:
        xs = np.arange(i - r, i + r + 1) % nx
        ic = r
    else:
        lo, hi = max(0, i - r), min(nx, i + r + 1)
        xs = np.arange(lo, hi)
        ic = i - lo
    if cfg["bc_y"] == oracle.PERIODIC:
        ys = np.arange(j - r, j + r + 1) % ny
        jc = r
    else:
        lo, hi = max(0, j - r), min(ny, j + r + 1)
        ys = np.arange(lo, hi)
        jc = j - lo
    if hasattr(U, "index_select"):  # a torch tensor, e.g. a state in device memory
        import torch
        iy = torch.as_tensor(ys, device=U.device)
        ix = torch.as_tensor(xs, device=U.device)
        patch = U.index_select(1, iy).index_select(2, ix).to(torch.float64).cpu().numpy()
        return np.ascontiguousarray(patch), ic, jc
    patch = np.ascontiguousarray(U[:, ys][:, :, xs])
    return patch, ic, jc


def oracle_step_at(U, cfg, dt, cells, r=4):
    """Oracle Heun step evaluated only at the listed cells, from patches."""
    out = np.empty((len(cells), U.shape[0]))
    for k, (i, j) in enumerate(cells):
        patch, ic, jc = sample_patch(U, cfg, i, j, r)
        P = oracle.Params(patch.shape[2], patch.shape[1], cfg["dx"], cfg["dy"], cfg["gamma"],
                          cfg["cfl"], cfg["beta"], oracle.TRANSMISSIVE, oracle.TRANSMISSIVE,
                          ns=U.shape[0] - 4, recon=cfg.get("recon", 0))
        out[k] = oracle.step(P, patch, dt)[:, jc, ic]
    return out


def oracle_steps_at(U, cfg, dts, cells):
    """Oracle values after len(dts) Heun steps (at the given time steps)
    from state U, evaluated only at the listed cells (i, j).  Each cell gets
    the patch of radius 4k around it (k = len(dts)) and the patch is stepped
    k times with transmissive boundaries: the step reads 4 cells along each
    axis, so the wrong ghost data of a patch side reaches 4 cells further in
    per step and never the centre.  Along periodic axes the patch wraps; at
    transmissive grid edges it is clipped and keeps the grid's own boundary.
    U may be a numpy array or a torch tensor (the patches are gathered where
    U lives and converted to float64)."""
    k = len(dts)
    out = np.empty((len(cells), U.shape[0]))
    for q, (i, j) in enumerate(cells):
        patch, ic, jc = sample_patch(U, cfg, i, j, 4 * k)
        P = oracle.Params(patch.shape[2], patch.shape[1], cfg["dx"], cfg["dy"], cfg["gamma"],
                          cfg["cfl"], cfg["beta"], oracle.TRANSMISSIVE, oracle.TRANSMISSIVE,
                          ns=U.shape[0] - 4, recon=cfg.get("recon", 0))
        for dt in dts:
            patch = oracle.step(P, patch, float(dt))
        out[q] = patch[:, jc, ic]
    return out


def values_at(U, cells):
    """U[:, j, i] for the listed cells (i, j), as a float64 numpy array of
    shape (len(cells), fields); U is a torch tensor or a numpy array."""
    if hasattr(U, "index_select"):
        import torch
        ii = torch.tensor([c[0] for c in cells], device=U.device)
        jj = torch.tensor([c[1] for c in cells], device=U.device)
        return U[:, jj, ii].to(torch.float64).cpu().numpy().T.copy()
    return np.array([U[:, j, i] for i, j in cells], dtype=np.float64)


def cfl_dt_torch(U, cfg):
    """The CFL time step of reading 7, cfl / max_K [(|u|+c)/dx + (|v|+c)/dy],
    evaluated with plain torch float64 operations wherever U lives: the
    property a device-side dt must satisfy, independent of the library."""
    import torch
    g = cfg["gamma"]
    rho = U[0].to(torch.float64)
    u = U[1].to(torch.float64) / rho
    v = U[2].to(torch.float64) / rho
    p = (g - 1.0) * (U[3].to(torch.float64) - 0.5 * (U[1].to(torch.float64) * u + U[2].to(torch.float64) * v))
    c = torch.sqrt(g * p / rho)
    s = (u.abs() + c) / cfg["dx"] + (v.abs() + c) / cfg["dy"]
    return cfg["cfl"] / s.max().item()
