"""Shared helpers for the GPU tests: run the library through its C ABI and the
oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import workloads as W


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def as_precision(tr: W.Trajectories, prec: str) -> W.Trajectories:
    """Round v, ug and r to the call's precision (float64 tensors on the CPU),
    so that the oracle sees exactly the values the GPU sees."""
    if prec == "f64":
        return tr
    f = lambda t: t.to(torch.float32).to(torch.float64)
    return W.Trajectories(tr.x, tr.J, f(tr.v), f(tr.ug), f(tr.r), tr.n0, tr.seed_volume)


def device_traj(tr: W.Trajectories, prec: str):
    """Device copies of a trajectory record in the call's precision; returns
    (fla_trajectories struct, tensors to keep alive)."""
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    dev = torch.device("cuda", 0)
    n0 = tr.n0.to(dev) if isinstance(tr.n0, torch.Tensor) else tr.n0
    return F.make_trajectories(tr.x.to(dev, torch.float64).contiguous(), tr.J.to(dev, torch.float64).contiguous(),
                               tr.v.to(dev, dt).contiguous(), tr.ug.to(dev, dt).contiguous(),
                               tr.r.to(dev, dt).contiguous(), n0, tr.seed_volume)


def gpu_run(ctx, wl: W.Workload, prec: str = None, mode: int = 0, count_pairs: bool = True,
            scale: float = 1.0, cell_scale=None, h_factor=None, psicell_cloud=None, weight: float = 1.0,
            traj: W.Trajectories = None, cell_pairs: bool = False):
    """Run fla_project_sources (or psicell_accumulate if a cloud is given) and
    return (S (C, M) float64 numpy, den numpy, stats dict).  With cell_pairs,
    the projection also fills the per-cell pair plane, returned as
    stats["cell_pairs"] (int64 numpy)."""
    import paper_2512_20829_amd as F
    prec = prec or wl.precision
    dt = torch.float64 if prec == "f64" else torch.float32
    tr = psicell_cloud if psicell_cloud is not None else (traj if traj is not None else wl.traj)
    dev = torch.device("cuda", 0)
    x = tr.x.to(dev, torch.float64).contiguous()
    J = tr.J.to(dev, torch.float64).contiguous()
    v = tr.v.to(dev, dt).contiguous()
    ug = tr.ug.to(dev, dt).contiguous()
    r = tr.r.to(dev, dt).contiguous()
    n0 = tr.n0.to(dev) if isinstance(tr.n0, torch.Tensor) else tr.n0
    st, keep = F.make_trajectories(x, J, v, ug, r, n0, tr.seed_volume)
    cs = None
    if cell_scale is not None:
        cs = torch.as_tensor(cell_scale).to(dev, dt).contiguous()
    mesh = F.mesh_of(wl.mesh, cs)
    M = wl.mesh.cells
    S_mass, S_mom, den = F.alloc_fields(M, wl.mesh.dim, dt, dev)
    for t in [S_mass, *S_mom, den]:
        t.fill_(float("nan"))
    hf = h_factor.to(dev, torch.float32).contiguous() if h_factor is not None else None
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, scale=scale,
                 mode=mode, count_pairs=count_pairs, h_factor=hf)
    pairs = None
    if cell_pairs and psicell_cloud is None:
        pairs = torch.full((M,), -1, dtype=torch.int32, device=dev)
    if psicell_cloud is not None:
        ctx.psicell_accumulate(mesh, st, weight, p, S_mass, S_mom, den)
    else:
        ctx.project_sources(mesh, st, p, S_mass, S_mom, den, pairs=pairs)
    torch.cuda.synchronize()
    S = torch.stack([S_mass, *S_mom]).double().cpu().numpy()
    stats = ctx.stats()
    if pairs is not None:
        stats["cell_pairs"] = pairs.cpu().numpy().astype(np.int64)
    return S, den.double().cpu().numpy(), stats


def oracle_run(wl: W.Workload, prec: str = None, scale: float = 1.0, cell_scale=None, cells=None,
               h_factor=None, traj: W.Trajectories = None):
    prec = prec or wl.precision
    tr = as_precision(traj if traj is not None else wl.traj, prec)
    hf = None
    if h_factor is not None:
        hf = h_factor.to(torch.float32).to(torch.float64).numpy()
    p, t = oracle.project(wl.mesh, tr, wl.rho_d, wl.mu, wl.delta, wl.h0, cutoff=wl.cutoff,
                          f32_decision=(prec == "f32"), scale=scale, cell_scale=cell_scale,
                          cells=cells, h_factor=hf)
    return p, t


def assert_fields_close(S_gpu, S_ref, tol: float, what: str = ""):
    """Per source field: relative L2 error within tol, and every cell within
    tol times the field's largest magnitude (a single cell cannot hide in
    the L2 norm)."""
    errs = [rel_l2(S_gpu[k], S_ref[k]) for k in range(S_ref.shape[0])]
    cell = [float(np.max(np.abs(S_gpu[k] - S_ref[k])) / max(np.max(np.abs(S_ref[k])), 1e-300))
            if S_ref[k].size else 0.0 for k in range(S_ref.shape[0])]
    print(f"[rel-l2] {what}: " + " ".join(f"{e:.2e}" for e in errs) +
          " | max cell err / max|S|: " + " ".join(f"{e:.2e}" for e in cell), flush=True)
    for k, e in enumerate(errs):
        assert e <= tol, f"{what} field {k}: rel L2 {e:.3e} > {tol:.1e}"
    for k, e in enumerate(cell):
        assert e <= tol, f"{what} field {k}: a cell is off by {e:.3e} of max|S| > {tol:.1e}"
