"""Parity of cic_accumulate (the cloud-in-cell comparator) with the FP64
oracle, through the C ABI.  Bars as for PSI-CELL: binary64 within 1e-12,
binary32 within 1e-5 (relative L2 and per cell); outside and skipped counts
exact; the weight sums within the same bars."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import as_precision, assert_fields_close, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_20829_amd as F
    c = F.Context(0)
    yield c
    c.close()


def _run(ctx, mesh, cloud, prec, weight, cell_scale=None):
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    st, keep = F.make_trajectories(cloud.x.to(DEV).contiguous(), None, cloud.v.to(DEV, dt).contiguous(),
                                   cloud.ug.to(DEV, dt).contiguous(), cloud.r.to(DEV, dt).contiguous(), 1.0)
    cs = torch.as_tensor(cell_scale).to(DEV, dt).contiguous() if cell_scale is not None else None
    M = mesh.cells
    S_mass, S_mom, den = F.alloc_fields(M, mesh.dim, dt, DEV)
    for t in [S_mass, *S_mom, den]:
        t.fill_(float("nan"))
    p = F.Params(rho_d=W.RHO_D, mu=W.MU_AIR, delta=W.DELTA_EVAP, h0=0.01)
    ctx.cic_accumulate(F.mesh_of(mesh, cs), st, weight, p, S_mass, S_mom, den)
    torch.cuda.synchronize()
    return torch.stack([S_mass, *S_mom]).double().cpu().numpy(), den.double().cpu().numpy(), ctx.stats()


def _check(ctx, mesh, cloud, prec, weight, what, cell_scale=None):
    print(f"[case] cic {what} prec={prec} N={cloud.count} mesh={mesh.n}", flush=True)
    S, ws, st = _run(ctx, mesh, cloud, prec, weight, cell_scale)
    c = as_precision(cloud, prec)
    Sref, wref, out, nf = oracle.cic(mesh, c, weight, W.RHO_D, W.MU_AIR, W.DELTA_EVAP, cell_scale=cell_scale)
    assert_fields_close(S, Sref, TOL[prec], f"cic {what} {prec}")
    assert rel_l2(ws, wref) <= TOL[prec]
    assert st["outside"] == out and st["skipped"] == nf
    return out, nf


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("periodic", [True, False])
def test_3d_ragged(ctx, prec, periodic):
    mesh = W.Mesh(3, (37, 21, 19), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (periodic,) * 3)
    cloud = W.abc_cloud(400_000, seed=31)
    cloud.x = cloud.x * 1.06 - 0.03          # some outside a closed box, some across the wrap
    cloud.r[::1009] = float("nan")
    out, nf = _check(ctx, mesh, cloud, prec, 0.7, f"3-D periodic={periodic}")
    assert nf > 0 and (out > 0) == (not periodic)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_3d_many_tiles_unsorted_scatter(ctx, prec):
    # 170 x 160 x 140 cells need more than 1024 of the sorted scatter's tiles
    # (16 x 16 x 8; 16 x 8 x 8 in binary64), so the records take the
    # unsorted scatter into the smaller tiles; ragged last tiles on every axis
    mesh = W.Mesh(3, (170, 160, 140), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (True, False, True))
    cloud = W.abc_cloud(600_000, seed=33)
    cloud.x = cloud.x * 1.04 - 0.02
    cloud.r[::997] = float("nan")
    out, nf = _check(ctx, mesh, cloud, prec, 0.3, "3-D many tiles")
    assert nf > 0 and out > 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_2d_taylor_green(ctx, prec):
    mesh = W.Mesh(2, (64, 45), (0.0, 0.0), (1.0, 1.0), (False, True))
    cloud = W.taylor_green_cloud(300_000, seed=32)
    cs = np.linspace(0.5, 2.0, mesh.cells)
    _check(ctx, mesh, cloud, prec, W.N0_DEFAULT / cloud.count, "2-D", cell_scale=cs)


def test_one_cell_periodic_axes_and_empty(ctx):
    """Periodic axes of one cell (both stencil corners on the same cell) and
    a cloud with no particle."""
    mesh = W.Mesh(3, (1, 5, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (True, True, True))
    cloud = W.abc_cloud(50_000, seed=33)
    _check(ctx, mesh, cloud, "f64", 2.0, "one-cell axes")
    S, ws, st = _run(ctx, W.unit_mesh(3, 8, True), cloud.subset(torch.arange(0)), "f32", 1.0)
    assert np.all(S == 0.0) and np.all(ws == 0.0)


def test_deterministic_and_conservative(ctx):
    mesh = W.unit_mesh(3, 32, False)
    cloud = W.abc_cloud(1_000_000, seed=34)
    S1, w1, _ = _run(ctx, mesh, cloud, "f32", 1.0)
    S2, w2, _ = _run(ctx, mesh, cloud, "f32", 1.0)
    assert np.array_equal(S1, S2) and np.array_equal(w1, w2)
    assert w1.sum() == pytest.approx(cloud.count, rel=1e-6)


@pytest.mark.timeout(300)
def test_full_size_sampled_cells(ctx):
    """200M particles on the 128^3 periodic mesh: the weights sum to the
    particle count, and 256 sampled cells match the oracle run over the
    particles within one cell of them (a cell's CIC sums depend only on
    particles whose cell is next to it)."""
    import paper_2512_20829_amd as F
    mesh = W.unit_mesh(3, 128, True)
    n = 128
    Np = 200_000_000
    print(f"[case] cic N={Np} mesh={mesh.n}", flush=True)
    cl = W.abc_cloud(Np, seed=0, device=DEV, jacobian=False)
    v, ug, r = cl.v.float().contiguous(), cl.ug.float().contiguous(), cl.r.float().contiguous()
    st, _ = F.make_trajectories(cl.x.contiguous(), None, v, ug, r, 1.0)
    S_mass, S_mom, den = F.alloc_fields(mesh.cells, 3, torch.float32, DEV)
    w = W.N0_DEFAULT / Np
    p = F.Params(rho_d=W.RHO_D, mu=W.MU_AIR, delta=W.DELTA_EVAP, h0=0.01)
    ctx.cic_accumulate(F.mesh_of(mesh), st, w, p, S_mass, S_mom, den)
    torch.cuda.synchronize()
    assert float(den.double().sum()) == pytest.approx(Np, rel=1e-6)
    S = torch.stack([S_mass, *S_mom]).double().cpu().numpy()
    g = np.random.default_rng(4)
    cells = np.sort(g.choice(mesh.cells, 256, replace=False))
    near = torch.zeros((n, n, n), dtype=torch.bool, device=DEV)
    c = torch.as_tensor(cells, device=DEV)
    cz, cy, cx = c // (n * n), (c // n) % n, c % n
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                near[(cz + dz) % n, (cy + dy) % n, (cx + dx) % n] = True
    ix = torch.floor(cl.x * n).to(torch.int64) % n
    pick = near[ix[2], ix[1], ix[0]]
    del ix
    sub = W.Trajectories(cl.x[:, pick].cpu(), torch.empty(0, dtype=torch.float64), v[:, pick].double().cpu(),
                         ug[:, pick].double().cpu(), r[pick].double().cpu(), 1.0)
    Sref, wref, _, _ = oracle.cic(mesh, sub, w, W.RHO_D, W.MU_AIR, W.DELTA_EVAP)
    assert_fields_close(S[:, cells], Sref[:, cells], TOL["f32"], "cic 200M sampled")
    assert rel_l2(den.double().cpu().numpy()[cells], wref[cells]) <= TOL["f32"]
