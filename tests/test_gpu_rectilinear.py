"""Rectilinear (stretched) Cartesian meshes through fla_project_sources:
per-axis cell edges in fla_mesh, cell centres at the edge midpoints.  Parity
with the oracle's estimator at the same centroids (element-wise, per-cell
pair counts exact), agreement with the general-mesh path on the same cells,
batches and the producer with such meshes, and the entry points that refuse
them."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import as_precision, assert_fields_close, device_traj, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_20829_amd as F
    c = F.Context(0)
    yield c
    c.close()


def _edges(n, lo, hi, beta):
    return [W.stretched_edges(n[a], lo[a], hi[a], beta[a]) if beta[a] > 0 else
            torch.linspace(lo[a], hi[a], n[a] + 1, dtype=torch.float64) for a in range(len(n))]


def _run(ctx, mesh, edges, wl, prec, traj=None, mode=0):
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    ed = [e.to(DEV).contiguous() for e in edges]
    tr, keep = device_traj(traj if traj is not None else wl.traj, prec)
    M = mesh.cells
    S_mass, S_mom, den = F.alloc_fields(M, mesh.dim, dt, DEV)
    for t in [S_mass, *S_mom, den]:
        t.fill_(float("nan"))
    pairs = torch.full((M,), -1, dtype=torch.int32, device=DEV)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, scale=0.8, count_pairs=True,
                 mode=mode)
    ctx.project_sources(F.mesh_of(mesh, edges=ed), tr, p, S_mass, S_mom, den, pairs=pairs)
    torch.cuda.synchronize()
    return (torch.stack([S_mass, *S_mom]).double().cpu().numpy(), den.double().cpu().numpy(),
            pairs.cpu().numpy().astype(np.int64), ctx.stats())


def _check(ctx, mesh, edges, wl, prec, what):
    print(f"[case] rectilinear {what} prec={prec} n={mesh.n}", flush=True)
    S, den, pairs, st = _run(ctx, mesh, edges, wl, prec)
    cells = W.rectilinear_cells(edges, mesh.periodic)
    ref, terms = oracle.project_points(cells, as_precision(wl.traj, prec), wl.rho_d, wl.mu, wl.delta, wl.h0,
                                       cutoff=wl.cutoff, f32_decision=(prec == "f32"), scale=0.8)
    assert_fields_close(S, ref.S, TOL[prec], f"rectilinear {what} {prec}")
    assert rel_l2(den, ref.den) <= TOL[prec]
    np.testing.assert_array_equal(pairs, ref.pairs)
    assert st["pairs"] == int(ref.pairs.sum()) and st["skipped"] == terms.skipped
    return S, pairs, cells


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_stretched_3d_ragged(ctx, prec):
    n = (21, 26, 17)
    mesh = W.Mesh(3, n, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (True, False, True))
    edges = _edges(n, mesh.lo, mesh.hi, (1.2, 2.5, 0.0))
    wl = W.small_random_3d(3000, 8, seed=81, periodic=True, h0=0.02)
    wl.traj.x = wl.traj.x * 1.04 - 0.02          # some outside the closed y walls
    S, pairs, cells = _check(ctx, mesh, edges, wl, prec, "3-D stretched")
    assert pairs.sum() > 0
    # the general-mesh path at the same centroids takes the same decisions
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    cs, ck = F.cells_of(cells, DEV)
    ix = ctx.cell_index(cs)
    tr, keep = device_traj(wl.traj, prec)
    Sm, Sv, den = F.alloc_fields(cells.count, 3, dt, DEV)
    pc = torch.full((cells.count,), -1, dtype=torch.int32, device=DEV)
    ctx.project_cells(ix, tr, F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, scale=0.8), Sm, Sv, den,
                      pairs=pc)
    torch.cuda.synchronize()
    ix.close()
    np.testing.assert_array_equal(pc.cpu().numpy().astype(np.int64), pairs)
    assert_fields_close(torch.stack([Sm, *Sv]).double().cpu().numpy(), S, TOL[prec], "rectilinear vs cells")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_stretched_2d_periodic(ctx, prec):
    n = (40, 29)
    mesh = W.Mesh(2, n, (0.0, 0.0), (1.0, 1.0), (True, True))
    edges = _edges(n, mesh.lo, mesh.hi, (2.0, 1.0))
    wl = W.taylor_green_2d(per_axis=48, mesh_n=32, seed=82)
    _check(ctx, mesh, edges, wl, prec, "2-D stretched periodic")


def test_uniform_edges_equal_the_uniform_mesh(ctx):
    """Edges at the uniform positions: bit for bit the uniform mesh's fields
    where the centres coincide bit for bit (the midpoints of lo + i w and
    lo + (i+1) w differ from lo + (i + 1/2) w by rounding only), and the
    same pair counts."""
    from helpers import gpu_run
    wl = W.small_random_3d(2000, 16, seed=83, periodic=True)
    mesh = wl.mesh
    edges = [torch.linspace(0.0, 1.0, 17, dtype=torch.float64) for _ in range(3)]
    S, den, pairs, st = _run(ctx, mesh, edges, wl, "f64")
    Su, denu, stu = gpu_run(ctx, wl, prec="f64", scale=0.8, cell_pairs=True)
    np.testing.assert_array_equal(pairs, stu["cell_pairs"])
    assert_fields_close(S, Su, 1e-12, "uniform edges")


def test_batch_and_producer_with_rectilinear_meshes(ctx):
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(2500, 12, seed=84, periodic=True, h0=0.03)
    n = wl.mesh.n
    edges = [e.to(DEV).contiguous() for e in _edges(n, wl.mesh.lo, wl.mesh.hi, (1.5, 1.0, 0.5))]
    mesh = F.mesh_of(wl.mesh, edges=edges)
    umesh = F.mesh_of(wl.mesh)
    tr, keep = device_traj(wl.traj, "f32")
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0)
    outs, singles = [], []
    for m in (mesh, umesh, mesh):
        o = F.alloc_fields(wl.mesh.cells, 3, torch.float32, DEV, den=False)
        outs.append((o[0], o[1], None))
        s = F.alloc_fields(wl.mesh.cells, 3, torch.float32, DEV, den=False)
        ctx.project_sources(m, tr, p, s[0], s[1])
        singles.append(s)
    ctx.set_batch_graph(False)
    ctx.project_batch([mesh, umesh, mesh], [tr, tr, tr], [p, p, p], outs)
    torch.cuda.synchronize()
    for (a, av, _), (b, bv, _) in zip(outs, singles):
        assert torch.equal(a, b) and all(torch.equal(x, y) for x, y in zip(av, bv))
    assert not torch.equal(singles[0][0], singles[1][0])
    # producer: advance, then project the advanced state the plain way
    d = W.seed_droplets(3, 14, seed=85, device=DEV)
    x0 = d.x.clone()
    dr, dk = F.make_droplets(d.x, d.v, d.J, d.dJ, d.r, d.n0, d.seed_volume)
    flow = F.make_flow(F.FLA_FLOW_ABC, U=0.2, k=1.0)
    Sa = F.alloc_fields(wl.mesh.cells, 3, torch.float64, DEV, den=False)
    pp = F.Params(rho_d=W.RHO_D, mu=W.MU_AIR, delta=W.DELTA_EVAP, h0=1.0 / 14)
    ctx.advance_project(mesh, dr, flow, F.make_step(2e-3, 4, True), pp, F.FLA_F64, Sa[0], Sa[1])
    torch.cuda.synchronize()
    assert not torch.equal(d.x, x0)
    assert torch.isfinite(Sa[0]).all() and float(Sa[0].abs().sum()) > 0.0


def test_entry_points_that_refuse_edges(ctx):
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(500, 8, seed=86, periodic=False)
    edges = [torch.linspace(0.0, 1.0, 9, dtype=torch.float64, device=DEV) for _ in range(3)]
    mesh = F.mesh_of(wl.mesh, edges=edges)
    tr, keep = device_traj(wl.traj, "f32")
    S_mass, S_mom, den = F.alloc_fields(wl.mesh.cells, 3, torch.float32, DEV)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0)
    for t in [S_mass, *S_mom]:
        t.fill_(float("nan"))
    with pytest.raises(F.FlaError, match="INVALID_ARG"):
        ctx.project_sources(mesh, tr, F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0,
                                               mode=F.FLA_DEPOSIT), S_mass, S_mom, den)
    with pytest.raises(F.FlaError, match="INVALID_ARG"):
        ctx.psicell_accumulate(mesh, tr, 1.0, p, S_mass, S_mom, den)
    with pytest.raises(F.FlaError, match="INVALID_ARG"):
        ctx.cic_accumulate(mesh, tr, 1.0, p, S_mass, S_mom, den)
    torch.cuda.synchronize()
    assert torch.isnan(S_mass).all()


@pytest.mark.timeout(300)
def test_full_size_stretched_mesh_sampled_cells(ctx):
    """The 2M-trajectory ABC workload on a 128^3 mesh stretched along every
    axis (periodic) through fla_project_sources: 256 sampled cells against
    the oracle over all trajectories, per-cell pairs exact."""
    wl = W.abc_lattice_3d()
    edges = [W.stretched_edges(128, 0.0, 1.0, 1.5) for _ in range(3)]
    print(f"[case] rectilinear stretched 128^3 N={wl.traj.count}", flush=True)
    S, den, pairs, st = _run(ctx, wl.mesh, edges, wl, "f32")
    cells = W.rectilinear_cells(edges, wl.mesh.periodic)
    sel = np.sort(np.random.default_rng(9).choice(cells.count, 256, replace=False))
    oracle.set_threads(16)
    ref, _ = oracle.project_points(cells, as_precision(wl.traj, "f32"), wl.rho_d, wl.mu, wl.delta, wl.h0,
                                   cutoff=wl.cutoff, f32_decision=True, scale=0.8, sel=sel)
    assert_fields_close(S[:, sel], ref.S, TOL["f32"], "rectilinear 128^3 sampled")
    np.testing.assert_array_equal(pairs[sel], ref.pairs)
    assert np.isfinite(S).all()
