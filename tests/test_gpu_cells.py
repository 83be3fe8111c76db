"""Parity of fla_project_cells (the estimator at the centroids of a general
mesh, with n_hat of App. A per cell) with the oracle, through the C ABI.
Bars: binary64 within 1e-12, binary32 within 1e-5 (relative L2 and per
cell); per-cell included-pair counts exact (both sides take the inclusion
decision in the same precision from the same binary64 offsets)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import as_precision, assert_fields_close, device_traj, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
TOL = {"f64": 1e-12, "f32": 1e-5}
INJ = dict(n_ref=2.0e5, tau_ref=1.0e-3, area=2.5e-3, v_inj=4.0)


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_20829_amd as F
    c = F.Context(0)
    yield c
    c.close()


def _run(ctx, cells, wl, prec, inj=None, traj=None, per_bucket=0, index=None):
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    cs, keep = F.cells_of(cells, DEV)
    ix = index or ctx.cell_index(cs, per_bucket)
    tr, keep2 = device_traj(traj if traj is not None else wl.traj, prec)
    M = cells.count
    S_mass, S_mom, den = F.alloc_fields(M, cells.dim, dt, DEV)
    for t in [S_mass, *S_mom, den]:
        t.fill_(float("nan"))
    pairs = torch.full((M,), -1, dtype=torch.int32, device=DEV)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, scale=1.3, count_pairs=True)
    ctx.project_cells(ix, tr, p, S_mass, S_mom, den, injection=F.make_injection(**inj) if inj else None,
                      pairs=pairs)
    torch.cuda.synchronize()
    st = ctx.stats()
    shape = ix.shape()
    if index is None:
        ix.close()
    return (torch.stack([S_mass, *S_mom]).double().cpu().numpy(), den.double().cpu().numpy(),
            pairs.cpu().numpy().astype(np.int64), st, shape)


def _oracle(cells, wl, prec, inj=None, sel=None, traj=None):
    tr = as_precision(traj if traj is not None else wl.traj, prec)
    cs = None
    if inj:
        vol = cells.volume.numpy() if sel is None else cells.volume.numpy()[sel]
        nh = oracle.nhat_cells(vol, inj["n_ref"], inj["tau_ref"], inj["area"], inj["v_inj"], N_fla=37.0,
                               tau_fla=0.02)
        cs = np.zeros(cells.count)
        cs[np.arange(cells.count) if sel is None else sel] = nh
    return oracle.project_points(cells, tr, wl.rho_d, wl.mu, wl.delta, wl.h0, cutoff=wl.cutoff,
                                 f32_decision=(prec == "f32"), scale=1.3, cell_scale=cs, sel=sel)


def _check(ctx, cells, wl, prec, what, inj=None, per_bucket=0):
    print(f"[case] cells {what} prec={prec} M={cells.count} N={wl.traj.count}", flush=True)
    S, den, pairs, st, shape = _run(ctx, cells, wl, prec, inj, per_bucket=per_bucket)
    ref, terms = _oracle(cells, wl, prec, inj)
    assert_fields_close(S, ref.S, TOL[prec], f"cells {what} {prec}")
    assert rel_l2(den, ref.den) <= TOL[prec]
    np.testing.assert_array_equal(pairs, ref.pairs)
    assert st["pairs"] == int(ref.pairs.sum()) and st["skipped"] == terms.skipped
    return S, pairs, st, shape


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_stretched_rectilinear_mesh_with_nhat(ctx, prec):
    """A wall-clustered rectilinear mesh (tanh stretching along y, closed in
    y, periodic in x and z), n_hat from the cell volumes."""
    edges = [W.stretched_edges(21, 0.0, 1.0, 1.2), W.stretched_edges(26, 0.0, 1.0, 2.5),
             W.stretched_edges(17, 0.0, 1.0, 0.8)]
    cells = W.rectilinear_cells(edges, (True, False, True))
    wl = W.small_random_3d(3000, 8, seed=51, periodic=True, h0=0.02)
    S, pairs, st, shape = _check(ctx, cells, wl, prec, "stretched 21x26x17", inj=INJ, per_bucket=40)
    assert pairs.sum() > 0 and st["max_class"] >= 1
    assert shape[0][1] > 1 and shape[1] >= cells.count / 128


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("dim,periodic", [(3, (False, False, False)), (2, (True, True))])
def test_scattered_cells_in_their_own_order(ctx, prec, dim, periodic):
    if dim == 3:
        cells = W.scattered_cells(3, 18, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), periodic, seed=52)
        wl = W.small_random_3d(2500, 8, seed=53, periodic=False, h0=0.03)
    else:
        cells = W.scattered_cells(2, 70, (0.0, 0.0), (1.0, 1.0), periodic, seed=54)
        wl = W.taylor_green_2d(per_axis=48, mesh_n=32, seed=55)
    _check(ctx, cells, wl, prec, f"scattered {dim}-D periodic={periodic}", inj=INJ if dim == 3 else None)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lattice_centroids_take_the_cartesian_decisions(ctx, prec):
    """The centres of a Cartesian mesh, listed in a scrambled order as a
    general mesh: the same per-cell pair counts as fla_project_sources and
    the same fields within the bar."""
    from helpers import gpu_run
    wl = W.small_random_3d(4000, 20, seed=56, periodic=True, h0=0.025)
    base = W.mesh_cells(wl.mesh)
    perm = torch.argsort(W.counter_uniform(7, 1, base.count))
    cells = W.Cells(3, base.centroids[:, perm].contiguous(), base.volume[perm].contiguous(), base.lo, base.hi,
                    base.periodic)
    S, den, pairs, st, _ = _run(ctx, cells, wl, prec)
    Sc, denc, stc = gpu_run(ctx, wl, prec=prec, scale=1.3, cell_pairs=True)
    p = perm.numpy()
    np.testing.assert_array_equal(pairs, stc["cell_pairs"][p])
    assert_fields_close(S, Sc[:, p], TOL[prec], f"lattice centroids {prec}")
    assert rel_l2(den, denc[p]) <= TOL[prec]


def test_edge_cases(ctx):
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(500, 8, seed=57, periodic=False, h0=0.05)
    # one cell; a cloud with no trajectory; trajectories all outside a closed box
    one = W.Cells(3, torch.tensor([[0.5], [0.5], [0.5]], dtype=torch.float64), torch.ones(1, dtype=torch.float64),
                  (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (False, False, False))
    _check(ctx, one, wl, "f64", "one cell", inj=INJ)
    cells = W.scattered_cells(3, 10, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (False,) * 3, seed=58)
    S, den, pairs, st, _ = _run(ctx, cells, wl, "f32", traj=wl.traj.subset(torch.arange(0)))
    assert np.all(S == 0.0) and np.all(den == 0.0) and np.all(pairs == 0)
    far = wl.traj.subset(torch.arange(100))
    far.x = far.x + 3.0
    S, den, pairs, st, _ = _run(ctx, cells, wl, "f32", traj=far)
    assert np.all(S == 0.0) and st["no_support"] == 100 and st["pairs"] == 0
    # skipped trajectories (non-finite radius) agree with the oracle
    bad = wl.traj.subset(torch.arange(500))
    bad.r = bad.r.clone()
    bad.r[::7] = float("nan")
    S, den, pairs, st, _ = _run(ctx, cells, wl, "f32", traj=bad)
    ref, terms = _oracle(cells, wl, "f32", traj=bad)
    assert_fields_close(S, ref.S, TOL["f32"], "cells with skipped trajectories")
    assert st["skipped"] == terms.skipped > 0


def test_invalid_arguments(ctx):
    import paper_2512_20829_amd as F
    cells = W.scattered_cells(3, 6, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (False,) * 3, seed=59)
    bad = W.Cells(3, cells.centroids.clone(), cells.volume, cells.lo, cells.hi, cells.periodic)
    bad.centroids[1, 5] = 1.5                      # outside the box
    cs, keep = F.cells_of(bad, DEV)
    with pytest.raises(F.FlaError, match="INVALID_ARG"):
        ctx.cell_index(cs)
    nov = W.Cells(3, cells.centroids, None, cells.lo, cells.hi, cells.periodic)
    cs, keep = F.cells_of(nov, DEV)
    ix = ctx.cell_index(cs)
    wl = W.small_random_3d(200, 6, seed=60, periodic=False)
    tr, keep2 = device_traj(wl.traj, "f32")
    S_mass, S_mom, den = F.alloc_fields(cells.count, 3, torch.float32, DEV)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0)
    with pytest.raises(F.FlaError, match="volumes"):
        ctx.project_cells(ix, tr, p, S_mass, S_mom, den, injection=F.make_injection(**INJ))
    with pytest.raises(F.FlaError, match="INVALID_ARG"):
        ctx.project_cells(ix, tr, F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, mode=F.FLA_DEPOSIT),
                          S_mass, S_mom, den)
    with pytest.raises(F.FlaError, match="INVALID_ARG"):
        ctx.project_cells(ix, tr, p, S_mass, S_mom, den, injection=F.make_injection(1.0, 0.0, 1.0, 1.0))
    ctx.project_cells(ix, tr, p, S_mass, S_mom, den)   # no n_hat: fine without volumes
    torch.cuda.synchronize()
    ix.close()


@pytest.mark.timeout(300)
def test_full_size_stretched_mesh_sampled_cells(ctx):
    """2M lattice trajectories of the 128^3 ABC workload on a 128^3 mesh
    stretched along every axis (periodic; 2,097,152 cells): 256 sampled
    cells against the oracle over all trajectories, and the pair total."""
    import paper_2512_20829_amd as F
    wl = W.abc_lattice_3d()
    edges = [W.stretched_edges(128, 0.0, 1.0, 1.5) for _ in range(3)]
    cells = W.rectilinear_cells(edges, (True, True, True))
    print(f"[case] cells stretched 128^3 N={wl.traj.count}", flush=True)
    S, den, pairs, st, shape = _run(ctx, cells, wl, "f32", INJ)
    sel = np.sort(np.random.default_rng(8).choice(cells.count, 256, replace=False))
    oracle.set_threads(16)
    ref, _ = _oracle(cells, wl, "f32", INJ, sel=sel)
    assert_fields_close(S[:, sel], ref.S, TOL["f32"], "stretched 128^3 sampled")
    np.testing.assert_array_equal(pairs[sel], ref.pairs)
    assert st["pairs"] == int(pairs.sum()) and np.isfinite(S).all()
