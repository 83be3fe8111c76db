"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: binary64 path within 1e-12 relative L2 per source field, binary32
path within 1e-5 (the targets stated for the two precisions); pair counts,
skip counts and PSI-CELL particle counts bit-exact (both sides take the
inclusion decision in the same precision)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import assert_fields_close, gpu_run, oracle_run, rel_l2, as_precision

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_20829_amd as F
    c = F.Context(0)
    yield c
    c.close()


def _check(ctx, wl, prec=None, **kw):
    prec = prec or wl.precision
    print(f"[case] {wl.name} prec={prec} N={wl.traj.count} mesh={wl.mesh.n} periodic={wl.mesh.periodic}",
          flush=True)
    S, den, st = gpu_run(ctx, wl, prec=prec, cell_pairs=True, **kw)
    okw = {k: v for k, v in kw.items() if k in ("scale", "cell_scale", "h_factor")}
    ref, terms = oracle_run(wl, prec=prec, **okw)
    assert_fields_close(S, ref.S, TOL[prec], wl.name)
    assert rel_l2(den, ref.den) <= TOL[prec]
    assert st["pairs"] == int(ref.pairs.sum())
    np.testing.assert_array_equal(st["cell_pairs"], ref.pairs)
    assert st["skipped"] == terms.skipped
    assert st["trajectories"] == wl.traj.count
    return S, den, st, ref


def test_taylor_green_2d_f64(ctx):
    wl = W.taylor_green_2d()
    S, den, st, ref = _check(ctx, wl, "f64")
    assert (ref.den > 0).all()


def test_taylor_green_non_evaporating(ctx):
    wl = W.taylor_green_2d(delta=0.0)
    S, _, _, _ = _check(ctx, wl, "f64")
    assert np.all(S[0] == 0.0)


def test_2d_f32_small(ctx):
    wl = W.taylor_green_2d(per_axis=40, mesh_n=37)
    _check(ctx, wl, "f32")


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_3d_random_ragged(ctx, periodic, prec):
    wl = W.small_random_3d(3000, 19, seed=3, periodic=periodic)
    wl.mesh = W.Mesh(3, (21, 19, 17), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (periodic,) * 3)
    _check(ctx, wl, prec)


def test_3d_positions_outside_closed_box(ctx):
    wl = W.small_random_3d(2000, 16, seed=4, periodic=False)
    wl.traj.x = wl.traj.x * 1.3 - 0.15          # some trajectories sit outside [0,1)^3
    wl.mesh = W.Mesh(3, (16, 16, 16), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (False,) * 3)
    _, _, st, _ = _check(ctx, wl, "f32")
    assert st["no_support"] > 0


def test_large_bandwidth_spans_whole_axes(ctx):
    wl = W.small_random_3d(500, 24, seed=5, periodic=True, h0=0.12)
    _, _, st, _ = _check(ctx, wl, "f32")
    assert st["max_class"] >= 2


def test_tiny_bandwidth(ctx):
    wl = W.small_random_3d(4000, 20, seed=6, periodic=True, h0=0.01)
    _check(ctx, wl, "f32")


def test_degenerate_trajectories_are_skipped(ctx):
    wl = W.small_random_3d(1500, 12, seed=7)
    J = wl.traj.J.clone()
    J[:, 0:10] = 0.0                          # det J = 0
    J[0, 10:20] = float("nan")                # non-finite
    wl.traj.J = J
    wl.traj.r = wl.traj.r.clone()
    wl.traj.r[20:25] = float("inf")
    _, _, st, _ = _check(ctx, wl, "f32")
    assert st["skipped"] == 25


def test_scale_cell_scale_and_bandwidth_factor(ctx):
    wl = W.small_random_3d(2000, 16, seed=8)
    cs = torch.linspace(0.5, 1.5, wl.mesh.cells, dtype=torch.float64)
    g = torch.Generator().manual_seed(1)
    hf = torch.exp(0.5 * (torch.rand(wl.traj.count, generator=g) - 0.5)).to(torch.float32)
    _check(ctx, wl, "f32", scale=2.5, cell_scale=cs.numpy(), h_factor=hf)
    _check(ctx, wl, "f64", scale=2.5, cell_scale=cs.numpy(), h_factor=hf)


def test_zero_trajectories_writes_zeros(ctx):
    wl = W.small_random_3d(10, 8, seed=9)
    wl.traj = wl.traj.subset(torch.arange(0))
    S, den, st = gpu_run(ctx, wl, prec="f32")
    assert np.all(S == 0.0) and np.all(den == 0.0)


def test_bitwise_deterministic(ctx):
    wl = W.small_random_3d(20000, 32, seed=10)
    S1, d1, _ = gpu_run(ctx, wl, prec="f32", count_pairs=False)
    S2, d2, _ = gpu_run(ctx, wl, prec="f32", count_pairs=False)
    assert np.array_equal(S1, S2) and np.array_equal(d1, d2)


def test_abc_full_size_whole_field(ctx):
    """The 128^3 / 2M-trajectory ABC case in the launch configuration the
    benchmark times, on every one of its 2,097,152 cells against the
    trajectory-centric oracle: per-field relative L2 and per-cell errors
    within 1e-5, and the included pairs of every cell exactly."""
    wl = W.abc_lattice_3d()
    S, den, st = gpu_run(ctx, wl, prec="f32", count_pairs=False, cell_pairs=True)
    oracle.set_threads(16)
    tr = as_precision(wl.traj, "f32")
    ref, terms = oracle.project_box(wl.mesh, tr, wl.rho_d, wl.mu, wl.delta, wl.h0, cutoff=wl.cutoff,
                                    f32_decision=True)
    np.testing.assert_array_equal(ref.cells, np.arange(wl.mesh.cells))
    assert_fields_close(S, ref.S, TOL["f32"], "abc 128^3 whole field")
    assert rel_l2(den, ref.den) <= TOL["f32"]
    np.testing.assert_array_equal(st["cell_pairs"], ref.pairs)
    assert st["pairs"] == int(ref.pairs.sum()) and st["skipped"] == 0


def test_abc_full_size_against_binary64_decisions(ctx):
    """The binary32 path against the pure binary64 definition (inclusion
    decided in binary64 too) on 16 planes of the 128^3 case: the boundary
    pairs that binary32 rounding flips change the fields by far less than
    the 1e-5 bar."""
    wl = W.abc_lattice_3d()
    S, den, st = gpu_run(ctx, wl, prec="f32", count_pairs=False, cell_pairs=True)
    oracle.set_threads(16)
    tr = as_precision(wl.traj, "f32")
    ref, _ = oracle.project_box(wl.mesh, tr, wl.rho_d, wl.mu, wl.delta, wl.h0, cutoff=wl.cutoff,
                                f32_decision=False, box_lo=[0, 0, 56], box_n=[128, 128, 16])
    flips = int(np.abs(st["cell_pairs"][ref.cells] - ref.pairs).sum())
    errs = [rel_l2(S[k, ref.cells], ref.S[k]) for k in range(4)]
    print(f"[f64-decision] rel L2 {' '.join(f'{e:.2e}' for e in errs)}; pair-count differences {flips} "
          f"of {int(ref.pairs.sum())}", flush=True)
    assert_fields_close(S[:, ref.cells], ref.S, TOL["f32"], "abc 128^3 vs binary64 decisions")


@pytest.mark.slow
@pytest.mark.timeout(400)
def test_multi_vortex_full_size_wrapped_block(ctx):
    """The 256^3 / 32.8M-trajectory multi-vortex case (|det J| down to ~1e-8,
    sign changes) in the benchmark's launch configuration, on a whole 32^3
    block of cells that straddles the periodic boundary on every axis,
    against the trajectory-centric oracle over all trajectories."""
    dev = torch.device("cuda", 0)
    wl = W.multi_vortex_lattice_3d(device=dev)
    wl.traj = wl.traj.to("cpu")
    print(f"[case] c5 N={wl.traj.count} mesh={wl.mesh.n}", flush=True)
    S, den, st = gpu_run(ctx, wl, prec="f32", count_pairs=False, cell_pairs=True)
    assert np.isfinite(S).all()
    oracle.set_threads(16)
    tr = as_precision(wl.traj, "f32")
    ref, terms = oracle.project_box(wl.mesh, tr, wl.rho_d, wl.mu, wl.delta, wl.h0, cutoff=wl.cutoff,
                                    f32_decision=True, box_lo=[240, 244, 248], box_n=[32, 32, 32])
    assert (ref.cells % 256 < 16).any() and (ref.cells % 256 >= 240).any()
    assert_fields_close(S[:, ref.cells], ref.S, TOL["f32"], "multi-vortex wrapped 32^3 block")
    assert rel_l2(den[ref.cells], ref.den) <= TOL["f32"]
    np.testing.assert_array_equal(st["cell_pairs"][ref.cells], ref.pairs)
    assert st["skipped"] == terms.skipped
    assert 7 <= st["max_class"] <= 15    # wide bandwidths reach seven tiles and more


# ------------------------------------------------------------------ deposition
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_deposit_matches_oracle_and_conserves(ctx, prec):
    wl = W.small_random_3d(1500, 14, seed=11, periodic=True)
    S, den, st = gpu_run(ctx, wl, prec=prec, mode=1)
    tr = as_precision(wl.traj, prec)
    t = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
    Sref, Z = oracle.deposit(wl.mesh, tr.x, t, tr.seed_volume, f32_decision=(prec == "f32"))
    assert_fields_close(S, Sref, TOL[prec], "deposit")
    Q = t.q * tr.seed_volume * np.abs(t.det)
    tot = S.sum(axis=1) * wl.mesh.cell_volume
    np.testing.assert_allclose(tot, -Q.sum(axis=1), rtol=TOL[prec] * 10)
    assert st["zero_support"] == int((Z[t.valid == 1] == 0).sum())


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_deposit_wide_supports_span_several_blocks(ctx, prec, periodic):
    # h0 = 0.15 on 70^3 cells: supports of 2 c h |det J| ~ 80 cells per axis
    # and more, wider than the normaliser's 64-cell blocks (the whole axis
    # on a periodic mesh, clipped at the walls of a closed one)
    print(f"[case] deposit wide supports {prec} periodic={periodic}", flush=True)
    wl = W.small_random_3d(200, 70, seed=17, periodic=periodic, h0=0.15)
    S, den, st = gpu_run(ctx, wl, prec=prec, mode=1)
    tr = as_precision(wl.traj, prec)
    t = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
    Sref, Z = oracle.deposit(wl.mesh, tr.x, t, tr.seed_volume, f32_decision=(prec == "f32"))
    assert_fields_close(S, Sref, TOL[prec], "deposit wide")
    assert st["zero_support"] == int((Z[t.valid == 1] == 0).sum())


def test_deposit_zero_support_goes_home(ctx):
    wl = W.small_random_3d(800, 12, seed=12, periodic=False, h0=0.004)
    S, _, st = gpu_run(ctx, wl, prec="f64", mode=1)
    tr = wl.traj
    t = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
    Sref, Z = oracle.deposit(wl.mesh, tr.x, t, tr.seed_volume)
    assert st["zero_support"] > 0 and st["zero_support"] == int((Z[t.valid == 1] == 0).sum())
    assert_fields_close(S, Sref, TOL["f64"], "deposit delta")


# ------------------------------------------------------------------ PSI-CELL
def test_psicell_taylor_green_cloud_f64(ctx):
    wl = W.taylor_green_2d()
    cloud = W.taylor_green_cloud()
    w = W.N0_DEFAULT / cloud.count
    S, den, st = gpu_run(ctx, wl, prec="f64", psicell_cloud=cloud, weight=w)
    Sref, counts, out, nf = oracle.psicell(wl.mesh, cloud, w, wl.rho_d, wl.mu, wl.delta, split=True)
    assert_fields_close(S, Sref, TOL["f64"], "psicell f64")
    assert np.array_equal(den.astype(np.int64), counts)
    assert st["outside"] == out and st["skipped"] == nf


def test_psicell_3d_f32_with_outside_particles(ctx):
    wl = W.small_random_3d(10, 23, seed=13, periodic=False)
    cloud = W.abc_cloud(300_000, seed=13)
    cloud.x = cloud.x * 1.1 - 0.05
    w = 3.0
    S, den, st = gpu_run(ctx, wl, prec="f32", psicell_cloud=cloud, weight=w)
    c64 = as_precision(cloud, "f32")
    Sref, counts, out, nf = oracle.psicell(wl.mesh, c64, w, wl.rho_d, wl.mu, wl.delta, split=True)
    assert_fields_close(S, Sref, TOL["f32"], "psicell f32")
    assert np.array_equal(den.astype(np.int64), counts)
    assert st["outside"] == out and out > 0 and st["skipped"] == nf == 0


def test_psicell_deterministic(ctx):
    wl = W.small_random_3d(10, 32, seed=14, periodic=True)
    cloud = W.abc_cloud(500_000, seed=14)
    S1, _, _ = gpu_run(ctx, wl, prec="f32", psicell_cloud=cloud, weight=1.0)
    S2, _, _ = gpu_run(ctx, wl, prec="f32", psicell_cloud=cloud, weight=1.0)
    assert np.array_equal(S1, S2)


def test_psicell_without_the_count_plane_gives_the_same_fields(ctx):
    # the per-cell counts are an optional output; leaving them out must not
    # change the source fields
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(10, 40, seed=23, periodic=True)
    cloud = W.abc_cloud(400_000, seed=23)
    S1, _, _ = gpu_run(ctx, wl, prec="f32", psicell_cloud=cloud, weight=2.0)
    dev = torch.device("cuda", 0)
    st, _ = F.make_trajectories(cloud.x.to(dev).contiguous(), None, cloud.v.to(dev, torch.float32).contiguous(),
                                cloud.ug.to(dev, torch.float32).contiguous(),
                                cloud.r.to(dev, torch.float32).contiguous(), 1.0)
    Sm, Sv, _ = F.alloc_fields(wl.mesh.cells, 3, torch.float32, dev)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
    ctx.psicell_accumulate(F.mesh_of(wl.mesh), st, 2.0, p, Sm, Sv)
    torch.cuda.synchronize()
    S2 = torch.stack([Sm, *Sv]).double().cpu().numpy()
    assert np.array_equal(S1, S2)


def test_psicell_edge_cases(ctx):
    wl = W.small_random_3d(10, 12, seed=24, periodic=False)
    base = W.abc_cloud(1000, seed=24)
    # no particle: zero fields and counts
    S, den, st = gpu_run(ctx, wl, prec="f32", psicell_cloud=base.subset(torch.arange(0)), weight=1.0)
    assert np.all(S == 0.0) and np.all(den == 0.0) and st["outside"] == 0
    # every particle outside the closed box
    out = W.Trajectories(base.x + 2.0, base.J, base.v, base.ug, base.r, 1.0)
    S, den, st = gpu_run(ctx, wl, prec="f32", psicell_cloud=out, weight=1.0)
    assert np.all(S == 0.0) and np.all(den == 0.0) and st["outside"] == 1000
    # every record skipped (non-finite radius): no cell receives anything
    bad = W.Trajectories(base.x, base.J, base.v, base.ug, torch.full_like(base.r, float("nan")), 1.0)
    S, den, st = gpu_run(ctx, wl, prec="f32", psicell_cloud=bad, weight=1.0)
    assert np.all(S == 0.0) and np.all(den == 0.0) and st["skipped"] == 1000 and st["outside"] == 0
    # non-finite positions are skipped too, not outside
    nanx = W.Trajectories(base.x.clone(), base.J, base.v, base.ug, base.r, 1.0)
    nanx.x[1, ::10] = float("nan")
    S, den, st = gpu_run(ctx, wl, prec="f32", psicell_cloud=nanx, weight=1.0)
    assert st["skipped"] == 100 and st["outside"] == 0 and int(den.sum()) == 900
    # one particle, with a cell scale
    one = base.subset(torch.arange(1))
    cs = np.linspace(0.5, 1.5, wl.mesh.cells)
    S, den, st = gpu_run(ctx, wl, prec="f64", psicell_cloud=one, weight=3.0, cell_scale=cs)
    Sref, counts, sk = oracle.psicell(wl.mesh, one, 3.0, wl.rho_d, wl.mu, wl.delta, cell_scale=cs)
    assert_fields_close(S, Sref, TOL["f64"], "psicell one particle")
    assert np.array_equal(den.astype(np.int64), counts) and counts.sum() == 1


@pytest.mark.timeout(300)
def test_psicell_full_size_sampled_cells(ctx):
    """PSI-CELL over 200M particles on the 128^3 periodic mesh, launched as
    the benchmark launches it.  Every particle is counted once, and 256
    sampled cells match the oracle run over the particles in and next to
    them (a cell's sums depend only on its own particles)."""
    import paper_2512_20829_amd as F
    dev = torch.device("cuda", 0)
    wl = W.abc_lattice_3d(per_axis=8)      # mesh and physical constants of the 128^3 case
    n = wl.mesh.n[0]
    Np = 200_000_000
    print(f"[case] psicell N={Np} mesh={wl.mesh.n}", flush=True)
    cl = W.abc_cloud(Np, seed=0, device=dev, jacobian=False)
    v, ug, r = (cl.v.to(torch.float32).contiguous(), cl.ug.to(torch.float32).contiguous(),
                cl.r.to(torch.float32).contiguous())
    st, _ = F.make_trajectories(cl.x.contiguous(), None, v, ug, r, 1.0)
    M = wl.mesh.cells
    Sm, Sv, den = F.alloc_fields(M, 3, torch.float32, dev)
    w = W.N0_DEFAULT / Np
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
    ctx.psicell_accumulate(F.mesh_of(wl.mesh), st, w, p, Sm, Sv, den)
    torch.cuda.synchronize()
    stats = ctx.stats()
    assert int(den.double().sum().item()) == Np - stats["outside"]
    S = torch.stack([Sm, *Sv]).double().cpu().numpy()
    g = np.random.default_rng(2)
    cells = np.sort(g.choice(M, 256, replace=False))
    # particles whose cell lies within one cell of a sampled cell on every axis
    near = torch.zeros((n, n, n), dtype=torch.bool, device=dev)      # [z, y, x]
    c = torch.as_tensor(cells, device=dev)
    cz, cy, cx = c // (n * n), (c // n) % n, c % n
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                near[(cz + dz) % n, (cy + dy) % n, (cx + dx) % n] = True
    ix = torch.floor(cl.x * n).to(torch.int64) % n
    pick = near[ix[2], ix[1], ix[0]]
    del ix
    sub = W.Trajectories(cl.x[:, pick].cpu(), torch.empty(0, dtype=torch.float64),
                         v[:, pick].double().cpu(), ug[:, pick].double().cpu(), r[pick].double().cpu(), 1.0)
    print(f"[case] psicell oracle over {sub.count} particles near the sampled cells", flush=True)
    Sref, counts, _ = oracle.psicell(wl.mesh, sub, w, wl.rho_d, wl.mu, wl.delta)
    assert_fields_close(S[:, cells], Sref[:, cells], TOL["f32"], "psicell 200M sampled")
    assert np.array_equal(den[cells].cpu().numpy().astype(np.int64), counts[cells])


@pytest.mark.timeout(300)
def test_psicell_binary64_100m_particles_sampled_cells(ctx):
    """Binary64 PSI-CELL over 100M particles on a 96^3 periodic mesh (about
    113 particles per cell): the per-particle quantisation error must not
    grow with the count, so 256 sampled cells match the oracle, run over the
    particles in and next to them, within 1e-12."""
    import paper_2512_20829_amd as F
    dev = torch.device("cuda", 0)
    wl = W.small_random_3d(10, 96, seed=26, periodic=True)
    n = wl.mesh.n[0]
    Np = 100_000_000
    print(f"[case] psicell f64 N={Np} mesh={wl.mesh.n}", flush=True)
    cl = W.abc_cloud(Np, seed=26, device=dev, jacobian=False)
    st, _ = F.make_trajectories(cl.x.contiguous(), None, cl.v.contiguous(), cl.ug.contiguous(),
                               cl.r.contiguous(), 1.0)
    M = wl.mesh.cells
    Sm, Sv, den = F.alloc_fields(M, 3, torch.float64, dev)
    w = W.N0_DEFAULT / Np
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
    ctx.psicell_accumulate(F.mesh_of(wl.mesh), st, w, p, Sm, Sv, den)
    torch.cuda.synchronize()
    stats = ctx.stats()
    assert int(den.sum().item()) == Np and stats["outside"] == 0 and stats["skipped"] == 0
    S = torch.stack([Sm, *Sv]).cpu().numpy()
    g = np.random.default_rng(3)
    cells = np.sort(g.choice(M, 256, replace=False))
    near = torch.zeros((n, n, n), dtype=torch.bool, device=dev)      # [z, y, x]
    c = torch.as_tensor(cells, device=dev)
    cz, cy, cx = c // (n * n), (c // n) % n, c % n
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                near[(cz + dz) % n, (cy + dy) % n, (cx + dx) % n] = True
    ix = torch.floor(cl.x * n).to(torch.int64) % n
    pick = near[ix[2], ix[1], ix[0]]
    del ix
    sub = W.Trajectories(cl.x[:, pick].cpu(), torch.empty(0, dtype=torch.float64), cl.v[:, pick].cpu(),
                         cl.ug[:, pick].cpu(), cl.r[pick].cpu(), 1.0)
    print(f"[case] psicell f64 oracle over {sub.count} particles near the sampled cells", flush=True)
    Sref, counts, _ = oracle.psicell(wl.mesh, sub, w, wl.rho_d, wl.mu, wl.delta)
    assert_fields_close(S[:, cells], Sref[:, cells], TOL["f64"], "psicell f64 100M sampled")
    assert np.array_equal(den[cells].cpu().numpy().astype(np.int64), counts[cells])


@pytest.mark.parametrize("n", [100, 160])
def test_psicell_many_bins_with_skipped_records_f32(ctx, n):
    # 100^3 cells: 7^3 = 343 tiles of 16^3 cells with partial tiles on every
    # axis, few enough to be the scatter's bins (no tile pass); 160^3 cells
    # would take 1000 such tiles, so the two partitions run: 10 x 20 x 20 =
    # 4000 tiles of 16 x 8 x 8 cells in 63 bins of 64 with a partial last bin.
    # Particles outside the closed box and records with non-finite velocity
    # or radius are spread over all of them
    print(f"[case] psicell many bins f32 n={n}", flush=True)
    wl = W.small_random_3d(10, n, seed=21, periodic=False)
    cloud = W.abc_cloud(2_000_000, seed=21)
    cloud.x = cloud.x * 1.1 - 0.05
    cloud.r[::997] = float("nan")
    cloud.v[1, 5::1013] = float("inf")
    w = 0.5
    S, den, st = gpu_run(ctx, wl, prec="f32", psicell_cloud=cloud, weight=w)
    c64 = as_precision(cloud, "f32")
    Sref, counts, out, nf = oracle.psicell(wl.mesh, c64, w, wl.rho_d, wl.mu, wl.delta, split=True)
    assert_fields_close(S, Sref, TOL["f32"], "psicell many bins f32")
    assert np.array_equal(den.astype(np.int64), counts)
    assert st["outside"] == out and out > 4000 and st["skipped"] == nf and nf > 2000


def test_psicell_direct_tiles_3d_f64(ctx):
    # binary64 3-D: 80^3 cells are 5 x 5 x 10 = 250 tiles of 16 x 16 x 8
    # cells (two-word sums, 136 KiB of LDS per tile), the scatter's bins
    # themselves; ragged last tiles on x and y, particles outside the closed
    # box and non-finite records throughout
    print("[case] psicell direct tiles 3-D f64 n=80", flush=True)
    wl = W.small_random_3d(10, 80, seed=23, periodic=False)
    cloud = W.abc_cloud(2_000_000, seed=23)
    cloud.x = cloud.x * 1.1 - 0.05
    cloud.r[::1009] = float("nan")
    w = 0.25
    S, den, st = gpu_run(ctx, wl, prec="f64", psicell_cloud=cloud, weight=w)
    Sref, counts, out, nf = oracle.psicell(wl.mesh, cloud, w, wl.rho_d, wl.mu, wl.delta, split=True)
    assert_fields_close(S, Sref, TOL["f64"], "psicell direct 3-D f64")
    assert np.array_equal(den.astype(np.int64), counts)
    assert st["outside"] == out and out > 0 and st["skipped"] == nf and nf > 1000


@pytest.mark.parametrize("mesh_n", [1000, 1500])
def test_psicell_many_bins_2d_f64(ctx, mesh_n):
    # binary64 2-D: 1000^2 cells are 16 x 32 = 512 tiles of 64 x 32 cells,
    # the scatter's bins themselves; 1500^2 cells would take 24 x 47 = 1128
    # such tiles, so the two partitions run over 47^2 = 2209 tiles of 32^2
    # cells in 35 bins
    print(f"[case] psicell many bins 2-D f64 n={mesh_n}", flush=True)
    wl = W.taylor_green_2d(per_axis=8, mesh_n=mesh_n)
    cloud = W.taylor_green_cloud(3_000_000, seed=22)
    w = W.N0_DEFAULT / cloud.count
    S, den, st = gpu_run(ctx, wl, prec="f64", psicell_cloud=cloud, weight=w)
    Sref, counts, out, nf = oracle.psicell(wl.mesh, cloud, w, wl.rho_d, wl.mu, wl.delta, split=True)
    assert_fields_close(S, Sref, TOL["f64"], "psicell many bins f64")
    assert np.array_equal(den.astype(np.int64), counts)
    assert st["outside"] == out and st["skipped"] == nf


# ------------------------------------------------------------------ plans / autotuner
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_every_gather_plan_gives_the_same_values(ctx, prec):
    """Plan codes plan + 4 * shape: under one shape (half tiles, whole tiles)
    every plan gives the same bits; between shapes binary64 gives the same
    bits and binary32 the same decisions with sums folded at other points."""
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(6000, 30, seed=15)
    pr = F.FLA_F64 if prec == "f64" else F.FLA_F32
    outs = []
    for code in range(F.GATHER_CONFIGS):
        print(f"[case] plan code {code} {prec}", flush=True)
        ctx.set_plan(3, pr, code)
        assert ctx.get_plan(3, pr) == code
        S, den, st = gpu_run(ctx, wl, prec=prec, cell_pairs=True)
        outs.append((S, den, st["pairs"], st["cell_pairs"]))
    ctx.set_plan(3, pr, -1)
    for code, (S, den, P, cp) in enumerate(outs):
        base = outs[code - code % F.GATHER_PLANS]
        assert np.array_equal(S, base[0]) and np.array_equal(den, base[1]) and P == base[2]
        np.testing.assert_array_equal(cp, outs[0][3])
        if prec == "f64":
            assert np.array_equal(S, outs[0][0]) and np.array_equal(den, outs[0][1])
        else:
            assert_fields_close(S, outs[0][0], 1e-6, f"shape of code {code}")
    ref, _ = oracle_run(wl, prec=prec)
    for code in (0, F.GATHER_PLANS):
        assert_fields_close(outs[code][0], ref.S, TOL[prec], f"plan code {code}")
    # 2-D has whole tiles only: codes 0..3
    with pytest.raises(F.FlaError, match="INVALID_ARG"):
        ctx.set_plan(2, pr, F.GATHER_PLANS)
    ctx.set_plan(2, pr, F.GATHER_PLANS - 1)
    ctx.set_plan(2, pr, -1)


def test_autotune_picks_a_plan(ctx):
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(20000, 32, seed=16)
    dev = torch.device("cuda", 0)
    tr = wl.traj
    st, keep = F.make_trajectories(tr.x.to(dev), tr.J.to(dev), tr.v.to(dev, torch.float32),
                                   tr.ug.to(dev, torch.float32), tr.r.to(dev, torch.float32), tr.n0,
                                   tr.seed_volume)
    S, Sm, den = F.alloc_fields(wl.mesh.cells, 3, torch.float32, dev)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
    times = ctx.autotune(F.mesh_of(wl.mesh), st, p, S, Sm, den)
    assert len(times) == F.GATHER_CONFIGS and all(t > 0 for t in times)
    assert ctx.get_plan(3, F.FLA_F32) == int(np.argmin(times))
    ctx.set_plan(3, F.FLA_F32, -1)
