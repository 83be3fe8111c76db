"""Batched projection of many uneven snapshots (fla_project_batch).

Each snapshot of a batch must come out bit for bit as the single-snapshot
entry point produces it under the same gather plan: the batch keys keep the
per-snapshot bucket order (the sort is stable and trajectories keep their
order inside a snapshot) and every workgroup runs the same tile body.  The
batch is also held to the oracle at the bars of the single path (1e-12 rel
L2 in binary64, 1e-5 in binary32, pair counts exact), and the captured graph
is replayed after the inputs change in place, with other library work in
between, and compared with direct launches each time."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import as_precision, assert_fields_close, device_traj, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_20829_amd as F
    c = F.Context(0)
    yield c
    c.close()


def _mesh(n, periodic, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    dim = len(n)
    return W.Mesh(dim, tuple(n), tuple(lo[:dim]), tuple(hi[:dim]), (periodic,) * dim)


def _snapshots_3d():
    """Uneven snapshots: ragged and tiny meshes, closed and periodic boxes,
    an empty snapshot, a wide-support one (whole-axis neighbourhoods) and
    one with non-finite and degenerate records."""
    out = []
    a = W.small_random_3d(3000, 20, seed=31)
    out.append(a)
    b = W.small_random_3d(12000, 33, seed=32, periodic=False)
    out.append(W.Workload("closed_ragged", _mesh((33, 21, 17), False), b.traj, b.h0, "f32"))
    e = W.small_random_3d(10, 12, seed=33)
    out.append(W.Workload("empty", _mesh((12, 12, 12), True), e.traj.subset(torch.arange(0)), e.h0, "f32"))
    out.append(W.small_random_3d(500, 40, seed=34, h0=0.08))
    out.append(W.small_random_3d(20000, 16, seed=35))
    bad = W.small_random_3d(4000, 24, seed=36)
    tr = bad.traj
    tr.x[0, 5] = float("nan")
    tr.J[:, 7] = 0.0
    tr.r[9] = float("inf")
    out.append(bad)
    out.append(W.small_random_3d(8000, 28, seed=37, amp=0.05))
    return out


def _single(ctx, wl, prec, dt, traj_struct):
    import paper_2512_20829_amd as F
    S_mass, S_mom, den = F.alloc_fields(wl.mesh.cells, wl.mesh.dim, dt, DEV)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, count_pairs=True)
    ctx.project_sources(F.mesh_of(wl.mesh), traj_struct, p, S_mass, S_mom, den)
    torch.cuda.synchronize()
    st = ctx.stats()
    return torch.stack([S_mass, *S_mom]).double().cpu().numpy(), den.double().cpu().numpy(), st


class Batch:
    """Device inputs and outputs of a batch, and its argument structs."""

    def __init__(self, wls, prec):
        import paper_2512_20829_amd as F
        self.wls, self.prec = wls, prec
        self.dt = torch.float64 if prec == "f64" else torch.float32
        self.trajs, self.keep = [], []
        for wl in wls:
            st, keep = device_traj(wl.traj, prec)
            self.trajs.append(st)
            self.keep.append(keep)
        self.outs = self.new_outs()
        self.meshes = [F.mesh_of(wl.mesh) for wl in wls]
        self.params = [F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff,
                                count_pairs=True) for wl in wls]

    def new_outs(self):
        """Output planes for every snapshot, filled with NaN (every cell must be written)."""
        import paper_2512_20829_amd as F
        outs = []
        for wl in self.wls:
            S_mass, S_mom, den = F.alloc_fields(wl.mesh.cells, wl.mesh.dim, self.dt, DEV)
            for t in [S_mass, *S_mom, den]:
                t.fill_(float("nan"))
            outs.append((S_mass, S_mom, den))
        return outs

    def run(self, ctx, outs=None):
        ctx.project_batch(self.meshes, self.trajs, self.params, outs if outs is not None else self.outs)

    def fields(self, s, outs=None):
        S_mass, S_mom, den = (outs if outs is not None else self.outs)[s]
        return torch.stack([S_mass, *S_mom]).double().cpu().numpy(), den.double().cpu().numpy()


def _assert_same_as_single(ctx, batch, stats):
    pairs = skipped = 0
    for s, wl in enumerate(batch.wls):
        print(f"[case] snapshot {s} {wl.name} N={wl.traj.count} mesh={wl.mesh.n}", flush=True)
        Sb, db = batch.fields(s)
        Ss, ds, st = _single(ctx, wl, batch.prec, batch.dt, batch.trajs[s])
        assert np.array_equal(Sb, Ss, equal_nan=False), f"snapshot {s}: fields differ from the single call"
        assert np.array_equal(db, ds), f"snapshot {s}: denominators differ"
        pairs += st["pairs"]
        skipped += st["skipped"]
    assert stats["pairs"] == pairs
    assert stats["skipped"] == skipped
    assert stats["trajectories"] == sum(wl.traj.count for wl in batch.wls)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_calls(ctx, prec, graph):
    wls = _snapshots_3d()
    b = Batch(wls, prec)
    ctx.set_batch_graph(graph)
    try:
        b.run(ctx)
        torch.cuda.synchronize()
        st = ctx.stats()
        assert st["skipped"] == 3
        _assert_same_as_single(ctx, b, st)
    finally:
        ctx.set_batch_graph(True)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_matches_oracle(ctx, prec):
    wls = [W.small_random_3d(2500, 18, seed=41), W.small_random_3d(6000, 25, seed=42, periodic=False),
           W.small_random_3d(900, 30, seed=43, h0=0.05)]
    b = Batch(wls, prec)
    b.run(ctx)
    torch.cuda.synchronize()
    st = ctx.stats()
    pairs = 0
    for s, wl in enumerate(wls):
        S, den = b.fields(s)
        ref, _ = oracle_run(wl, prec=prec)
        assert_fields_close(S, ref.S, TOL[prec], f"batch snapshot {s}")
        assert rel_l2(den, ref.den) <= TOL[prec]
        pairs += int(ref.pairs.sum())
    assert st["pairs"] == pairs


def test_batch_2d(ctx):
    wls = [W.taylor_green_2d(), W.taylor_green_2d()]
    wls[1] = W.Workload("tg_small_h", wls[1].mesh, wls[1].traj, wls[1].h0 * 0.5, "f64")
    b = Batch(wls, "f64")
    b.run(ctx)
    torch.cuda.synchronize()
    for s, wl in enumerate(wls):
        S, den = b.fields(s)
        ref, _ = oracle_run(wl, prec="f64")
        assert_fields_close(S, ref.S, TOL["f64"], f"2-D batch snapshot {s}")


def test_graph_replays_follow_input_changes(ctx):
    """Replays of the captured graph see buffer contents written in place, and
    other calls that reuse the workspace between replays do not disturb them;
    a second context without graphs gives the reference of every replay."""
    import paper_2512_20829_amd as F
    wls = _snapshots_3d()[:5]
    b = Batch(wls, "f32")
    ctx.set_batch_graph(True)
    direct_ctx = F.Context(0)
    direct_ctx.set_batch_graph(False)
    other = W.small_random_3d(30000, 40, seed=44)
    ost, okeep = device_traj(other.traj, "f32")
    replays0 = ctx.stats()["graph_replays"]
    try:
        for rep in range(4):
            print(f"[case] replay {rep}", flush=True)
            if rep > 0:
                # change the inputs in place: radii scaled, positions along axis 0 shifted
                for s, keep in enumerate(b.keep):
                    if b.wls[s].traj.count == 0:
                        continue
                    x0, r = keep[0], keep[10]     # make_trajectories keeps x, v, ug rows, then J, r
                    r.mul_(1.0 + 0.1 * rep)
                    x0.copy_(torch.remainder(x0 + 0.013 * rep, 1.0))
            b.run(ctx)
            # unrelated work on the same context between replays (reuses the workspace)
            _single(ctx, other, "f32", torch.float32, ost)
            direct = b.new_outs()
            b.run(direct_ctx, direct)
            torch.cuda.synchronize()
            for s in range(len(wls)):
                Sg, dg = b.fields(s)
                Se, de = b.fields(s, direct)
                assert np.array_equal(Sg, Se) and np.array_equal(dg, de), f"replay {rep} snapshot {s}"
        assert ctx.stats()["graph_replays"] == replays0 + 3
        assert direct_ctx.stats()["graph_replays"] == 0
    finally:
        direct_ctx.close()


def test_autotune_batch(ctx):
    import paper_2512_20829_amd as F
    b = Batch(_snapshots_3d(), "f32")
    times = ctx.autotune_batch(b.meshes, b.trajs, b.params, b.outs)
    assert len(times) == F.GATHER_CONFIGS * F.BATCH_CHUNKS and all(t > 0 for t in times)
    plan, chunk = ctx.get_batch_plan(3, F.FLA_F32)
    k = int(np.argmin(times))
    assert plan == k // F.BATCH_CHUNKS and chunk == [1, 4, 16, 64][k % F.BATCH_CHUNKS]
    b.run(ctx)
    torch.cuda.synchronize()
    _assert_same_as_single_plan(ctx, b, plan)
    ctx.set_batch_plan(3, F.FLA_F32, -1, 0)
    assert ctx.get_batch_plan(3, F.FLA_F32) == (1, 16)


@pytest.mark.parametrize("code", [1, 5])
def test_batch_equals_single_calls_under_each_shape(ctx, code):
    """Half tiles (code 1) and whole tiles (code 5, plan 1): every snapshot of
    the batch equals its single call under the same plan code."""
    import paper_2512_20829_amd as F
    print(f"[case] batch plan code {code}", flush=True)
    b = Batch(_snapshots_3d(), "f32")
    ctx.set_batch_graph(False)
    ctx.set_batch_plan(3, F.FLA_F32, code, 4)
    try:
        b.run(ctx)
        torch.cuda.synchronize()
        _assert_same_as_single_plan(ctx, b, code)
    finally:
        ctx.set_batch_plan(3, F.FLA_F32, -1, 0)


def _assert_same_as_single_plan(ctx, b, plan):
    import paper_2512_20829_amd as F
    ctx.set_plan(3, F.FLA_F32, plan)
    try:
        for s, wl in enumerate(b.wls):
            Sb, db = b.fields(s)
            Ss, ds, _ = _single(ctx, wl, "f32", torch.float32, b.trajs[s])
            assert np.array_equal(Sb, Ss) and np.array_equal(db, ds)
    finally:
        ctx.set_plan(3, F.FLA_F32, -1)


def test_batch_rejects_bad_arguments(ctx):
    import paper_2512_20829_amd as F
    wls = [W.small_random_3d(100, 8, seed=45), W.small_random_3d(100, 8, seed=46)]
    b = Batch(wls, "f32")
    # deposition mode is not batched
    b.params[1].mode = F.FLA_DEPOSIT
    with pytest.raises(F.FlaError, match="snapshot 1"):
        b.run(ctx)
    b.params[1].mode = F.FLA_NW
    # mixed precisions
    st64, keep64 = device_traj(wls[1].traj, "f64")
    with pytest.raises(F.FlaError, match="same prec"):
        ctx.project_batch(b.meshes, [b.trajs[0], st64], b.params, b.outs)
    # mixed dimensions
    tg = W.taylor_green_2d()
    with pytest.raises(F.FlaError, match="same mesh.dim"):
        ctx.project_batch([b.meshes[0], F.mesh_of(tg.mesh)], b.trajs, b.params, b.outs)
    # an invalid h0 names its snapshot
    b.params[0].h0 = -1.0
    with pytest.raises(F.FlaError, match="snapshot 0"):
        b.run(ctx)
    b.params[0].h0 = wls[0].h0
    b.run(ctx)
    torch.cuda.synchronize()


@pytest.mark.slow
@pytest.mark.timeout(400)
def test_uneven_batch_full_size_sampled(ctx):
    """The 64-snapshot uneven batch (meshes 32^3..128^3, 10k..2M trajectories,
    about 24M in all) in the launch form the benchmark times, checked against
    the oracle on sampled cells of every snapshot."""
    import paper_2512_20829_amd as F
    wls = [W.uneven_snapshot(s, device=DEV) for s in range(64)]
    b = Batch(wls, "f32")
    print(f"[case] c3 batch N={sum(w.traj.count for w in wls)} cells={sum(w.mesh.cells for w in wls)}", flush=True)
    b.run(ctx)
    b.run(ctx)          # second call replays the captured graph
    torch.cuda.synchronize()
    st = ctx.stats()
    assert st["trajectories"] == sum(w.traj.count for w in wls)
    assert st["skipped"] == 0
    g = torch.Generator().manual_seed(7)
    worst = 0.0
    for s, wl in enumerate(wls):
        S, den = b.fields(s)
        assert np.isfinite(S).all()
        cells = torch.randint(0, wl.mesh.cells, (12,), generator=g).numpy()
        tr = wl.traj.to("cpu")
        ref, _ = oracle.project(wl.mesh, as_precision(tr, "f32"), wl.rho_d, wl.mu, wl.delta, wl.h0,
                                cutoff=wl.cutoff, f32_decision=True, cells=cells)
        for k in range(S.shape[0]):
            got, exp = S[k][cells], ref.S[k]
            scale = np.abs(exp).max()
            if scale == 0.0:
                assert np.all(got == 0.0)
                continue
            err = np.abs(got - exp).max() / scale
            worst = max(worst, err)
            assert err <= 1e-5, f"snapshot {s} field {k}: sampled max rel error {err:.2e}"
        dref = ref.den
        assert np.abs(den[cells] - dref).max() <= 1e-5 * max(np.abs(dref).max(), 1e-300)
    print(f"[uneven snapshots] worst sampled relative error {worst:.2e}", flush=True)
