"""Training step of the learned bandwidth on the GPU: the loss decreases on
the training snapshots and, on held-out snapshots of other ABC maps, the
trained network does better than the plain rule; checkpoint/resume
reproduces an uninterrupted run bit for bit (all reductions are in a fixed
order)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def setup():
    import paper_2512_20829_amd as F
    from paper_2512_20829_amd import train as T
    ctx = F.Context(0)
    snaps = []
    for s in range(6):
        wl, abc = W.training_snapshot(s, n_traj=6000, mesh_n=16, device=DEV)
        tr = wl.traj
        st, keep = F.make_trajectories(tr.x, tr.J, tr.v.float(), tr.ug.float(), tr.r.float(), tr.n0, tr.seed_volume)
        keep.append(tr)
        p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
        cl = W.abc_cloud(600_000, seed=10_000 + s, device=DEV, abc=abc, jacobian=False)
        cst, ck = F.make_trajectories(cl.x, None, cl.v.float(), cl.ug.float(), cl.r.float(), 1.0)
        Sm, Sv, _ = F.alloc_fields(wl.mesh.cells, 3, torch.float32, DEV, den=False)
        ctx.psicell_accumulate(F.mesh_of(wl.mesh), cst, W.N0_DEFAULT / cl.count, p, Sm, Sv)
        snaps.append(T.Snapshot(wl.mesh, st, keep, tr.count, p, [Sm, *Sv]))
    theta = T.fit_standardisation(ctx, snaps[:4], T.initial_theta(1))
    yield ctx, snaps, theta
    ctx.close()


def test_training_reduces_the_loss(setup):
    from paper_2512_20829_amd import train as T
    ctx, all_snaps, theta = setup
    snaps, held = all_snaps[:4], all_snaps[4:]
    model = T.BandwidthModel(ctx, theta, lr=3e-3)
    before = np.mean([model.evaluate(s) for s in snaps])
    for it in range(80):
        model.train_step(snaps[it % len(snaps)])
    after = np.mean([model.evaluate(s) for s in snaps])
    plain = np.mean([model.evaluate(s, learned=False) for s in snaps])
    held_learned = np.mean([model.evaluate(s) for s in held])
    held_plain = np.mean([model.evaluate(s, learned=False) for s in held])
    print(f"loss before {before:.4f} after {after:.4f} plain {plain:.4f}; held-out learned {held_learned:.4f} "
          f"plain {held_plain:.4f}")
    assert before == pytest.approx(plain, rel=1e-6)      # zero output layer: the plain rule
    assert after < 0.95 * before
    assert held_learned < held_plain


def test_checkpoint_resume_is_bitwise(setup):
    from paper_2512_20829_amd import train as T
    ctx, snaps, theta = setup
    a = T.BandwidthModel(ctx, theta, lr=2e-3)
    for it in range(12):
        a.train_step(snaps[it % 4])
    state = a.state_dict()
    b = T.BandwidthModel(ctx, theta, lr=0.0)
    b.load_state_dict(state)
    for it in range(12, 24):
        b.train_step(snaps[it % 4])
    c = T.BandwidthModel(ctx, theta, lr=2e-3)
    for it in range(24):
        c.train_step(snaps[it % 4])
    torch.cuda.synchronize()
    assert torch.equal(b.theta, c.theta) and torch.equal(b.m, c.m) and torch.equal(b.v, c.v)


def test_library_train_step_equals_the_six_call_composition(setup):
    """fla_mlp_train_step against the same stages called one by one:
    parameters, moments and loss bit for bit over several steps."""
    from paper_2512_20829_amd import train as T
    ctx, snaps, theta = setup
    a = T.BandwidthModel(ctx, theta, lr=2e-3)
    b = T.BandwidthModel(ctx, theta, lr=2e-3)
    for it in range(7):
        ra = a.train_step(snaps[it % 4])
        rb = b.train_step_composed(snaps[it % 4])
        torch.cuda.synchronize()
        assert torch.equal(ra, rb), it
    assert torch.equal(a.theta, b.theta) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
    assert not torch.equal(a.theta, torch.tensor(theta, dtype=torch.float32, device=DEV))


def test_train_step_rejects_bad_arguments(setup):
    import paper_2512_20829_amd as F
    from paper_2512_20829_amd import train as T
    ctx, snaps, theta = setup
    model = T.BandwidthModel(ctx, theta)
    s = snaps[0]
    before = model.theta.clone()
    bad = [F.Params(**{**s.params.__dict__, "mode": F.FLA_DEPOSIT}),
           F.Params(**{**s.params.__dict__, "h_factor": torch.ones(s.count, device=DEV)}),
           F.Params(**{**s.params.__dict__, "h0": -1.0})]
    for p in bad:
        with pytest.raises(F.FlaError) as e:
            ctx.mlp_train_step(F.mesh_of(s.mesh), s.traj, p, s.ref, model.theta, model.m, model.v, 1)
        assert e.value.status == F.FLA_ERR_INVALID_ARG
    with pytest.raises(F.FlaError):
        ctx.mlp_train_step(F.mesh_of(s.mesh), s.traj, s.params, s.ref, model.theta, model.m, model.v, 0)
    torch.cuda.synchronize()
    assert torch.equal(model.theta, before)


def test_standardisation_over_valid_trajectories():
    """fla_bandwidth_standardise against numpy over the trajectories the
    oracle finds valid, with trajectories whose |det J| is exactly 1 (raw
    feature log(n/n0) = 0, still valid) and skipped ones (det J = 0)."""
    import oracle
    import oracle.learned as LN
    import paper_2512_20829_amd as F
    from helpers import as_precision, device_traj
    ctx = F.Context(0)
    try:
        wls = [W.small_random_3d(3000, 12, seed=60 + k, periodic=True) for k in range(3)]
        for k, wl in enumerate(wls):
            J = wl.traj.J.clone()
            J[:, :50] = torch.eye(3, dtype=torch.float64).reshape(9, 1)      # |det J| = 1
            J[:, 50:60] = 0.0                                                 # det J = 0: skipped
            wl.traj.J = J
        feats = []
        for wl in wls:
            tr = as_precision(wl.traj, "f32")
            t = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
            f = LN.features(wl.mesh, tr.x.numpy(), tr.J.numpy(), t.valid)
            feats.append(f[:, t.valid == 1])
            assert (t.valid[:50] == 1).all() and (t.valid[50:60] == 0).all()
        fall = np.concatenate(feats, axis=1)
        mu_ref, sd_ref = fall.mean(axis=1), fall.std(axis=1, ddof=1) + 1e-3
        structs = [device_traj(wl.traj, "f32") for wl in wls]
        th = torch.zeros(F.MLP_PARAMS, dtype=torch.float32, device=DEV)
        th[F.MLP_TRAINABLE + 5:] = 1.0
        ctx.bandwidth_standardise([F.mesh_of(wl.mesh) for wl in wls], [s for s, _ in structs], th)
        torch.cuda.synchronize()
        got = th.cpu().double().numpy()
        print(f"[standardise] mu {got[F.MLP_TRAINABLE:F.MLP_TRAINABLE + 5]} ref {mu_ref}", flush=True)
        np.testing.assert_allclose(got[F.MLP_TRAINABLE:F.MLP_TRAINABLE + 5], mu_ref, rtol=2e-6, atol=2e-6)
        np.testing.assert_allclose(got[F.MLP_TRAINABLE + 5:], sd_ref, rtol=2e-6, atol=2e-6)
        assert np.all(got[:F.MLP_TRAINABLE] == 0.0)
        # deterministic
        th2 = th.clone()
        ctx.bandwidth_standardise([F.mesh_of(wl.mesh) for wl in wls], [s for s, _ in structs], th2)
        torch.cuda.synchronize()
        assert torch.equal(th, th2)
    finally:
        ctx.close()
