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
