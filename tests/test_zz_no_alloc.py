"""The allocation-free projection entry point against fla_project_sources,
through the C ABI: bit-identical fields, denominators and per-cell pair
counts on two calls in a row (the second with a smaller input, so stale
workspace contents from the first call would show), in both precisions and
modes, and a clear argument error for inputs beyond the fixed workspace."""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import device_traj

pytestmark = pytest.mark.gpu


def _run(ctx, wl, prec, mode, noalloc):
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    dev = torch.device("cuda", 0)
    st, keep = device_traj(wl.traj, prec)
    M = wl.mesh.cells
    S_mass, S_mom, den = F.alloc_fields(M, wl.mesh.dim, dt, dev)
    for t in [S_mass, *S_mom, den]:
        t.fill_(float("nan"))
    pairs = torch.full((M,), -1, dtype=torch.int32, device=dev)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, mode=mode)
    fn = ctx.project_sources_noalloc if noalloc else ctx.project_sources
    fn(F.mesh_of(wl.mesh), st, p, S_mass, S_mom, den, pairs=pairs)
    torch.cuda.synchronize()
    return (torch.stack([S_mass, *S_mom]).cpu().numpy(), den.cpu().numpy(), pairs.cpu().numpy(),
            ctx.stats())


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_matches_the_allocating_entry_point(prec, mode):
    import paper_2512_20829_amd as F
    ctx = F.Context(0)
    try:
        big = W.small_random_3d(60000, 24, seed=90, periodic=True)
        small = W.small_random_3d(7000, 11, seed=91, periodic=False)
        for wl in (big, small):
            print(f"[case] noalloc prec={prec} mode={mode} N={wl.traj.count} mesh={wl.mesh.n}", flush=True)
            S1, d1, p1, st1 = _run(ctx, wl, prec, mode, noalloc=True)
            S0, d0, p0, st0 = _run(ctx, wl, prec, mode, noalloc=False)
            assert np.isfinite(S1).all() and (p1 >= 0).all()
            assert np.array_equal(S1, S0) and np.array_equal(d1, d0) and np.array_equal(p1, p0)
            for k in ("trajectories", "skipped", "pairs", "zero_support", "max_class"):
                assert st1[k] == st0[k], k
    finally:
        ctx.close()


def test_noalloc_rejects_inputs_beyond_its_workspace_and_writes_nothing():
    import paper_2512_20829_amd as F
    ctx = F.Context(0)
    try:
        n = F.NOALLOC_SCRATCH_BYTES // 144 + 1000
        wl = W.small_random_3d(n, 8, seed=92, periodic=True)
        st, keep = device_traj(wl.traj, "f32")
        dev = torch.device("cuda", 0)
        S_mass, S_mom, den = F.alloc_fields(wl.mesh.cells, 3, torch.float32, dev)
        for t in [S_mass, *S_mom, den]:
            t.fill_(3.0)
        p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
        with pytest.raises(F.FlaError, match="bytes of workspace") as e:
            ctx.project_sources_noalloc(F.mesh_of(wl.mesh), st, p, S_mass, S_mom, den)
        assert e.value.status == F.FLA_ERR_INVALID_ARG
        torch.cuda.synchronize()
        assert all(bool((t == 3.0).all()) for t in [S_mass, *S_mom, den])
        # the context is still usable, and so is the entry point on a fitting input
        ok = W.small_random_3d(5000, 8, seed=93, periodic=True)
        S1, d1, p1, _ = _run(ctx, ok, "f32", 0, noalloc=True)
        S0, d0, p0, _ = _run(ctx, ok, "f32", 0, noalloc=False)
        assert np.array_equal(S1, S0) and np.array_equal(p1, p0)
    finally:
        ctx.close()
