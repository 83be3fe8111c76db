"""Graphs of single fla_project_sources calls (fla_set_graph): the first call
with a set of arguments runs directly, the next one captures and launches,
later identical calls replay.  Every call is compared bit for bit with the
same call on a context without graphs, with inputs changed in place between
replays and other library calls (which may grow the workspace) in between."""
import numpy as np
import pytest
import torch

import workloads as W
from helpers import device_traj

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctxs():
    import paper_2512_20829_amd as F
    a, b = F.Context(0), F.Context(0)
    yield a, b
    a.close()
    b.close()


def _setup(kind):
    import paper_2512_20829_amd as F
    if kind == "2d_f64":
        wl = W.taylor_green_2d()
        prec, dt, dim = "f64", torch.float64, 2
    else:
        wl = W.small_random_3d(3000, 12, seed=41, periodic=True, h0=0.03)
        prec, dt, dim = "f32", torch.float32, 3
    tr, keep = device_traj(wl.traj, prec)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, count_pairs=True)
    outs = [F.alloc_fields(wl.mesh.cells, dim, dt, DEV) for _ in range(2)]
    pairs = [torch.zeros(wl.mesh.cells, dtype=torch.int32, device=DEV) for _ in range(2)]
    return wl, F.mesh_of(wl.mesh), tr, keep, p, outs, pairs


def _same(o, q, pa, pb):
    assert torch.equal(o[0], q[0]) and all(torch.equal(x, y) for x, y in zip(o[1], q[1]))
    assert torch.equal(o[2], q[2]) and torch.equal(pa, pb)


@pytest.mark.parametrize("kind", ["2d_f64", "3d_f32"])
def test_single_call_graphs(ctxs, kind):
    import paper_2512_20829_amd as F
    g, d = ctxs
    print(f"[case] single-call graphs {kind}", flush=True)
    wl, mesh, tr, keep, p, outs, pairs = _setup(kind)
    g.set_graph(True)
    try:
        def both(params=p):
            g.project_sources(mesh, tr, params, *outs[0], pairs=pairs[0])
            d.project_sources(mesh, tr, params, *outs[1], pairs=pairs[1])
            torch.cuda.synchronize()
            _same(outs[0], outs[1], pairs[0], pairs[1])
            return g.stats(), d.stats()

        r0 = g.stats()["graph_replays"]
        v = keep[wl.mesh.dim]  # the first velocity plane (after the dim position planes), changed in place
        for call in range(5):
            if call >= 2:
                v.mul_(1.0 + 0.01 * call)
            sg, sd = both()
            assert sg["pairs"] == sd["pairs"] > 0
        assert g.stats()["graph_replays"] - r0 == 3
        # other calls on the graph context in between (PSI-CELL grows its workspace)
        cloud = W.abc_cloud(200_000, seed=42) if kind == "3d_f32" else W.taylor_green_cloud(200_000, seed=42)
        pc, pk = device_traj(cloud, "f32" if kind == "3d_f32" else "f64")
        tmp = F.alloc_fields(wl.mesh.cells, wl.mesh.dim, outs[0][0].dtype, DEV)
        for call in range(4):
            g.psicell_accumulate(mesh, pc, 1.0, p, *tmp)
            v.mul_(0.99)
            both()
        # a changed argument is a new set: direct, then captured again
        r1 = g.stats()["graph_replays"]
        p2 = F.Params(**{**p.__dict__, "scale": 0.5})
        for call in range(3):
            both(p2)
        assert g.stats()["graph_replays"] - r1 == 1
        # disabled: no more replays
        g.set_graph(False)
        r2 = g.stats()["graph_replays"]
        both(p2)
        both(p2)
        assert g.stats()["graph_replays"] == r2
    finally:
        g.set_graph(False)
