"""Launch log (FLA_TRACE) and the simulated out-of-memory hook
(FLA_FAIL_ALLOC) through the C ABI: a failed workspace allocation returns
FLA_ERR_OUT_OF_MEMORY with the outputs untouched, and the next call on the
same context succeeds with the fields of an unaffected context."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from helpers import device_traj

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _fresh_ctx(**env):
    import paper_2512_20829_amd as F
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return F.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _fields(M, dim, dt):
    import paper_2512_20829_amd as F
    S_mass, S_mom, den = F.alloc_fields(M, dim, dt, DEV)
    for t in [S_mass, *S_mom, den]:
        t.fill_(float("nan"))
    return S_mass, S_mom, den


def test_launch_log(capfd):
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(2000, 12, seed=71, periodic=True)
    tr, keep = device_traj(wl.traj, "f32")
    ctx = _fresh_ctx(FLA_TRACE=1)
    try:
        S_mass, S_mom, den = _fields(wl.mesh.cells, 3, torch.float32)
        p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0)
        ctx.project_sources(F.mesh_of(wl.mesh), tr, p, S_mass, S_mom, den)
        torch.cuda.synchronize()
        err = capfd.readouterr().err
    finally:
        ctx.close()
        _fresh_ctx(FLA_TRACE=0).close()          # the log is per process: switch it off again
    lines = [l for l in err.splitlines() if l.startswith("[flaproj]")]
    assert any("call fla_project_sources mesh=12x12x12 N=2000 f32 -> 0" in l for l in lines), lines[-5:]
    for k in ("k_prepass", "k_radix_scatter", "k_permute", "k_gather"):
        assert any(f"launch" in l and k in l for l in lines), k
    n_lines = len(lines)
    ctx2 = F.Context(0)
    S_mass, S_mom, den = _fields(wl.mesh.cells, 3, torch.float32)
    ctx2.project_sources(F.mesh_of(wl.mesh), tr, F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0),
                         S_mass, S_mom, den)
    torch.cuda.synchronize()
    ctx2.close()
    assert "[flaproj]" not in capfd.readouterr().err and n_lines > 5


@pytest.mark.parametrize("entry", ["project", "psicell", "cells"])
def test_simulated_out_of_memory_leaves_outputs_untouched(entry):
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(3000, 14, seed=72, periodic=False)
    tr, keep = device_traj(wl.traj, "f32")
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0)
    mesh = F.mesh_of(wl.mesh)
    cells = W.scattered_cells(3, 14, (0.0,) * 3, (1.0,) * 3, (False,) * 3, seed=73)
    cs, ck = F.cells_of(cells, DEV)

    def call(ctx, out, index=None):
        if entry == "project":
            ctx.project_sources(mesh, tr, p, *out)
        elif entry == "psicell":
            ctx.psicell_accumulate(mesh, tr, 2.0, p, *out)
        else:
            ctx.project_cells(index, tr, p, *out)

    M = cells.count if entry == "cells" else wl.mesh.cells
    good = F.Context(0)
    ref = _fields(M, 3, torch.float32)
    gix = good.cell_index(cs) if entry == "cells" else None     # an index serves any context on its device
    call(good, ref, gix)
    torch.cuda.synchronize()
    bad = _fresh_ctx(FLA_FAIL_ALLOC=1)       # the call's workspace is the context's first allocation
    try:
        ix = gix
        out = _fields(M, 3, torch.float32)
        with pytest.raises(F.FlaError, match="OUT_OF_MEMORY"):
            call(bad, out, ix)
        torch.cuda.synchronize()
        for t in [out[0], *out[1], out[2]]:
            assert torch.isnan(t).all()
        call(bad, out, ix)                        # the next allocation succeeds
        torch.cuda.synchronize()
        for a, b in zip([out[0], *out[1], out[2]], [ref[0], *ref[1], ref[2]]):
            assert torch.equal(a, b)
    finally:
        bad.close()
        if gix is not None:
            gix.close()
        good.close()


def test_out_of_memory_while_building_an_index():
    import paper_2512_20829_amd as F
    cells = W.scattered_cells(3, 10, (0.0,) * 3, (1.0,) * 3, (True,) * 3, seed=74)
    cs, ck = F.cells_of(cells, DEV)
    for k in (1, 2, 4, 6, 7):
        ctx = _fresh_ctx(FLA_FAIL_ALLOC=k)
        try:
            with pytest.raises(F.FlaError, match="OUT_OF_MEMORY"):
                ctx.cell_index(cs)
            ix = ctx.cell_index(cs)                # partial buffers were released; a retry succeeds
            assert ix.shape()[1] > 0
            ix.close()
        finally:
            ctx.close()
