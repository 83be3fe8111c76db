"""Argument errors of fla_project_sources and psicell_accumulate, through the
C ABI: each bad argument returns FLA_ERR_INVALID_ARG with a message, and no
output plane is written (the checks run on the host before any launch)."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from helpers import device_traj

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_20829_amd as F
    c = F.Context(0)
    yield c
    c.close()


class Case:
    """A valid small 3-D call whose arguments the tests then break one at a time."""

    def __init__(self):
        import paper_2512_20829_amd as F
        self.wl = W.small_random_3d(300, 8, seed=70, periodic=True)
        self.traj, self.keep = device_traj(self.wl.traj, "f32")
        self.mesh = F.mesh_of(self.wl.mesh)
        M = self.wl.mesh.cells
        dev = torch.device("cuda", 0)
        self.planes = [torch.full((M,), 12345.0, dtype=torch.float32, device=dev) for _ in range(5)]
        self.pairs = torch.full((M,), 777, dtype=torch.int32, device=dev)
        self.out = F.make_fields(self.planes[0], self.planes[1:4], self.planes[4], self.pairs)
        self.params = F.Params(rho_d=self.wl.rho_d, mu=self.wl.mu, delta=self.wl.delta, h0=self.wl.h0,
                               cutoff=self.wl.cutoff).to_c()

    def untouched(self):
        torch.cuda.synchronize()
        return all(bool((p == 12345.0).all()) for p in self.planes) and bool((self.pairs == 777).all())


def _project(ctx, c, mesh=None, traj=None, params=None, out=None):
    import paper_2512_20829_amd as F
    L = F.lib()
    ref = lambda s: C.byref(s) if s is not None else None
    return L.fla_project_sources(ctx.handle, ref(mesh), ref(traj), ref(params), ref(out), None)


def _psicell(ctx, c, mesh=None, traj=None, weight=1.0, params=None, out=None):
    import paper_2512_20829_amd as F
    L = F.lib()
    ref = lambda s: C.byref(s) if s is not None else None
    return L.psicell_accumulate(ctx.handle, ref(mesh), ref(traj), weight, ref(params), ref(out), None)


def _copy(s):
    t = type(s)()
    C.memmove(C.byref(t), C.byref(s), C.sizeof(s))
    return t


def _bad_variants(c):
    """(label, mesh, traj, params, out) with one argument broken."""
    out = []
    out.append(("NULL mesh", None, c.traj, c.params, c.out))
    out.append(("NULL trajectories", c.mesh, None, c.params, c.out))
    out.append(("NULL params", c.mesh, c.traj, None, c.out))
    out.append(("NULL out", c.mesh, c.traj, c.params, None))
    for dim in (1, 4, 0):
        m = _copy(c.mesh)
        m.dim = dim
        out.append((f"dim {dim}", m, c.traj, c.params, c.out))
    m = _copy(c.mesh)
    m.n[1] = 0
    out.append(("zero cells on an axis", m, c.traj, c.params, c.out))
    m = _copy(c.mesh)
    m.hi[2] = m.lo[2]
    out.append(("hi == lo", m, c.traj, c.params, c.out))
    t = _copy(c.traj)
    t.count = -5
    out.append(("negative count", c.mesh, t, c.params, c.out))
    t = _copy(c.traj)
    t.x[1] = None
    out.append(("NULL x[1]", c.mesh, t, c.params, c.out))
    t = _copy(c.traj)
    t.r = None
    out.append(("NULL r", c.mesh, t, c.params, c.out))
    t = _copy(c.traj)
    t.prec = 7
    out.append(("bad precision", c.mesh, t, c.params, c.out))
    o = _copy(c.out)
    o.S_mom[2] = None
    out.append(("NULL S_mom[2]", c.mesh, c.traj, c.params, o))
    for name, val in (("rho_d", -1.0), ("mu", 0.0), ("delta", float("nan"))):
        p = _copy(c.params)
        setattr(p, name, val)
        out.append((f"{name} = {val}", c.mesh, c.traj, p, c.out))
    return out


def test_project_sources_rejects_bad_arguments_and_writes_nothing(ctx):
    import paper_2512_20829_amd as F
    c = Case()
    cases = _bad_variants(c)
    for name, val in (("h0", 0.0), ("h0", -1.0), ("h0", float("inf")), ("cutoff", 0.0), ("cutoff", -4.0),
                      ("cutoff", float("nan")), ("scale", float("inf")), ("mode", 9)):
        p = _copy(c.params)
        setattr(p, name, val)
        cases.append((f"{name} = {val}", c.mesh, c.traj, p, c.out))
    t = _copy(c.traj)
    t.J = None
    cases.append(("NULL J", c.mesh, t, c.params, c.out))
    p = _copy(c.params)
    p.mode = F.FLA_DEPOSIT
    t = _copy(c.traj)
    t.seed_volume = 0.0
    cases.append(("deposition without a seed volume", c.mesh, t, p, c.out))
    for label, m, t, p, o in cases:
        print(f"[case] project_sources: {label}", flush=True)
        st = _project(ctx, c, m, t, p, o)
        assert st == F.FLA_ERR_INVALID_ARG, label
        assert ctx.last_error(), label
        assert c.untouched(), label
    # the unbroken call still works on the same context
    assert _project(ctx, c, c.mesh, c.traj, c.params, c.out) == F.FLA_OK
    torch.cuda.synchronize()
    assert not c.untouched()
    assert ctx.last_error() == ""


def test_psicell_rejects_bad_arguments_and_writes_nothing(ctx):
    import paper_2512_20829_amd as F
    c = Case()
    cases = [(label, m, t, p, o, 1.0) for label, m, t, p, o in _bad_variants(c)]
    cases.append(("weight = nan", c.mesh, c.traj, c.params, c.out, float("nan")))
    cases.append(("weight = inf", c.mesh, c.traj, c.params, c.out, float("inf")))
    for label, m, t, p, o, w in cases:
        print(f"[case] psicell_accumulate: {label}", flush=True)
        st = _psicell(ctx, c, m, t, w, p, o)
        assert st == F.FLA_ERR_INVALID_ARG, label
        assert ctx.last_error(), label
        assert c.untouched(), label
    # J, h0 and cutoff are not used by PSI-CELL
    t = _copy(c.traj)
    t.J = None
    p = _copy(c.params)
    p.h0 = -1.0
    assert _psicell(ctx, c, c.mesh, t, 1.0, p, c.out) == F.FLA_OK
    torch.cuda.synchronize()
    assert not c.untouched()


def test_null_context_is_rejected():
    import paper_2512_20829_amd as F
    L = F.lib()
    assert L.fla_project_sources(None, None, None, None, None, None) == F.FLA_ERR_INVALID_ARG
    assert L.psicell_accumulate(None, None, None, 1.0, None, None, None) == F.FLA_ERR_INVALID_ARG
