"""Python binding of libflaproj.so, the gfx950 FLA source-projection library.

Argument marshalling only: torch tensors (device memory) are turned into the
C structs of ``include/flaproj.h`` and every step runs in the library's HIP
kernels.  There is no CPU fallback; importing this module fails if the
shared library has not been built (``python paper_2512_20829_amd/build.py``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflaproj.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python {os.path.join(HERE, 'build.py')}`")

_lib = C.CDLL(LIB_PATH)

FLA_OK, FLA_ERR_INVALID_ARG, FLA_ERR_OUT_OF_MEMORY, FLA_ERR_DEVICE, FLA_ERR_UNSUPPORTED = range(5)
FLA_F32, FLA_F64 = 0, 1
FLA_NW, FLA_DEPOSIT = 0, 1
STATUS_NAMES = {0: "FLA_OK", 1: "FLA_ERR_INVALID_ARG", 2: "FLA_ERR_OUT_OF_MEMORY", 3: "FLA_ERR_DEVICE",
                4: "FLA_ERR_UNSUPPORTED"}


class fla_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("periodic", C.c_int32 * 3), ("cell_scale", C.c_void_p), ("edges", C.c_void_p * 3)]


class fla_trajectories(C.Structure):
    _fields_ = [("count", C.c_int64), ("prec", C.c_int32), ("reserved", C.c_int32),
                ("x", C.c_void_p * 3), ("J", C.c_void_p), ("v", C.c_void_p * 3), ("ug", C.c_void_p * 3),
                ("r", C.c_void_p), ("n0", C.c_void_p), ("n0_scalar", C.c_double),
                ("seed_volume", C.c_double)]


class fla_params(C.Structure):
    _fields_ = [("rho_d", C.c_double), ("mu", C.c_double), ("delta", C.c_double), ("h0", C.c_double),
                ("cutoff", C.c_double), ("scale", C.c_double), ("mode", C.c_int32),
                ("count_pairs", C.c_int32), ("h_factor", C.c_void_p)]


class fla_fields(C.Structure):
    _fields_ = [("S_mass", C.c_void_p), ("S_mom", C.c_void_p * 3), ("den", C.c_void_p), ("pairs", C.c_void_p)]


class fla_stats(C.Structure):
    _fields_ = [("trajectories", C.c_int64), ("skipped", C.c_int64), ("no_support", C.c_int64),
                ("pairs", C.c_int64), ("outside", C.c_int64), ("zero_support", C.c_int64),
                ("max_class", C.c_int64), ("graph_replays", C.c_int64)]


class fla_flow(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("U", C.c_double), ("k", C.c_double),
                ("abc", C.c_double * 3), ("phase", C.c_double * 3), ("u0", C.c_double * 3), ("G", C.c_double * 9)]


class fla_droplets(C.Structure):
    _fields_ = [("count", C.c_int64), ("x", C.c_void_p * 3), ("v", C.c_void_p * 3), ("J", C.c_void_p),
                ("dJ", C.c_void_p), ("r", C.c_void_p), ("n0", C.c_void_p), ("n0_scalar", C.c_double),
                ("seed_volume", C.c_double), ("phibar", C.c_void_p)]


class fla_step(C.Structure):
    _fields_ = [("dt", C.c_double), ("substeps", C.c_int32), ("update_state", C.c_int32)]


FLA_FLOW_NONE, FLA_FLOW_TAYLOR_GREEN, FLA_FLOW_ABC = 0, 1, 2

PROFILE_STAGES = ["prepass", "sort", "deposit_norm", "gather", "psicell", "mlp_forward", "proj_backward",
                  "mlp_backward"]
MLP_TRAINABLE = 4609
MLP_PARAMS = 4619
GATHER_PLANS = 4
GATHER_SHAPES = 2
GATHER_CONFIGS = GATHER_PLANS * GATHER_SHAPES   # plan codes: plan + GATHER_PLANS * shape
BATCH_CHUNKS = 4
BATCH_MAX = 65536


class fla_profile(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8)]


class fla_cells(C.Structure):
    _fields_ = [("dim", C.c_int32), ("periodic", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("count", C.c_int64), ("centroid", C.c_void_p * 3), ("volume", C.c_void_p)]


class fla_injection(C.Structure):
    _fields_ = [("n_ref", C.c_double), ("tau_ref", C.c_double), ("area", C.c_double), ("v_inj", C.c_double)]


_vp = C.c_void_p
_lib.fla_cell_index_create.restype = C.c_int
_lib.fla_cell_index_create.argtypes = [_vp, C.POINTER(fla_cells), C.c_int32, C.POINTER(_vp)]
_lib.fla_cell_index_destroy.restype = C.c_int
_lib.fla_cell_index_destroy.argtypes = [_vp]
_lib.fla_cell_index_shape.restype = C.c_int
_lib.fla_cell_index_shape.argtypes = [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
_lib.fla_project_cells.restype = C.c_int
_lib.fla_project_cells.argtypes = [_vp, _vp, C.POINTER(fla_trajectories), C.POINTER(fla_params),
                                   C.POINTER(fla_injection), C.POINTER(fla_fields), _vp]
_lib.fla_ctx_create.restype = C.c_int
_lib.fla_ctx_create.argtypes = [C.POINTER(_vp), C.c_int]
_lib.fla_ctx_destroy.restype = C.c_int
_lib.fla_ctx_destroy.argtypes = [_vp]
_lib.fla_project_sources.restype = C.c_int
_lib.fla_project_sources.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories),
                                     C.POINTER(fla_params), C.POINTER(fla_fields), _vp]
_lib.fla_project_sources_noalloc.restype = C.c_int
_lib.fla_project_sources_noalloc.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories),
                                             C.POINTER(fla_params), C.POINTER(fla_fields), _vp]
NOALLOC_SCRATCH_BYTES = 64 << 20
_lib.psicell_accumulate.restype = C.c_int
_lib.psicell_accumulate.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories), C.c_double,
                                    C.POINTER(fla_params), C.POINTER(fla_fields), _vp]
_lib.cic_accumulate.restype = C.c_int
_lib.cic_accumulate.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories), C.c_double,
                                C.POINTER(fla_params), C.POINTER(fla_fields), _vp]
_lib.fla_get_stats.restype = C.c_int
_lib.fla_get_stats.argtypes = [_vp, C.POINTER(fla_stats)]
_lib.fla_profile_enable.restype = C.c_int
_lib.fla_profile_enable.argtypes = [_vp, C.c_int]
_lib.fla_profile_read.restype = C.c_int
_lib.fla_profile_read.argtypes = [_vp, C.POINTER(fla_profile)]
_lib.fla_set_plan.restype = C.c_int
_lib.fla_set_plan.argtypes = [_vp, C.c_int, C.c_int, C.c_int]
_lib.fla_get_plan.restype = C.c_int
_lib.fla_get_plan.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(C.c_int)]
_lib.fla_autotune.restype = C.c_int
_lib.fla_autotune.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories), C.POINTER(fla_params),
                              C.POINTER(fla_fields), _vp, C.POINTER(C.c_double)]
_lib.fla_bandwidth_forward.restype = C.c_int
_lib.fla_bandwidth_forward.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories), _vp, _vp, _vp, _vp,
                                       _vp, _vp]
_lib.fla_project_backward.restype = C.c_int
_lib.fla_project_backward.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories), C.POINTER(fla_params),
                                      C.POINTER(fla_fields), C.POINTER(fla_fields), _vp, _vp]
_lib.fla_bandwidth_backward.restype = C.c_int
_lib.fla_bandwidth_backward.argtypes = [_vp, C.c_int, _vp, C.c_int64, _vp, _vp, _vp, _vp, _vp]
_lib.fla_adam_step.restype = C.c_int
_lib.fla_adam_step.argtypes = [_vp, _vp, _vp, _vp, _vp, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double, _vp]
_lib.fla_rel_l2_loss.restype = C.c_int
_lib.fla_rel_l2_loss.argtypes = [_vp, C.c_int, C.c_int64, C.c_int, C.POINTER(fla_fields), C.POINTER(fla_fields),
                                 C.POINTER(fla_fields), _vp, _vp]
_lib.fla_advance_project.restype = C.c_int
_lib.fla_advance_project.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_droplets), C.POINTER(fla_flow),
                                     C.POINTER(fla_step), C.POINTER(fla_params), C.c_int, C.POINTER(fla_fields), _vp]
_lib.fla_bandwidth_standardise.restype = C.c_int
_lib.fla_bandwidth_standardise.argtypes = [_vp, C.c_int, C.POINTER(fla_mesh), C.POINTER(fla_trajectories), _vp, _vp]
_lib.fla_mlp_train_step.restype = C.c_int
_lib.fla_mlp_train_step.argtypes = [_vp, C.POINTER(fla_mesh), C.POINTER(fla_trajectories), C.POINTER(fla_params),
                                    C.POINTER(fla_fields), _vp, _vp, _vp, C.c_int64, C.c_double, C.c_double,
                                    C.c_double, C.c_double, _vp, _vp]
_lib.fla_project_batch.restype = C.c_int
_lib.fla_project_batch.argtypes = [_vp, C.c_int, C.POINTER(fla_mesh), C.POINTER(fla_trajectories),
                                   C.POINTER(fla_params), C.POINTER(fla_fields), _vp]
_lib.fla_set_batch_graph.restype = C.c_int
_lib.fla_set_batch_graph.argtypes = [_vp, C.c_int]
_lib.fla_save_plans.restype = C.c_int
_lib.fla_save_plans.argtypes = [_vp, C.c_char_p]
_lib.fla_load_plans.restype = C.c_int
_lib.fla_load_plans.argtypes = [_vp, C.c_char_p]
_lib.fla_set_graph.restype = C.c_int
_lib.fla_set_graph.argtypes = [_vp, C.c_int]
_lib.fla_set_batch_plan.restype = C.c_int
_lib.fla_set_batch_plan.argtypes = [_vp, C.c_int, C.c_int, C.c_int, C.c_int]
_lib.fla_get_batch_plan.restype = C.c_int
_lib.fla_get_batch_plan.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
_lib.fla_autotune_batch.restype = C.c_int
_lib.fla_autotune_batch.argtypes = [_vp, C.c_int, C.POINTER(fla_mesh), C.POINTER(fla_trajectories),
                                    C.POINTER(fla_params), C.POINTER(fla_fields), _vp, C.POINTER(C.c_double)]
_lib.fla_last_error.restype = C.c_char_p
_lib.fla_last_error.argtypes = [_vp]


def lib() -> C.CDLL:
    return _lib


class FlaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


@dataclass
class Params:
    rho_d: float
    mu: float
    delta: float
    h0: float
    cutoff: float = 4.0
    scale: float = 1.0
    mode: int = FLA_NW
    count_pairs: bool = False
    h_factor: object = None      # optional float32 device tensor (N,)

    def to_c(self) -> fla_params:
        p = fla_params()
        p.rho_d, p.mu, p.delta, p.h0, p.cutoff, p.scale = (self.rho_d, self.mu, self.delta, self.h0,
                                                            self.cutoff, self.scale)
        p.mode = int(self.mode)
        p.count_pairs = int(bool(self.count_pairs))
        p.h_factor = _ptr(self.h_factor)
        return p


def make_mesh(dim: int, n: Sequence[int], lo: Sequence[float], hi: Sequence[float],
              periodic: Sequence[bool], cell_scale=None, edges=None) -> fla_mesh:
    """edges: None, or per axis None (uniform) or a contiguous float64 device
    tensor of n[a] + 1 increasing cell edges (a rectilinear axis); the
    caller keeps the tensors alive."""
    m = fla_mesh()
    m.dim = dim
    for a in range(3):
        m.n[a] = int(n[a]) if a < dim else 1
        m.lo[a] = float(lo[a]) if a < dim else 0.0
        m.hi[a] = float(hi[a]) if a < dim else 1.0
        m.periodic[a] = int(bool(periodic[a])) if a < dim else 0
    m.cell_scale = _ptr(cell_scale)
    for a in range(3):
        e = edges[a] if (edges is not None and a < dim) else None
        if e is not None:
            import torch
            if e.dtype != torch.float64 or e.numel() != int(n[a]) + 1:
                raise ValueError("edges[a] must be float64 with n[a] + 1 values")
        m.edges[a] = _ptr(e)
    return m


def mesh_of(obj, cell_scale=None, edges=None) -> fla_mesh:
    """From an object with dim, n, lo, hi, periodic attributes."""
    return make_mesh(obj.dim, obj.n, obj.lo, obj.hi, obj.periodic, cell_scale, edges)


def make_trajectories(x, J, v, ug, r, n0=1.0, seed_volume: float = 0.0) -> tuple:
    """Build the C struct from device tensors.  x: (dim, N) float64, J: (dim*dim, N)
    float64, v, ug: (dim, N) and r: (N,) float32 or float64 (that dtype sets the
    call's precision), n0: float or (N,) float64 tensor.  Returns (struct, keepalive)."""
    import torch
    dim, N = int(x.shape[0]), int(x.shape[1])
    prec = FLA_F64 if v.dtype == torch.float64 else FLA_F32
    want = torch.float64 if prec == FLA_F64 else torch.float32
    for name, t in (("v", v), ("ug", ug), ("r", r)):
        if t.dtype != want:
            raise ValueError(f"{name} must be {want}")
    if x.dtype != torch.float64 or (J is not None and J.dtype != torch.float64):
        raise ValueError("x and J must be float64")
    keep = []
    tr = fla_trajectories()
    tr.count = N
    tr.prec = prec
    rows = lambda t: [t[a].contiguous() for a in range(dim)]
    xs, vs, us = rows(x), rows(v), rows(ug)
    keep += xs + vs + us
    for a in range(dim):
        tr.x[a] = xs[a].data_ptr()
        tr.v[a] = vs[a].data_ptr()
        tr.ug[a] = us[a].data_ptr()
    if J is not None:
        Jc = J.contiguous()
        keep.append(Jc)
        tr.J = Jc.data_ptr()
    rc = r.contiguous()
    keep.append(rc)
    tr.r = rc.data_ptr()
    if isinstance(n0, (int, float)):
        tr.n0 = None
        tr.n0_scalar = float(n0)
    else:
        n0c = n0.to(torch.float64).contiguous()
        keep.append(n0c)
        tr.n0 = n0c.data_ptr()
        tr.n0_scalar = 0.0
    tr.seed_volume = float(seed_volume)
    return tr, keep


def make_cells(dim: int, centroids, volume, lo: Sequence[float], hi: Sequence[float],
               periodic: Sequence[bool]) -> tuple:
    """fla_cells from device tensors: centroids (dim, M) float64, volume (M,)
    float64 or None.  Returns (struct, keepalive)."""
    import torch
    if centroids.dtype != torch.float64 or (volume is not None and volume.dtype != torch.float64):
        raise ValueError("centroids and volume must be float64")
    c = fla_cells()
    c.dim = dim
    c.count = int(centroids.shape[1])
    keep = [centroids[a].contiguous() for a in range(dim)]
    for a in range(3):
        c.periodic[a] = int(bool(periodic[a])) if a < dim else 0
        c.lo[a] = float(lo[a]) if a < dim else 0.0
        c.hi[a] = float(hi[a]) if a < dim else 1.0
        c.centroid[a] = keep[a].data_ptr() if a < dim else None
    if volume is not None:
        vc = volume.contiguous()
        keep.append(vc)
        c.volume = vc.data_ptr()
    return c, keep


def cells_of(obj, device) -> tuple:
    """fla_cells from an object with dim, centroids, volume, lo, hi, periodic
    (tensors moved to `device`)."""
    vol = obj.volume.to(device) if obj.volume is not None else None
    return make_cells(obj.dim, obj.centroids.to(device), vol, obj.lo, obj.hi, obj.periodic)


def make_injection(n_ref: float, tau_ref: float, area: float, v_inj: float) -> fla_injection:
    j = fla_injection()
    j.n_ref, j.tau_ref, j.area, j.v_inj = float(n_ref), float(tau_ref), float(area), float(v_inj)
    return j


class CellIndex:
    """Owns one fla_cell_index (the spatial index of a general mesh)."""

    def __init__(self, ctx: "Context", cells: fla_cells, cells_per_bucket: int = 0):
        h = _vp()
        ctx._check(_lib.fla_cell_index_create(ctx.handle, C.byref(cells), int(cells_per_bucket), C.byref(h)))
        self._h = h
        self.count = int(cells.count)
        self.dim = int(cells.dim)

    @property
    def handle(self):
        return self._h

    def shape(self) -> tuple:
        nb = (C.c_int32 * 3)()
        nw = C.c_int64()
        st = _lib.fla_cell_index_shape(self._h, nb, C.byref(nw))
        if st != FLA_OK:
            raise FlaError(st, "fla_cell_index_shape")
        return tuple(int(v) for v in nb), int(nw.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.fla_cell_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_flow(kind: int = FLA_FLOW_NONE, U: float = 0.0, k: float = 1.0, abc=(1.0, 1.0, 1.0),
              phase=(0.0, 0.0, 0.0), u0=(0.0, 0.0, 0.0), G=None) -> fla_flow:
    """Gas field u = u0 + G x + (Taylor-Green or ABC part); G: nested lists or None."""
    f = fla_flow()
    f.kind, f.U, f.k = int(kind), float(U), float(k)
    pad = lambda t: [float(v) for v in t] + [0.0] * (3 - len(t))
    for a, (A, P, U0) in enumerate(zip(pad(abc), pad(phase), pad(u0))):
        f.abc[a], f.phase[a], f.u0[a] = A, P, U0
    if G is not None:
        for a, row in enumerate(G):
            for b, g in enumerate(row):
                f.G[a * 3 + b] = float(g)
    return f


def make_droplets(x, v, J, dJ, r, n0=1.0, seed_volume: float = 0.0, phibar=None) -> tuple:
    """Droplet state from float64 device tensors x, v (dim, N), J, dJ (dim*dim, N),
    r (N,); phibar: optional (1 + dim, N) float64 output.  The planes are used in
    place (the tensors must be contiguous).  Returns (struct, keepalive)."""
    import torch
    dim, N = int(x.shape[0]), int(x.shape[1])
    for name, t in (("x", x), ("v", v), ("J", J), ("dJ", dJ), ("r", r)):
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor")
    d = fla_droplets()
    d.count = N
    keep = [x, v, J, dJ, r]
    for a in range(dim):
        d.x[a] = x[a].data_ptr()
        d.v[a] = v[a].data_ptr()
    d.J, d.dJ, d.r = J.data_ptr(), dJ.data_ptr(), r.data_ptr()
    if isinstance(n0, (int, float)):
        d.n0, d.n0_scalar = None, float(n0)
    else:
        n0c = n0.to(torch.float64).contiguous()
        keep.append(n0c)
        d.n0, d.n0_scalar = n0c.data_ptr(), 0.0
    d.seed_volume = float(seed_volume)
    if phibar is not None:
        if phibar.dtype != torch.float64 or not phibar.is_contiguous():
            raise ValueError("phibar must be a contiguous float64 tensor")
        d.phibar = phibar.data_ptr()
        keep.append(phibar)
    return d, keep


def make_step(dt: float, substeps: int, update_state: bool = True) -> fla_step:
    st = fla_step()
    st.dt, st.substeps, st.update_state = float(dt), int(substeps), int(bool(update_state))
    return st


def make_fields(S_mass, S_mom: Sequence, den=None, pairs=None) -> fla_fields:
    """pairs: optional int32 device tensor (read as uint32 per cell)."""
    f = fla_fields()
    f.S_mass = _ptr(S_mass)
    for a, t in enumerate(S_mom):
        f.S_mom[a] = _ptr(t)
    f.den = _ptr(den)
    f.pairs = _ptr(pairs)
    return f


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Context:
    """Owns one fla_ctx (workspace and statistics) on a device."""

    def __init__(self, device: int = 0):
        h = _vp()
        st = _lib.fla_ctx_create(C.byref(h), int(device))
        if st != FLA_OK:
            raise FlaError(st, _lib.fla_last_error(None).decode())
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            _lib.fla_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return _lib.fla_last_error(self._h).decode()

    def _check(self, st: int):
        if st != FLA_OK:
            raise FlaError(st, self.last_error())

    # -- raw struct entry points ---------------------------------------------------------
    def project_sources_raw(self, mesh: fla_mesh, traj: fla_trajectories, params: fla_params,
                            out: fla_fields, stream=None) -> int:
        return _lib.fla_project_sources(self._h, C.byref(mesh), C.byref(traj), C.byref(params),
                                        C.byref(out), _stream_handle(stream))

    def psicell_raw(self, mesh, particles, weight, params, out, stream=None) -> int:
        return _lib.psicell_accumulate(self._h, C.byref(mesh), C.byref(particles), float(weight),
                                       C.byref(params), C.byref(out), _stream_handle(stream))

    # -- tensor-level helpers ------------------------------------------------------------
    def project_sources(self, mesh: fla_mesh, traj: fla_trajectories, params: Params, S_mass, S_mom,
                        den=None, stream=None, pairs=None):
        st = self.project_sources_raw(mesh, traj, params.to_c(), make_fields(S_mass, S_mom, den, pairs), stream)
        self._check(st)

    def project_sources_noalloc(self, mesh: fla_mesh, traj: fla_trajectories, params: Params, S_mass, S_mom,
                                den=None, stream=None, pairs=None):
        """fla_project_sources on the library's fixed workspace (no allocation)."""
        st = _lib.fla_project_sources_noalloc(self._h, C.byref(mesh), C.byref(traj), C.byref(params.to_c()),
                                              C.byref(make_fields(S_mass, S_mom, den, pairs)),
                                              _stream_handle(stream))
        self._check(st)

    def cell_index(self, cells: fla_cells, cells_per_bucket: int = 0) -> CellIndex:
        """fla_cell_index_create: the spatial index of a general mesh."""
        return CellIndex(self, cells, cells_per_bucket)

    def project_cells(self, index: CellIndex, traj: fla_trajectories, params: Params, S_mass, S_mom, den=None,
                      injection: Optional[fla_injection] = None, stream=None, pairs=None):
        """fla_project_cells: the estimator at the centroids of an indexed general mesh."""
        st = _lib.fla_project_cells(self._h, index.handle, C.byref(traj), C.byref(params.to_c()),
                                    C.byref(injection) if injection is not None else None,
                                    C.byref(make_fields(S_mass, S_mom, den, pairs)), _stream_handle(stream))
        self._check(st)

    def psicell_accumulate(self, mesh: fla_mesh, particles: fla_trajectories, weight: float,
                           params: Params, S_mass, S_mom, den=None, stream=None):
        st = self.psicell_raw(mesh, particles, weight, params.to_c(), make_fields(S_mass, S_mom, den), stream)
        self._check(st)

    def advance_project(self, mesh: fla_mesh, drops: fla_droplets, flow: fla_flow, step: fla_step, params: Params,
                        prec: int, S_mass, S_mom, den=None, pairs=None, stream=None):
        """fla_advance_project: advance the droplets one carrier step and project them."""
        self._check(_lib.fla_advance_project(self._h, C.byref(mesh), C.byref(drops), C.byref(flow), C.byref(step),
                                             C.byref(params.to_c()), int(prec),
                                             C.byref(make_fields(S_mass, S_mom, den, pairs)),
                                             _stream_handle(stream)))

    def cic_accumulate(self, mesh: fla_mesh, particles: fla_trajectories, weight: float, params: Params, S_mass,
                       S_mom, den=None, stream=None):
        st = _lib.cic_accumulate(self._h, C.byref(mesh), C.byref(particles), float(weight), C.byref(params.to_c()),
                                 C.byref(make_fields(S_mass, S_mom, den)), _stream_handle(stream))
        self._check(st)

    def profile_enable(self, on: bool = True):
        self._check(_lib.fla_profile_enable(self._h, int(bool(on))))

    def profile_read(self) -> dict:
        """{stage: (total_ms, launches)} since profiling was enabled."""
        p = fla_profile()
        self._check(_lib.fla_profile_read(self._h, C.byref(p)))
        return {PROFILE_STAGES[k]: (float(p.ms[k]), int(p.launches[k])) for k in range(8)}

    def set_plan(self, dim: int, prec: int, plan: int):
        self._check(_lib.fla_set_plan(self._h, dim, prec, plan))

    def get_plan(self, dim: int, prec: int) -> int:
        v = C.c_int()
        self._check(_lib.fla_get_plan(self._h, dim, prec, C.byref(v)))
        return int(v.value)

    def autotune(self, mesh: fla_mesh, traj: fla_trajectories, params: Params, S_mass, S_mom, den=None,
                 stream=None):
        """Time every gather plan code on these inputs, keep the fastest; returns the ms per code
        (GATHER_CONFIGS values, -1 for codes the dimension does not have)."""
        t = (C.c_double * GATHER_CONFIGS)()
        self._check(_lib.fla_autotune(self._h, C.byref(mesh), C.byref(traj), C.byref(params.to_c()),
                                      C.byref(make_fields(S_mass, S_mom, den)), _stream_handle(stream), t))
        return [float(v) for v in t]

    # -- learned bandwidth ------------------------------------------------------------
    def bandwidth_forward(self, mesh: fla_mesh, traj: fla_trajectories, theta, h_factor, z=None, o=None,
                          features=None, stream=None):
        self._check(_lib.fla_bandwidth_forward(self._h, C.byref(mesh), C.byref(traj), _ptr(theta), _ptr(h_factor),
                                               _ptr(z), _ptr(o), _ptr(features), _stream_handle(stream)))

    def project_backward(self, mesh: fla_mesh, traj: fla_trajectories, params: Params, S_mass, S_mom, den,
                         G_mass, G_mom, dL_dlogh, stream=None):
        self._check(_lib.fla_project_backward(self._h, C.byref(mesh), C.byref(traj), C.byref(params.to_c()),
                                              C.byref(make_fields(S_mass, S_mom, den)),
                                              C.byref(make_fields(G_mass, G_mom)), _ptr(dL_dlogh),
                                              _stream_handle(stream)))

    def bandwidth_backward(self, dim: int, theta, count: int, z, o, dL_dlogh, grad, stream=None):
        self._check(_lib.fla_bandwidth_backward(self._h, dim, _ptr(theta), int(count), _ptr(z), _ptr(o),
                                                _ptr(dL_dlogh), _ptr(grad), _stream_handle(stream)))

    def adam_step(self, theta, m, v, grad, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self._check(_lib.fla_adam_step(self._h, _ptr(theta), _ptr(m), _ptr(v), _ptr(grad), int(step), lr, beta1,
                                       beta2, eps, _stream_handle(stream)))

    def rel_l2_loss(self, channels: int, cells: int, prec: int, S: Sequence, R: Sequence, G: Sequence = None,
                    result=None, stream=None):
        """S, R, G: lists of channel planes (S_mass first).  result: float64 device tensor of
        1 + 2*channels entries (allocated if None); returned."""
        import torch
        if result is None:
            result = torch.empty(1 + 2 * channels, dtype=torch.float64, device=S[0].device)
        fs = make_fields(S[0], S[1:])
        fr = make_fields(R[0], R[1:])
        fg = make_fields(G[0], G[1:]) if G is not None else None
        self._check(_lib.fla_rel_l2_loss(self._h, channels, int(cells), prec, C.byref(fs), C.byref(fr),
                                         C.byref(fg) if fg is not None else None, _ptr(result),
                                         _stream_handle(stream)))
        return result

    def bandwidth_standardise(self, meshes: Sequence, trajs: Sequence, theta, stream=None):
        """Fit mu, sd of the parameter block (in place) over the snapshots."""
        n = len(meshes)
        if n == 0 or len(trajs) != n:
            raise ValueError("meshes and trajs must be non-empty and of equal length")
        Ms = (fla_mesh * n)(*meshes)
        Ts = (fla_trajectories * n)(*trajs)
        self._check(_lib.fla_bandwidth_standardise(self._h, n, Ms, Ts, _ptr(theta), _stream_handle(stream)))

    def mlp_train_step(self, mesh: fla_mesh, traj: fla_trajectories, params: Params, ref: Sequence, theta, m, v,
                       step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss=None, stream=None):
        """One training step in the library; ref: reference planes (S_mass first)."""
        self._check(_lib.fla_mlp_train_step(self._h, C.byref(mesh), C.byref(traj), C.byref(params.to_c()),
                                            C.byref(make_fields(ref[0], ref[1:])), _ptr(theta), _ptr(m), _ptr(v),
                                            int(step), lr, beta1, beta2, eps, _ptr(loss), _stream_handle(stream)))

    # -- batched snapshots --------------------------------------------------------------
    @staticmethod
    def _batch_arrays(meshes: Sequence, trajs: Sequence, params: Sequence, outs: Sequence):
        n = len(meshes)
        if not (len(trajs) == len(params) == len(outs) == n) or n == 0:
            raise ValueError("meshes, trajs, params and outs must be non-empty and of equal length")
        M = (fla_mesh * n)(*meshes)
        T = (fla_trajectories * n)(*trajs)
        P = (fla_params * n)(*[p.to_c() if isinstance(p, Params) else p for p in params])
        F = (fla_fields * n)(*[o if isinstance(o, fla_fields) else
                               make_fields(o[0], o[1], o[2] if len(o) > 2 else None, o[3] if len(o) > 3 else None)
                               for o in outs])
        return n, M, T, P, F

    def project_batch(self, meshes: Sequence, trajs: Sequence, params: Sequence, outs: Sequence, stream=None):
        """outs[s]: fla_fields or (S_mass, [S_mom...], den or None)."""
        n, M, T, P, F = self._batch_arrays(meshes, trajs, params, outs)
        self._check(_lib.fla_project_batch(self._h, n, M, T, P, F, _stream_handle(stream)))

    def save_plans(self, path: str):
        """Write the context's gather and batch plans (per dim, precision) for this device's architecture."""
        self._check(_lib.fla_save_plans(self._h, os.fsencode(path)))

    def load_plans(self, path: str):
        """Set the plans saved for this device's architecture; a bad file changes nothing."""
        self._check(_lib.fla_load_plans(self._h, os.fsencode(path)))

    def set_graph(self, enable: bool):
        """Capture and replay graphs of repeated identical fla_project_sources calls."""
        self._check(_lib.fla_set_graph(self._h, int(bool(enable))))

    def set_batch_graph(self, enable: bool):
        self._check(_lib.fla_set_batch_graph(self._h, int(bool(enable))))

    def set_batch_plan(self, dim: int, prec: int, plan: int, chunk: int = 16):
        self._check(_lib.fla_set_batch_plan(self._h, dim, prec, plan, chunk))

    def get_batch_plan(self, dim: int, prec: int) -> tuple:
        p, c = C.c_int(), C.c_int()
        self._check(_lib.fla_get_batch_plan(self._h, dim, prec, C.byref(p), C.byref(c)))
        return p.value, c.value

    def autotune_batch(self, meshes: Sequence, trajs: Sequence, params: Sequence, outs: Sequence,
                       stream=None) -> list:
        """Returns the gather time (ms) of every (plan code, chunk), code-major (-1: not tried)."""
        n, M, T, P, F = self._batch_arrays(meshes, trajs, params, outs)
        times = (C.c_double * (GATHER_CONFIGS * BATCH_CHUNKS))()
        self._check(_lib.fla_autotune_batch(self._h, n, M, T, P, F, _stream_handle(stream), times))
        return list(times)

    def stats(self) -> dict:
        s = fla_stats()
        self._check(_lib.fla_get_stats(self._h, C.byref(s)))
        return {k: int(getattr(s, k)) for k, _ in fla_stats._fields_}


def alloc_fields(M: int, dim: int, dtype, device="cuda", den: bool = True):
    """Allocate output planes: returns (S_mass, [S_mom...], den or None)."""
    import torch
    S_mass = torch.empty(M, dtype=dtype, device=device)
    S_mom = [torch.empty(M, dtype=dtype, device=device) for _ in range(dim)]
    d = torch.empty(M, dtype=dtype, device=device) if den else None
    return S_mass, S_mom, d
