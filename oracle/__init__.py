"""FP64 CPU oracle for the FLA source projection (test infrastructure only).

This package is the plain, slow, obviously correct reference that the GPU
library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
it shares no code with the GPU library.

The arithmetic lives in ``fla_oracle.c`` (binary64, no fused multiply-add,
OpenMP over cells); this module marshals numpy arrays into it.  The learned
bandwidth form and its gradients are in ``oracle.learned`` (numpy, binary64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fla_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class OrcMesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("periodic", C.c_int * 3)]


class OrcFlow(C.Structure):
    _fields_ = [("kind", C.c_int), ("U", C.c_double), ("k", C.c_double), ("abc", C.c_double * 3),
                ("phase", C.c_double * 3), ("u0", C.c_double * 3), ("G", C.c_double * 9)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_int64)


def _declare(L):
    L.orc_det.restype = C.c_double
    L.orc_det.argtypes = [C.c_int, _dp]
    L.orc_droplet_phi.restype = None
    L.orc_droplet_phi.argtypes = [C.c_int, C.c_double, _dp, _dp, C.c_double, C.c_double,
                                  C.c_double, _dp, _dp, _dp, _dp]
    L.orc_trajectory_terms.restype = C.c_int64
    L.orc_trajectory_terms.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp,
                                       C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, _dp, _dp, _dp, _dp, _dp, _ip]
    L.orc_nw_cells.restype = None
    L.orc_nw_cells.argtypes = [C.POINTER(OrcMesh), C.c_int64, _dp, _dp, _dp, _ip, C.c_double,
                               C.c_int, C.c_double, _dp, C.c_int64, _lp, _dp, _dp, _lp]
    L.orc_nw_points.restype = None
    L.orc_nw_points.argtypes = [C.c_int, C.c_int64, _dp, _ip, _dp, C.c_int64, _dp, _dp, _dp, _ip, C.c_double,
                                C.c_int, C.c_double, _dp, C.c_int64, _lp, _dp, _dp, _lp]
    L.orc_nw_box.restype = C.c_int
    L.orc_nw_box.argtypes = [C.POINTER(OrcMesh), C.c_int64, _dp, _dp, _dp, _ip, C.c_double, C.c_int,
                             C.c_double, _dp, _lp, _lp, _dp, _dp, _lp]
    L.orc_box_cells.restype = None
    L.orc_box_cells.argtypes = [C.POINTER(OrcMesh), _lp, _lp, _lp]
    L.orc_deposit_scatter.restype = None
    L.orc_deposit_scatter.argtypes = [C.POINTER(OrcMesh), C.c_int64, _dp, _dp, _dp, _dp, _ip,
                                      C.c_double, C.c_double, C.c_int, C.c_double, _dp, _dp, _dp]
    L.orc_deposit.restype = None
    L.orc_deposit.argtypes = [C.POINTER(OrcMesh), C.c_int64, _dp, _dp, _dp, _dp, _ip,
                              C.c_double, C.c_double, C.c_int, C.c_double, _dp, _dp, _dp]
    L.orc_psicell.restype = C.c_int64
    L.orc_psicell.argtypes = [C.POINTER(OrcMesh), C.c_int64, _dp, _dp, _dp, _dp, C.c_double,
                              C.c_double, C.c_double, C.c_double, _dp, _dp, _lp, _lp]
    L.orc_cic.restype = C.c_int64
    L.orc_cic.argtypes = [C.POINTER(OrcMesh), C.c_int64, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                          C.c_double, _dp, _dp, _dp, _lp]
    L.orc_psicell_cell_of.restype = C.c_int64
    L.orc_psicell_cell_of.argtypes = [C.POINTER(OrcMesh), _dp]
    L.orc_flow_eval.restype = None
    L.orc_flow_eval.argtypes = [C.c_int, C.POINTER(OrcFlow), _dp, _dp, _dp]
    L.orc_advance.restype = C.c_int64
    L.orc_advance.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp, _dp, C.POINTER(OrcFlow), C.c_double,
                              C.c_double, C.c_double, C.c_double, C.c_int, _dp, _ip]
    L.orc_state_terms.restype = C.c_int64
    L.orc_state_terms.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _ip, _dp, C.c_double, C.c_double, _dp, _dp,
                                  _dp, _dp, _ip]
    L.orc_app_a_scaling.restype = None
    L.orc_app_a_scaling.argtypes = [C.c_double] * 7 + [_dp]
    L.orc_num_threads.restype = C.c_int
    L.orc_num_threads.argtypes = []
    L.orc_set_threads.restype = None
    L.orc_set_threads.argtypes = [C.c_int]


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_mesh(dim: int, n: Sequence[int], lo: Sequence[float], hi: Sequence[float],
              periodic: Sequence[bool]) -> OrcMesh:
    m = OrcMesh()
    m.dim = dim
    for a in range(3):
        m.n[a] = int(n[a]) if a < dim else 1
        m.lo[a] = float(lo[a]) if a < dim else 0.0
        m.hi[a] = float(hi[a]) if a < dim else 1.0
        m.periodic[a] = int(bool(periodic[a])) if a < dim else 0
    return m


def mesh_from(w) -> OrcMesh:
    """Accept a ``workloads.Mesh``-like object."""
    return make_mesh(w.dim, w.n, w.lo, w.hi, w.periodic)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------------------
def det(J: np.ndarray) -> float:
    J = _f64(J).reshape(-1)
    dim = 2 if J.size == 4 else 3
    return float(lib().orc_det(dim, _d(J)))


def droplet_phi(dim: int, r: float, v, ug, rho_d: float, mu: float, delta: float):
    """Returns (phi, m, tau, mdot) for one droplet."""
    v = _f64(v)
    ug = _f64(ug)
    phi = np.zeros(4)
    m = np.zeros(1)
    tau = np.zeros(1)
    md = np.zeros(1)
    lib().orc_droplet_phi(dim, float(r), _d(v), _d(ug), rho_d, mu, delta, _d(phi), _d(m),
                          _d(tau), _d(md))
    return phi[:1 + dim].copy(), float(m[0]), float(tau[0]), float(md[0])


@dataclass
class Terms:
    det: np.ndarray
    h: np.ndarray
    n: np.ndarray
    q: np.ndarray       # (C, N)
    valid: np.ndarray   # (N,) int32
    skipped: int


def trajectory_terms(traj, rho_d: float, mu: float, delta: float, h0: float,
                     h_factor: Optional[np.ndarray] = None) -> Terms:
    """det J, n = n0/|det J|, h = h0 |det J| (x factor), q = n * phi per trajectory."""
    dim = traj.dim if hasattr(traj, "dim") else int(np.asarray(traj["x"]).shape[0])
    x, J, v, ug, r = (_f64(traj.x), _f64(traj.J), _f64(traj.v), _f64(traj.ug), _f64(traj.r))
    N = r.shape[0]
    n0 = traj.n0
    n0_arr = None
    n0_s = 0.0
    if hasattr(n0, "shape") and np.ndim(_f64(n0)) == 1:
        n0_arr = _f64(n0)
    else:
        n0_s = float(n0)
    hf = _f64(h_factor) if h_factor is not None else None
    det_ = np.zeros(N)
    h = np.zeros(N)
    n = np.zeros(N)
    q = np.zeros((1 + dim, N))
    valid = np.zeros(N, dtype=np.int32)
    sk = lib().orc_trajectory_terms(dim, N, _d(x), _d(J), _d(v), _d(ug), _d(r),
                                    _d(n0_arr) if n0_arr is not None else None, n0_s, rho_d,
                                    mu, delta, h0, _d(hf) if hf is not None else None,
                                    _d(det_), _d(h), _d(n), _d(q),
                                    valid.ctypes.data_as(_ip))
    return Terms(det_, h, n, q, valid, int(sk))


@dataclass
class Projection:
    S: np.ndarray        # (C, ncells)
    den: np.ndarray      # (ncells,)
    pairs: np.ndarray    # (ncells,) int64


def nw_cells(mesh, x, terms: Terms, cells: Optional[np.ndarray] = None, cutoff: float = 4.0,
             f32_decision: bool = False, scale: float = 1.0,
             cell_scale: Optional[np.ndarray] = None) -> Projection:
    """Nadaraya-Watson source terms at the listed cells (all cells if None)."""
    m = mesh if isinstance(mesh, OrcMesh) else mesh_from(mesh)
    dim = m.dim
    M = int(np.prod([m.n[a] for a in range(dim)]))
    if cells is None:
        cells = np.arange(M, dtype=np.int64)
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    x = _f64(x)
    N = x.shape[1]
    S = np.zeros((1 + dim, cells.size))
    den = np.zeros(cells.size)
    pairs = np.zeros(cells.size, dtype=np.int64)
    cs = _f64(cell_scale) if cell_scale is not None else None
    lib().orc_nw_cells(C.byref(m), N, _d(x), _d(terms.h), _d(np.ascontiguousarray(terms.q)),
                       terms.valid.ctypes.data_as(_ip), cutoff, int(bool(f32_decision)), scale,
                       _d(cs) if cs is not None else None, cells.size,
                       cells.ctypes.data_as(_lp), _d(S), _d(den), pairs.ctypes.data_as(_lp))
    return Projection(S, den, pairs)


def nw_points(cells, x, terms: Terms, sel: Optional[np.ndarray] = None, cutoff: float = 4.0,
              f32_decision: bool = False, scale: float = 1.0,
              cell_scale: Optional[np.ndarray] = None) -> Projection:
    """Nadaraya-Watson source terms at the centroids of a general mesh
    (``workloads.Cells``-like: dim, centroids (dim, M), lo, hi, periodic),
    at the listed cells (all if None), by brute force over trajectories."""
    dim = cells.dim
    xc = _f64(cells.centroids)
    M = xc.shape[1]
    per = np.ascontiguousarray([int(bool(cells.periodic[a])) if a < dim else 0 for a in range(3)], dtype=np.int32)
    L = np.ascontiguousarray([float(cells.hi[a]) - float(cells.lo[a]) if a < dim else 1.0 for a in range(3)])
    sel = np.arange(M, dtype=np.int64) if sel is None else np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    x = _f64(x)
    N = x.shape[1]
    S = np.zeros((1 + dim, sel.size))
    den = np.zeros(sel.size)
    pairs = np.zeros(sel.size, dtype=np.int64)
    cs = _f64(cell_scale) if cell_scale is not None else None
    lib().orc_nw_points(dim, M, _d(xc), per.ctypes.data_as(_ip), _d(L), N, _d(x), _d(terms.h),
                        _d(np.ascontiguousarray(terms.q)), terms.valid.ctypes.data_as(_ip), cutoff,
                        int(bool(f32_decision)), scale, _d(cs) if cs is not None else None, sel.size,
                        sel.ctypes.data_as(_lp), _d(S), _d(den), pairs.ctypes.data_as(_lp))
    return Projection(S, den, pairs)


@dataclass
class BoxProjection:
    S: np.ndarray        # (C, B) in box order
    den: np.ndarray      # (B,)
    pairs: np.ndarray    # (B,) int64
    cells: np.ndarray    # (B,) linear mesh index of each box cell


def nw_box(mesh, x, terms: Terms, box_lo: Optional[Sequence[int]] = None,
           box_n: Optional[Sequence[int]] = None, cutoff: float = 4.0, f32_decision: bool = False,
           scale: float = 1.0, cell_scale: Optional[np.ndarray] = None) -> BoxProjection:
    """Nadaraya-Watson source terms on a box of cells by the trajectory-centric
    scatter (each trajectory visits the bounding box of its cutoff sphere).
    The box starts at cell box_lo and spans box_n cells per axis, wrapping
    across periodic boundaries; the default is the whole mesh.  Bit for bit
    the result of ``nw_cells`` on the same cells."""
    m = mesh if isinstance(mesh, OrcMesh) else mesh_from(mesh)
    dim = m.dim
    lo = np.zeros(3, dtype=np.int64)
    bn = np.ones(3, dtype=np.int64)
    for a in range(dim):
        lo[a] = int(box_lo[a]) if box_lo is not None else 0
        bn[a] = int(box_n[a]) if box_n is not None else m.n[a]
    B = int(np.prod(bn))
    x = _f64(x)
    N = x.shape[1]
    S = np.zeros((1 + dim, B))
    den = np.zeros(B)
    pairs = np.zeros(B, dtype=np.int64)
    cells = np.zeros(B, dtype=np.int64)
    cs = _f64(cell_scale) if cell_scale is not None else None
    rc = lib().orc_nw_box(C.byref(m), N, _d(x), _d(terms.h), _d(np.ascontiguousarray(terms.q)),
                          terms.valid.ctypes.data_as(_ip), cutoff, int(bool(f32_decision)), scale,
                          _d(cs) if cs is not None else None, lo.ctypes.data_as(_lp),
                          bn.ctypes.data_as(_lp), _d(S), _d(den), pairs.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError(f"box {lo[:dim]} + {bn[:dim]} does not fit the mesh")
    lib().orc_box_cells(C.byref(m), lo.ctypes.data_as(_lp), bn.ctypes.data_as(_lp), cells.ctypes.data_as(_lp))
    return BoxProjection(S, den, pairs, cells)


def deposit_scatter(mesh, x, terms: Terms, seed_volume: float, cutoff: float = 4.0,
                    f32_decision: bool = False, scale: float = 1.0,
                    cell_scale: Optional[np.ndarray] = None):
    """Trajectory-centric form of ``deposit`` (bit for bit the same result);
    returns (S (C, M), Z (N,))."""
    m = mesh if isinstance(mesh, OrcMesh) else mesh_from(mesh)
    dim = m.dim
    M = int(np.prod([m.n[a] for a in range(dim)]))
    x = _f64(x)
    N = x.shape[1]
    S = np.zeros((1 + dim, M))
    Z = np.zeros(N)
    cs = _f64(cell_scale) if cell_scale is not None else None
    lib().orc_deposit_scatter(C.byref(m), N, _d(x), _d(terms.h), _d(np.ascontiguousarray(terms.q)),
                              _d(terms.det), terms.valid.ctypes.data_as(_ip), seed_volume, cutoff,
                              int(bool(f32_decision)), scale, _d(cs) if cs is not None else None,
                              _d(S), _d(Z))
    return S, Z


def deposit(mesh, x, terms: Terms, seed_volume: float, cutoff: float = 4.0,
            f32_decision: bool = False, scale: float = 1.0,
            cell_scale: Optional[np.ndarray] = None):
    """Normalised-kernel deposition; returns (S (C, M), Z (N,))."""
    m = mesh if isinstance(mesh, OrcMesh) else mesh_from(mesh)
    dim = m.dim
    M = int(np.prod([m.n[a] for a in range(dim)]))
    x = _f64(x)
    N = x.shape[1]
    S = np.zeros((1 + dim, M))
    Z = np.zeros(N)
    cs = _f64(cell_scale) if cell_scale is not None else None
    lib().orc_deposit(C.byref(m), N, _d(x), _d(terms.h), _d(np.ascontiguousarray(terms.q)),
                      _d(terms.det), terms.valid.ctypes.data_as(_ip), seed_volume, cutoff,
                      int(bool(f32_decision)), scale, _d(cs) if cs is not None else None,
                      _d(S), _d(Z))
    return S, Z


def psicell(mesh, cloud, weight: float, rho_d: float, mu: float, delta: float,
            cell_scale: Optional[np.ndarray] = None, split: bool = False):
    """PSI-CELL box counting; returns (S (C, M), counts (M,), skipped), or with
    split (S, counts, outside, nonfinite): particles outside a closed box and
    particles with a non-finite input."""
    m = mesh if isinstance(mesh, OrcMesh) else mesh_from(mesh)
    dim = m.dim
    M = int(np.prod([m.n[a] for a in range(dim)]))
    x, v, ug, r = _f64(cloud.x), _f64(cloud.v), _f64(cloud.ug), _f64(cloud.r)
    Np = r.shape[0]
    S = np.zeros((1 + dim, M))
    counts = np.zeros(M, dtype=np.int64)
    cs = _f64(cell_scale) if cell_scale is not None else None
    nf = np.zeros(1, dtype=np.int64)
    sk = lib().orc_psicell(C.byref(m), Np, _d(x), _d(v), _d(ug), _d(r), rho_d, mu, delta,
                           weight, _d(cs) if cs is not None else None, _d(S),
                           counts.ctypes.data_as(_lp), nf.ctypes.data_as(_lp))
    if split:
        return S, counts, int(sk) - int(nf[0]), int(nf[0])
    return S, counts, int(sk)


def cic(mesh, cloud, weight: float, rho_d: float, mu: float, delta: float,
        cell_scale: Optional[np.ndarray] = None):
    """Cloud-in-cell accumulation; returns (S (C, M), weight sums (M,),
    outside, nonfinite)."""
    m = mesh if isinstance(mesh, OrcMesh) else mesh_from(mesh)
    dim = m.dim
    M = int(np.prod([m.n[a] for a in range(dim)]))
    x, v, ug, r = _f64(cloud.x), _f64(cloud.v), _f64(cloud.ug), _f64(cloud.r)
    Np = r.shape[0]
    S = np.zeros((1 + dim, M))
    ws = np.zeros(M)
    cs = _f64(cell_scale) if cell_scale is not None else None
    nf = np.zeros(1, dtype=np.int64)
    sk = lib().orc_cic(C.byref(m), Np, _d(x), _d(v), _d(ug), _d(r), rho_d, mu, delta, weight,
                       _d(cs) if cs is not None else None, _d(S), _d(ws), nf.ctypes.data_as(_lp))
    return S, ws, int(sk) - int(nf[0]), int(nf[0])


def psicell_cell_of(mesh, xp) -> int:
    m = mesh if isinstance(mesh, OrcMesh) else mesh_from(mesh)
    xp = _f64(list(xp) + [0.0] * (3 - len(xp)))
    return int(lib().orc_psicell_cell_of(C.byref(m), _d(xp)))


def app_a_scaling(N_ref, tau_ref, N_fla, tau_fla, V_cell, A_inj, v_inj):
    out = np.zeros(3)
    lib().orc_app_a_scaling(N_ref, tau_ref, N_fla, tau_fla, V_cell, A_inj, v_inj, _d(out))
    return float(out[0]), float(out[1]), float(out[2])


def nhat_cells(volume, N_ref, tau_ref, A_inj, v_inj, N_fla=1.0, tau_fla=1.0) -> np.ndarray:
    """Per-cell factor n_hat = M_scal V_scal of App. A (eqs. mass-load-scaling,
    vscal-def, vfla, vinj, dinj), formed from the two factors separately; the
    FLA seeding parameters N_fla and tau_fla cancel in the product."""
    vol = _f64(volume)
    out = np.empty_like(vol)
    for c in range(vol.size):
        out[c] = app_a_scaling(N_ref, tau_ref, N_fla, tau_fla, float(vol[c]), A_inj, v_inj)[2]
    return out


def project_points(cells, traj, rho_d, mu, delta, h0, cutoff=4.0, f32_decision=False, scale=1.0,
                   cell_scale=None, sel=None, h_factor=None):
    """Whole plain path on a general mesh: terms, then the estimator at the
    listed centroids (all by default)."""
    t = trajectory_terms(traj, rho_d, mu, delta, h0, h_factor)
    return nw_points(cells, traj.x, t, sel, cutoff, f32_decision, scale, cell_scale), t


def project_box(mesh, traj, rho_d, mu, delta, h0, cutoff=4.0, f32_decision=False, scale=1.0,
                cell_scale=None, box_lo=None, box_n=None, h_factor=None):
    """Whole plain path by the trajectory-centric scatter: terms, then the
    estimator on a box of cells (the whole mesh by default)."""
    t = trajectory_terms(traj, rho_d, mu, delta, h0, h_factor)
    return nw_box(mesh, traj.x, t, box_lo, box_n, cutoff, f32_decision, scale, cell_scale), t


def project(mesh, traj, rho_d, mu, delta, h0, cutoff=4.0, f32_decision=False, scale=1.0,
            cell_scale=None, cells=None, h_factor=None):
    """Whole plain path: terms, then the estimator at all (or listed) cells."""
    t = trajectory_terms(traj, rho_d, mu, delta, h0, h_factor)
    return nw_cells(mesh, traj.x, t, cells, cutoff, f32_decision, scale, cell_scale), t


# ---------------------------------------------------------------------------
# Trajectory producer (eqs. Stokes-drag, evap-model, Jacobian-evolution; App. B 1a-1b)
FLOW_NONE, FLOW_TAYLOR_GREEN, FLOW_ABC = 0, 1, 2


def make_flow(kind: int = FLOW_NONE, U: float = 0.0, k: float = 1.0, abc=(1.0, 1.0, 1.0), phase=(0.0, 0.0, 0.0),
              u0=(0.0, 0.0, 0.0), G=None) -> OrcFlow:
    """Gas field u = u0 + G x + (Taylor-Green or ABC part of amplitude U and wavenumber k)."""
    f = OrcFlow()
    f.kind, f.U, f.k = int(kind), float(U), float(k)
    pad = lambda t: list(t) + [0.0] * (3 - len(t))
    abc, phase, u0 = pad(abc), pad(phase), pad(u0)
    for a in range(3):
        f.abc[a], f.phase[a], f.u0[a] = float(abc[a]), float(phase[a]), float(u0[a])
    Gm = np.zeros((3, 3)) if G is None else np.asarray(G, dtype=np.float64)
    Gp = np.zeros((3, 3))
    Gp[:Gm.shape[0], :Gm.shape[1]] = Gm
    for e in range(9):
        f.G[e] = float(Gp.reshape(-1)[e])
    return f


def flow_eval(dim: int, flow: OrcFlow, x):
    """(u (dim,), grad u (dim, dim)) at one point."""
    xv = _f64(list(x) + [0.0] * (3 - len(x)))
    u = np.zeros(3)
    gu = np.zeros(dim * dim)
    lib().orc_flow_eval(dim, C.byref(flow), _d(xv), _d(u), _d(gu))
    return u[:dim].copy(), gu.reshape(dim, dim)


@dataclass
class DropletState:
    """Binary64 state planes: x, v (dim, N); J, K = dJ/dt (dim*dim, N), entry a*dim+b; r (N,)."""
    x: np.ndarray
    v: np.ndarray
    J: np.ndarray
    K: np.ndarray
    r: np.ndarray

    @property
    def dim(self):
        return self.x.shape[0]

    def copy(self):
        return DropletState(self.x.copy(), self.v.copy(), self.J.copy(), self.K.copy(), self.r.copy())


def advance(state: DropletState, flow: OrcFlow, rho_d: float, mu: float, delta: float, dt: float,
            substeps: int):
    """Advance a copy of the state by dt (RK4, `substeps` substeps); returns
    (new state, phibar (1 + dim, N) source rates of the step, valid (N,), skipped)."""
    st = DropletState(*(np.ascontiguousarray(np.array(a, dtype=np.float64)) for a in
                        (state.x, state.v, state.J, state.K, state.r)))
    dim, N = st.x.shape
    phibar = np.zeros((1 + dim, N))
    valid = np.zeros(N, dtype=np.int32)
    sk = lib().orc_advance(dim, N, _d(st.x), _d(st.v), _d(st.J), _d(st.K), _d(st.r), C.byref(flow), rho_d, mu,
                           delta, dt, int(substeps), _d(phibar), valid.ctypes.data_as(_ip))
    return st, phibar, valid, int(sk)


def state_terms(state: DropletState, phibar: np.ndarray, valid: np.ndarray, n0, h0: float) -> Terms:
    """Estimator terms of advanced droplets (q = n * phibar)."""
    dim, N = state.x.shape
    n0_arr = _f64(n0) if np.ndim(n0) == 1 else None
    det_ = np.zeros(N)
    h = np.zeros(N)
    n = np.zeros(N)
    q = np.zeros((1 + dim, N))
    vout = np.zeros(N, dtype=np.int32)
    vin = np.ascontiguousarray(valid, dtype=np.int32)
    sk = lib().orc_state_terms(dim, N, _d(_f64(state.x)), _d(_f64(state.J)), _d(_f64(phibar)),
                               vin.ctypes.data_as(_ip), _d(n0_arr) if n0_arr is not None else None,
                               0.0 if n0_arr is not None else float(n0), h0, _d(det_), _d(h), _d(n), _d(q),
                               vout.ctypes.data_as(_ip))
    return Terms(det_, h, n, q, vout, int(sk))
