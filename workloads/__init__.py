"""Seeded synthetic inputs for the FLA source projection and its PSI-CELL comparator.

This module is the only code shared by the oracle side and the GPU side.  It
produces *inputs* (trajectory positions, deformation Jacobians, velocities,
radii, particle clouds, meshes) and contains none of the projection's
arithmetic: no determinant, number density, smoothing length, source term,
kernel weight or average is evaluated here.

Random numbers come from a counter-based hash (murmur3's 32-bit finaliser
applied to (seed, stream, index)), written with int64 torch ops so that the
same seed gives bit-identical uniforms on the CPU and on a GPU.  Normal
variates use the Box-Muller transform; their last bits may differ between
devices (libm differs), which is harmless because every test generates its
inputs once and hands the same tensors to both sides.

Flow maps (the paper's cylinder case is not available, so analytic maps stand
in for the trajectory producer; each map is one step of length T = 1 s):

* Taylor-Green, 2-D, amplitude a on the unit square (non-periodic).
* ABC flow, 3-D, amplitude a, coefficients A, B, C, optional phases and
  wavenumber, on the periodic unit cube.
* multi-vortex: composition of two ABC maps (amplitudes 0.2 and 0.1,
  wavenumbers 1 and 2, seeded phases); its Jacobian is the chain-rule product.

For every map the droplet velocity is v = (x' - x)/T and the gas velocity is
the same field shape evaluated at x' with the map's amplitude in m/s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import torch

TWO_PI = 2.0 * math.pi
MASK32 = 0xFFFFFFFF

# Physical constants used by every configuration: water droplets in air.
RHO_D = 1000.0          # droplet density, kg/m^3
MU_AIR = 1.81e-5        # gas dynamic viscosity, Pa s
DELTA_EVAP = -1.0e-9    # rate of change of droplet surface area, m^2/s
N0_DEFAULT = 1.0e10     # initial number density, m^-3


# --------------------------------------------------------------------------
# counter-based random numbers
# --------------------------------------------------------------------------
def _fmix32(h: torch.Tensor) -> torch.Tensor:
    h = h & MASK32
    h = h ^ (h >> 16)
    h = (h * 0x85EBCA6B) & MASK32
    h = h ^ (h >> 13)
    h = (h * 0xC2B2AE35) & MASK32
    h = h ^ (h >> 16)
    return h


def _hash32(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    lo = idx & MASK32
    hi = (idx >> 32) & MASK32
    key = (seed * 0x9E3779B1 + stream * 0x7F4A7C15 + 0x632BE59B) & MASK32
    h = _fmix32(lo ^ key)
    h = _fmix32(h ^ hi ^ ((key * 0x27D4EB2F) & MASK32))
    return h


def counter_uniform(seed: int, stream: int, n: int, device="cpu", offset: int = 0) -> torch.Tensor:
    """n float64 uniforms in the open interval (0, 1), 53 random bits each."""
    idx = torch.arange(offset, offset + n, dtype=torch.int64, device=device)
    a = _hash32(seed, 2 * stream, idx) >> 5          # 27 bits
    b = _hash32(seed, 2 * stream + 1, idx) >> 6      # 26 bits
    m = (a << 26) | b                                # 53 bits
    return (m.to(torch.float64) + 0.5) * (1.0 / 9007199254740992.0)


def counter_normal(seed: int, stream: int, n: int, device="cpu", offset: int = 0) -> torch.Tensor:
    u1 = counter_uniform(seed, 2 * stream + 1000, n, device, offset)
    u2 = counter_uniform(seed, 2 * stream + 1001, n, device, offset)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(TWO_PI * u2)


# --------------------------------------------------------------------------
# meshes and seeding
# --------------------------------------------------------------------------
@dataclass
class Mesh:
    dim: int
    n: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    periodic: Tuple[bool, ...]

    @property
    def cells(self) -> int:
        c = 1
        for k in self.n:
            c *= k
        return c

    @property
    def cell_volume(self) -> float:
        v = 1.0
        for a in range(self.dim):
            v *= (self.hi[a] - self.lo[a]) / self.n[a]
        return v

    @property
    def domain_volume(self) -> float:
        v = 1.0
        for a in range(self.dim):
            v *= self.hi[a] - self.lo[a]
        return v


def unit_mesh(dim: int, n: int, periodic: bool) -> Mesh:
    return Mesh(dim, (n,) * dim, (0.0,) * dim, (1.0,) * dim, (periodic,) * dim)


@dataclass
class Cells:
    """A general mesh as the projection sees it: cell centroids (dim, M),
    binary64, in the mesh's own cell order, and cell volumes (M,).  Every
    centroid lies in the box [lo, hi]; axes flagged periodic repeat with
    period hi - lo."""
    dim: int
    centroids: torch.Tensor
    volume: torch.Tensor
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    periodic: Tuple[bool, ...]

    @property
    def count(self) -> int:
        return int(self.centroids.shape[1])

    @property
    def L(self) -> Tuple[float, ...]:
        return tuple(self.hi[a] - self.lo[a] for a in range(self.dim))

    def to(self, device) -> "Cells":
        return Cells(self.dim, self.centroids.to(device), self.volume.to(device), self.lo, self.hi, self.periodic)


def _tensor_cells(axes_c: Sequence[torch.Tensor], axes_w: Sequence[torch.Tensor], lo, hi, periodic) -> Cells:
    """Cells of the tensor product of per-axis centres and widths, linear
    order with axis 0 fastest (as the Cartesian meshes)."""
    dim = len(axes_c)
    gc = torch.meshgrid(*axes_c, indexing="ij")
    gw = torch.meshgrid(*axes_w, indexing="ij")
    flat = lambda g: g.permute(*reversed(range(dim))).reshape(-1)
    cen = torch.stack([flat(gc[a]) for a in range(dim)]).contiguous()
    vol = flat(gw[0]).clone()
    for a in range(1, dim):
        vol = vol * flat(gw[a])
    return Cells(dim, cen, vol.contiguous(), tuple(lo), tuple(hi), tuple(bool(p) for p in periodic))


def mesh_cells(mesh: Mesh) -> Cells:
    """The cells of a uniform Cartesian mesh as a general mesh: centres
    lo + (i + 1/2) w with w = (hi - lo)/n, formed in that order."""
    cs, ws = [], []
    for a in range(mesh.dim):
        w = (mesh.hi[a] - mesh.lo[a]) / mesh.n[a]
        t = (torch.arange(mesh.n[a], dtype=torch.float64) + 0.5) * w
        cs.append(mesh.lo[a] + t)
        ws.append(torch.full((mesh.n[a],), w, dtype=torch.float64))
    return _tensor_cells(cs, ws, mesh.lo, mesh.hi, mesh.periodic)


def stretched_edges(n: int, lo: float, hi: float, beta: float) -> torch.Tensor:
    """n + 1 cell edges on [lo, hi] clustered toward both ends (a tanh
    stretching of strength beta > 0, as for a wall-resolved channel)."""
    s = torch.linspace(-1.0, 1.0, n + 1, dtype=torch.float64)
    e = torch.tanh(beta * s) / math.tanh(beta)
    e = lo + (hi - lo) * 0.5 * (e + 1.0)
    e[0], e[-1] = lo, hi
    return e


def rectilinear_cells(edges: Sequence[torch.Tensor], periodic: Sequence[bool]) -> Cells:
    """A rectilinear (tensor-product, non-uniform) mesh from its per-axis
    cell edges: centroids at edge midpoints, volumes the width products."""
    cs = [0.5 * (e[:-1] + e[1:]) for e in edges]
    ws = [e[1:] - e[:-1] for e in edges]
    lo = tuple(float(e[0]) for e in edges)
    hi = tuple(float(e[-1]) for e in edges)
    return _tensor_cells(cs, ws, lo, hi, periodic)


def scattered_cells(dim: int, n: int, lo, hi, periodic, seed: int, jitter: float = 0.35) -> Cells:
    """An unstructured stand-in: the centres of an n^dim lattice each moved
    by up to `jitter` cells in every axis (kept inside the box), with
    volumes varying by a factor up to 2 around the lattice volume, listed
    in a seeded random order (an unstructured mesh has no lattice order)."""
    M = n ** dim
    base = mesh_cells(Mesh(dim, (n,) * dim, tuple(lo), tuple(hi), tuple(periodic)))
    cen = base.centroids.clone()
    for a in range(dim):
        w = (hi[a] - lo[a]) / n
        u = counter_uniform(seed, 60 + a, M, "cpu") * 2.0 - 1.0
        c = cen[a] + jitter * w * u
        cen[a] = c.clamp(min=lo[a], max=hi[a])
    vol = base.volume * (0.5 + 1.5 * counter_uniform(seed, 63, M, "cpu"))
    perm = torch.argsort(counter_uniform(seed, 64, M, "cpu"))
    return Cells(dim, cen[:, perm].contiguous(), vol[perm].contiguous(), tuple(lo), tuple(hi),
                 tuple(bool(p) for p in periodic))


def lattice(dim: int, per_axis: int, device="cpu") -> torch.Tensor:
    """Cell-centred lattice (i + 1/2)/L on the unit cube, shape (dim, L^dim);
    axis 0 varies fastest."""
    g = (torch.arange(per_axis, dtype=torch.float64, device=device) + 0.5) / per_axis
    grids = torch.meshgrid(*([g] * dim), indexing="ij")  # grids[a][i0, i1, ...]
    # flatten so that axis 0 is fastest: permute to (i_{d-1}, ..., i_0)
    out = [grids[a].permute(*reversed(range(dim))).reshape(-1) for a in range(dim)]
    return torch.stack(out)


def random_points(dim: int, n: int, seed: int, device="cpu", offset: int = 0) -> torch.Tensor:
    return torch.stack([counter_uniform(seed, 10 + a, n, device, offset) for a in range(dim)])


# --------------------------------------------------------------------------
# flow maps: each returns (x', J, ug) with J stored as (dim*dim, N), entry a*dim+b = dx'_a/dx0_b
# --------------------------------------------------------------------------
def taylor_green_map(x0: torch.Tensor, amp: float = 0.1):
    X, Y = x0[0], x0[1]
    k = TWO_PI
    sx, cx = torch.sin(k * X), torch.cos(k * X)
    sy, cy = torch.sin(k * Y), torch.cos(k * Y)
    xp = torch.stack([X + amp * sx * cy, Y - amp * cx * sy])
    ka = k * amp
    J = torch.stack([1.0 + ka * cx * cy, -ka * sx * sy,
                     ka * sx * sy, 1.0 - ka * cx * cy])
    sxp, cxp = torch.sin(k * xp[0]), torch.cos(k * xp[0])
    syp, cyp = torch.sin(k * xp[1]), torch.cos(k * xp[1])
    ug = torch.stack([amp * sxp * cyp, -amp * cxp * syp])   # m/s
    return xp, J, ug


@dataclass
class ABC:
    amp: float = 0.2
    A: float = 1.0
    B: float = 1.0
    C: float = 1.0
    k: float = 1.0              # wavenumber (periods per unit length)
    phase: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    def field(self, x: torch.Tensor) -> torch.Tensor:
        w = TWO_PI * self.k
        px, py, pz = self.phase
        X, Y, Z = x[0], x[1], x[2]
        return torch.stack([
            self.A * torch.sin(w * Z + pz) + self.C * torch.cos(w * Y + py),
            self.B * torch.sin(w * X + px) + self.A * torch.cos(w * Z + pz),
            self.C * torch.sin(w * Y + py) + self.B * torch.cos(w * X + px),
        ])

    def grad(self, x: torch.Tensor) -> torch.Tensor:
        """d field_a / d x_b as (9, N)."""
        w = TWO_PI * self.k
        px, py, pz = self.phase
        X, Y, Z = x[0], x[1], x[2]
        z = torch.zeros_like(X)
        return torch.stack([
            z, -self.C * w * torch.sin(w * Y + py), self.A * w * torch.cos(w * Z + pz),
            self.B * w * torch.cos(w * X + px), z, -self.A * w * torch.sin(w * Z + pz),
            -self.B * w * torch.sin(w * X + px), self.C * w * torch.cos(w * Y + py), z,
        ])

    def apply(self, x0: torch.Tensor):
        xp = x0 + self.amp * self.field(x0)
        G = self.grad(x0) * self.amp
        G[0] += 1.0
        G[4] += 1.0
        G[8] += 1.0
        return xp, G


def _matmul3(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    out = []
    for a in range(3):
        for b in range(3):
            out.append(A[3 * a] * B[b] + A[3 * a + 1] * B[3 + b] + A[3 * a + 2] * B[6 + b])
    return torch.stack(out)


def abc_map(x0: torch.Tensor, abc: ABC):
    xp, J = abc.apply(x0)
    ug = abc.amp * abc.field(xp)
    return xp, J, ug


def multi_vortex_map(x0: torch.Tensor, maps: Sequence[ABC]):
    x = x0
    J = None
    for m in maps:
        xn, G = m.apply(x)
        J = G if J is None else _matmul3(G, J)
        x = xn
    ug = sum(m.amp * m.field(x) for m in maps)
    return x, J, ug


def multi_vortex_default(seed: int = 0) -> List[ABC]:
    ph = counter_uniform(seed, 900, 6).tolist()
    return [ABC(amp=0.2, k=1.0, phase=tuple(TWO_PI * p for p in ph[:3])),
            ABC(amp=0.1, k=2.0, phase=tuple(TWO_PI * p for p in ph[3:]))]


def wrap_unit(x: torch.Tensor) -> torch.Tensor:
    return x - torch.floor(x)


# --------------------------------------------------------------------------
# trajectory sets
# --------------------------------------------------------------------------
@dataclass
class Trajectories:
    """Structure-of-arrays trajectory record (all float64 on `device`).

    x: (dim, N) positions; J: (dim*dim, N) deformation Jacobian, entry
    a*dim+b; v, ug: (dim, N) droplet and gas velocity; r: (N,) radius;
    n0: scalar initial number density (or (N,) tensor)."""
    x: torch.Tensor
    J: torch.Tensor
    v: torch.Tensor
    ug: torch.Tensor
    r: torch.Tensor
    n0: object = N0_DEFAULT
    seed_volume: float = 0.0

    @property
    def count(self) -> int:
        return int(self.r.shape[0])

    @property
    def dim(self) -> int:
        return int(self.x.shape[0])

    def to(self, device) -> "Trajectories":
        n0 = self.n0.to(device) if isinstance(self.n0, torch.Tensor) else self.n0
        return Trajectories(self.x.to(device), self.J.to(device), self.v.to(device),
                            self.ug.to(device), self.r.to(device), n0, self.seed_volume)

    def subset(self, idx: torch.Tensor) -> "Trajectories":
        n0 = self.n0[idx] if isinstance(self.n0, torch.Tensor) else self.n0
        return Trajectories(self.x[:, idx], self.J[:, idx], self.v[:, idx],
                            self.ug[:, idx], self.r[idx], n0, self.seed_volume)


def radius_uniform(n, seed, lo_um, hi_um, device="cpu", stream=50, offset=0):
    u = counter_uniform(seed, stream, n, device, offset)
    return (lo_um + (hi_um - lo_um) * u) * 1e-6


def radius_lognormal(n, seed, median_um=10.0, sigma=0.3, device="cpu", stream=51, offset=0):
    z = counter_normal(seed, stream, n, device, offset)
    return median_um * 1e-6 * torch.exp(sigma * z)


def from_map(x0: torch.Tensor, kind: str, params=None, wrap: bool = False):
    if kind == "tg":
        xp, J, ug = taylor_green_map(x0, **(params or {}))
    elif kind == "abc":
        xp, J, ug = abc_map(x0, params if params is not None else ABC())
    elif kind == "multi":
        xp, J, ug = multi_vortex_map(x0, params if params is not None else multi_vortex_default())
    else:
        raise ValueError(kind)
    v = xp - x0                         # one map step of T = 1 s
    if wrap:
        xp = wrap_unit(xp)
    return xp, J, v, ug


# --------------------------------------------------------------------------
# the benchmark configurations (sizes as stated by the workload definitions)
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    mesh: Mesh
    traj: Trajectories
    h0: float
    precision: str                  # "f64" or "f32"
    rho_d: float = RHO_D
    mu: float = MU_AIR
    delta: float = DELTA_EVAP
    cutoff: float = 4.0
    extra: Dict = field(default_factory=dict)


def taylor_green_2d(per_axis: int = 64, mesh_n: int = 64, seed: int = 0, device="cpu",
                    delta: float = DELTA_EVAP) -> Workload:
    """2-D FP64: unit square, Taylor-Green map amplitude 0.1, lattice seeding,
    r ~ U[5, 20] um, n0 = 1e10 m^-3, h0 = lattice pitch."""
    x0 = lattice(2, per_axis, device)
    xp, J, v, ug = from_map(x0, "tg", {"amp": 0.1})
    r = radius_uniform(x0.shape[1], seed, 5.0, 20.0, device)
    tr = Trajectories(xp, J, v, ug, r, N0_DEFAULT, seed_volume=1.0 / per_axis ** 2)
    return Workload("tg2d_f64", unit_mesh(2, mesh_n, False), tr, 1.0 / per_axis, "f64", delta=delta)


def taylor_green_cloud(n_particles: int = 400_000, seed: int = 0, device="cpu"):
    """PSI-CELL comparator cloud for the 2-D case: X0 ~ U[0,1]^2, same map and radius law."""
    x0 = random_points(2, n_particles, seed, device)
    xp, J, v, ug = from_map(x0, "tg", {"amp": 0.1})
    r = radius_uniform(n_particles, seed, 5.0, 20.0, device, stream=60)
    return Trajectories(xp, J, v, ug, r, 1.0)


def abc_lattice_3d(per_axis: int = 128, mesh_n: int = 128, seed: int = 0, device="cpu",
           amp: float = 0.2) -> Workload:
    """3-D: periodic unit cube, ABC map amplitude 0.2 (A=B=C=1), lattice seeding,
    r ~ lognormal(ln 10 um, 0.3), h0 = lattice pitch, FP32 kernel evaluation."""
    x0 = lattice(3, per_axis, device)
    xp, J, v, ug = from_map(x0, "abc", ABC(amp=amp), wrap=True)
    r = radius_lognormal(x0.shape[1], seed, device=device)
    tr = Trajectories(xp, J, v, ug, r, N0_DEFAULT, seed_volume=1.0 / per_axis ** 3)
    return Workload("abc3d_f32", unit_mesh(3, mesh_n, True), tr, 1.0 / per_axis, "f32")


def abc_cloud(n_particles: int, seed: int = 0, device="cpu", abc: Optional[ABC] = None,
              offset: int = 0, radius="lognormal", jacobian: bool = True):
    """Dense PSI-CELL cloud: X0 ~ U[0,1)^3 through the ABC map.  With
    jacobian=False the (unused) Jacobian is not formed and J is empty."""
    x0 = random_points(3, n_particles, seed, device, offset)
    abc = abc if abc is not None else ABC()
    if jacobian:
        xp, J, v, ug = from_map(x0, "abc", abc, wrap=True)
    else:
        xp = x0 + abc.amp * abc.field(x0)
        v = xp - x0
        del x0
        ug = abc.amp * abc.field(xp)
        xp = wrap_unit(xp)
        J = torch.empty(0, dtype=torch.float64, device=device)
    if radius == "lognormal":
        r = radius_lognormal(n_particles, seed, device=device, stream=61, offset=offset)
    else:
        r = radius_uniform(n_particles, seed, 5.0, 20.0, device, stream=61, offset=offset)
    return Trajectories(xp, J, v, ug, r, 1.0)


def multi_vortex_cloud(n_particles: int, seed: int = 0, device="cpu", maps: Optional[Sequence[ABC]] = None,
                       offset: int = 0):
    """Dense PSI-CELL cloud: X0 ~ U[0,1)^3 through the multi-vortex map (the
    composition of the given ABC maps, same positions and velocities as
    multi_vortex_map), radius lognormal; no Jacobian."""
    maps = maps if maps is not None else multi_vortex_default()
    x0 = random_points(3, n_particles, seed, device, offset)
    x = x0
    for m in maps:
        x = x + m.amp * m.field(x)
    v = x - x0
    del x0
    ug = sum(m.amp * m.field(x) for m in maps)
    r = radius_lognormal(n_particles, seed, device=device, stream=61, offset=offset)
    return Trajectories(wrap_unit(x), torch.empty(0, dtype=torch.float64, device=device), v, ug, r, 1.0)


def multi_vortex_lattice_3d(per_axis: int = 320, mesh_n: int = 256, seed: int = 0, device="cpu") -> Workload:
    x0 = lattice(3, per_axis, device)
    xp, J, v, ug = from_map(x0, "multi", multi_vortex_default(seed), wrap=True)
    r = radius_lognormal(x0.shape[1], seed, device=device)
    tr = Trajectories(xp, J, v, ug, r, N0_DEFAULT, seed_volume=1.0 / per_axis ** 3)
    return Workload("multivortex3d_f32", unit_mesh(3, mesh_n, True), tr, 1.0 / per_axis, "f32")


def uneven_snapshot(s: int, device="cpu") -> Workload:
    """One snapshot of the uneven batch: edge L = round(32*4^u), N = round(1e4*200^u'),
    random seeding, ABC amplitude U[0.05, 0.2] with random phases, h0 = N^(-1/3)."""
    u = counter_uniform(1000 + s, 0, 6)
    L = int(round(32 * 4 ** float(u[0])))
    N = int(round(1e4 * 200 ** float(u[1])))
    amp = 0.05 + 0.15 * float(u[2])
    abc = ABC(amp=amp, phase=(TWO_PI * float(u[3]), TWO_PI * float(u[4]), TWO_PI * float(u[5])))
    x0 = random_points(3, N, 1000 + s, device)
    xp, J, v, ug = from_map(x0, "abc", abc, wrap=True)
    r = radius_lognormal(N, 1000 + s, device=device)
    tr = Trajectories(xp, J, v, ug, r, N0_DEFAULT, seed_volume=1.0 / N)
    return Workload(f"uneven_snap{s}", unit_mesh(3, L, True), tr, N ** (-1.0 / 3.0), "f32")


def training_snapshot(s: int, n_traj: int = 200_000, mesh_n: int = 64, device="cpu") -> Tuple[Workload, ABC]:
    """Training snapshot: random seeding, ABC with A,B,C ~ U[0.5,1.5], amplitude
    U[0.05,0.25], random phases; h0 = N^(-1/3)."""
    u = counter_uniform(2000 + s, 0, 7)
    abc = ABC(amp=0.05 + 0.2 * float(u[0]), A=0.5 + float(u[1]), B=0.5 + float(u[2]),
              C=0.5 + float(u[3]),
              phase=(TWO_PI * float(u[4]), TWO_PI * float(u[5]), TWO_PI * float(u[6])))
    x0 = random_points(3, n_traj, 2000 + s, device)
    xp, J, v, ug = from_map(x0, "abc", abc, wrap=True)
    r = radius_lognormal(n_traj, 2000 + s, device=device)
    tr = Trajectories(xp, J, v, ug, r, N0_DEFAULT, seed_volume=1.0 / n_traj)
    return Workload(f"training_snap{s}", unit_mesh(3, mesh_n, True), tr, n_traj ** (-1.0 / 3.0), "f32"), abc


def small_random_3d(n_traj: int, mesh_n: int, seed: int, device="cpu", periodic=True,
                    amp: float = 0.2, h0: Optional[float] = None) -> Workload:
    """Small 3-D case for parity tests: random seeding through an ABC map."""
    x0 = random_points(3, n_traj, seed, device)
    xp, J, v, ug = from_map(x0, "abc", ABC(amp=amp), wrap=periodic)
    r = radius_lognormal(n_traj, seed, device=device)
    tr = Trajectories(xp, J, v, ug, r, N0_DEFAULT, seed_volume=1.0 / n_traj)
    return Workload(f"rand3d_{n_traj}_{mesh_n}", unit_mesh(3, mesh_n, periodic), tr,
                    h0 if h0 is not None else n_traj ** (-1.0 / 3.0), "f32")


# ---------------------------------------------------------------------------
# Droplet seeds for the trajectory producer (initial state only: the
# integration and the gas field belong to the method)
@dataclass
class Droplets:
    """Initial droplet state (float64): x, v (dim, N); J = I, dJ (dim*dim, N);
    r (N,); scalar n0; seed volume."""
    x: torch.Tensor
    v: torch.Tensor
    J: torch.Tensor
    dJ: torch.Tensor
    r: torch.Tensor
    n0: float
    seed_volume: float

    @property
    def count(self) -> int:
        return int(self.r.shape[0])

    def to(self, device) -> "Droplets":
        return Droplets(self.x.to(device), self.v.to(device), self.J.to(device), self.dJ.to(device),
                        self.r.to(device), self.n0, self.seed_volume)

    def clone(self) -> "Droplets":
        return Droplets(self.x.clone(), self.v.clone(), self.J.clone(), self.dJ.clone(), self.r.clone(), self.n0,
                        self.seed_volume)


def seed_droplets(dim: int, per_axis: int, seed: int = 0, device="cpu", speed: float = 0.2,
                  radius: str = "lognormal", jitter: float = 0.0) -> Droplets:
    """Droplets on the cell-centred lattice of the unit square/cube (optionally
    jittered by up to `jitter` pitches), injected with a velocity that does not
    depend on position (uniform random per droplet, |v_a| <= speed), so that
    dJ = dv0/dx0 = 0 and J = I at seeding; radius lognormal(ln 10 um, 0.3) or
    U[5, 20] um."""
    x0 = lattice(dim, per_axis, device)
    N = x0.shape[1]
    if jitter > 0.0:
        x0 = x0 + (counter_uniform(seed, 60, N * dim, device).reshape(dim, N) - 0.5) * (jitter / per_axis)
    v0 = (counter_uniform(seed, 61, N * dim, device).reshape(dim, N) * 2.0 - 1.0) * speed
    J = torch.eye(dim, dtype=torch.float64, device=device).reshape(dim * dim, 1).repeat(1, N).contiguous()
    dJ = torch.zeros((dim * dim, N), dtype=torch.float64, device=device)
    r = radius_lognormal(N, seed, device=device) if radius == "lognormal" else \
        radius_uniform(N, seed, 5.0, 20.0, device)
    return Droplets(x0.contiguous(), v0.contiguous(), J, dJ, r.to(torch.float64).contiguous(), N0_DEFAULT,
                    1.0 / N)


# ---------------------------------------------------------------------------
# Table 1 of the paper (simulation parameters): droplet density and radius
# (SI), carrier kinematic viscosity, Stokes number, carrier density 1, for
# the non-evaporating and evaporating cases at Re = 20 and Re = 100.
TABLE1 = [
    {"case": "non-evaporating Re=20", "rho_d": 2500.0, "r_d": 0.003, "nu": 0.05, "St": 0.1, "evaporating": False},
    {"case": "non-evaporating Re=100", "rho_d": 2000.0, "r_d": 0.0015, "nu": 0.01, "St": 0.1, "evaporating": False},
    {"case": "evaporating Re=20", "rho_d": 2500.0, "r_d": 0.003, "nu": 0.05, "St": 0.1, "evaporating": True},
    {"case": "evaporating Re=100", "rho_d": 2500.0, "r_d": 0.003, "nu": 0.01, "St": 0.5, "evaporating": True},
]
TABLE1_RHO_F = 1.0


def table1_droplets(column: int, n: int, seed: int = 0, device="cpu", lattice_seeding: bool = True,
                    offset: int = 0) -> Droplets:
    """Monodisperse droplets of a Table 1 column at rest on the periodic unit
    square (J = I, dJ = 0): n = per-axis count of a cell-centred lattice, or
    the number of uniform random positions (counter-hash stream, `offset`
    for disjoint sub-clouds)."""
    c = TABLE1[column]
    if lattice_seeding:
        x0 = lattice(2, n, device)
    else:
        x0 = random_points(2, n, seed, device, offset)
    N = x0.shape[1]
    J = torch.eye(2, dtype=torch.float64, device=device).reshape(4, 1).repeat(1, N).contiguous()
    z = torch.zeros((2, N), dtype=torch.float64, device=device)
    return Droplets(x0.contiguous(), z.clone(), J, torch.zeros((4, N), dtype=torch.float64, device=device),
                    torch.full((N,), c["r_d"], dtype=torch.float64, device=device), N0_DEFAULT, 1.0 / N)
