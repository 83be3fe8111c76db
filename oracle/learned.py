"""FP64 oracle of the learned bandwidth correction and of its gradients.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The learned form multiplies the smoothing length of eq. (smoothing-length),
h_i = h0 |det J_i|, by a per-trajectory factor predicted from the local
deformation:

  features  f_i = [log s1, log s2, log s3, log(n_i/n0_i), log(1 + N_nbr,i)]
            (s_k the singular values of J_i, largest first; N_nbr the number of
            valid trajectories whose home cell lies in the 3^d block of cells
            around trajectory i's home cell, i itself included);
  inputs    z = (f - mu) / sd, rounded to bfloat16;
  network   a1 = W1 z + b1, h1 = bf16(silu(a1)); a2 = W2 h1 + b2,
            h2 = silu(a2); o = w3 . h2 + b3, with W1, W2, w3 rounded to bf16
            (the products are exact; sums in binary64 here);
  factor    g = exp(s_max tanh o), s_max = ln 4.

Training minimises L = sum_k |S_k - R_k|^2 / |R_k|^2 over the source
channels against a reference field R (dense PSI-CELL).  With the estimator
S_kc = -scale cs_c N_kc / D_c, N_kc = sum_i K_ci q_ik, D_c = sum_i K_ci and
K = (1/h) exp(-s/2), s = |x_c - x_i|^2 / h^2:

  dK/dh = (K / h) (s - 1)
  dL/dh_i = sum_c (K_ci / h_i)(s_ci - 1) a_c (sum_k g_kc q_ik - sum_k g_kc N_kc / D_c),
            g_kc = dL/dS_kc = 2 (S_kc - R_kc) / |R_k|^2,  a_c = -scale cs_c / D_c,

over the included pairs (the truncation radius moves with h; its boundary
term is of the order of the kernel tail exp(-c^2/2) and is ignored).  Then
dL/do_i = dL/dh_i * h_i * s_max * (1 - tanh^2 o_i) and the network gradient
follows by the chain rule.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

S_MAX = math.log(4.0)
HIDDEN = 64
N_FEAT = 5
# parameter block layout (float32 on the device, float64 here)
LAYOUT = [("W1", (HIDDEN, N_FEAT)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("w3", (HIDDEN,)), ("b3", (1,)), ("mu", (N_FEAT,)), ("sd", (N_FEAT,))]
N_TRAIN = 4609          # trainable entries (W1 .. b3)
N_PARAM = N_TRAIN + 2 * N_FEAT


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in LAYOUT])


def bf16(x: np.ndarray) -> np.ndarray:
    """Round binary32 values of x to bfloat16 (round to nearest, ties to even),
    returned as float64.  x is first rounded to binary32."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    r = r.astype(np.uint32).view(np.float32)
    r = np.where(nan, np.float32(np.nan), r)
    return r.astype(np.float64)


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def init_params(seed: int = 0, mu=None, sd=None) -> np.ndarray:
    """He-style random W1, W2 (standard normal scaled by sqrt(2/fan_in)),
    zero biases, zero last layer (so the initial factor is exactly 1)."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.standard_normal((HIDDEN, N_FEAT)) * math.sqrt(2.0 / N_FEAT),
        "b1": np.zeros(HIDDEN),
        "W2": rng.standard_normal((HIDDEN, HIDDEN)) * math.sqrt(2.0 / HIDDEN),
        "b2": np.zeros(HIDDEN),
        "w3": np.zeros(HIDDEN),
        "b3": np.zeros(1),
        "mu": np.zeros(N_FEAT) if mu is None else np.asarray(mu, float),
        "sd": np.ones(N_FEAT) if sd is None else np.asarray(sd, float),
    }
    return pack(p).astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------- features
def home_cells(mesh, x: np.ndarray) -> np.ndarray:
    """Cell of each point: floor((x - lo)/dx) per axis, wrapped on periodic
    axes, clamped on closed ones; returned as per-axis indices (dim, N)."""
    dim = mesh.dim
    idx = np.zeros((dim, x.shape[1]), dtype=np.int64)
    for a in range(dim):
        w = (mesh.hi[a] - mesh.lo[a]) / mesh.n[a]
        g = np.floor((x[a] - mesh.lo[a]) / w).astype(np.int64)
        if mesh.periodic[a]:
            g = np.mod(g, mesh.n[a])
        else:
            g = np.clip(g, 0, mesh.n[a] - 1)
        idx[a] = g
    return idx


def neighbour_counts(mesh, x: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """N_nbr: valid trajectories with home cell in the 3^d block around each
    trajectory's home cell (cells outside a closed box do not exist)."""
    dim = mesh.dim
    idx = home_cells(mesh, x)
    n = list(mesh.n[:dim])
    grid = np.zeros(n[::-1], dtype=np.int64)          # [z][y][x] or [y][x]
    v = valid.astype(bool)
    np.add.at(grid, tuple(idx[a][v] for a in reversed(range(dim))), 1)
    out = np.zeros(x.shape[1], dtype=np.int64)
    offs = np.array(np.meshgrid(*([[-1, 0, 1]] * dim), indexing="ij")).reshape(dim, -1).T
    for o in offs:
        j = idx + o[:, None]
        ok = np.ones(x.shape[1], dtype=bool)
        for a in range(dim):
            if mesh.periodic[a]:
                j[a] = np.mod(j[a], mesh.n[a])
            else:
                ok &= (j[a] >= 0) & (j[a] < mesh.n[a])
                j[a] = np.clip(j[a], 0, mesh.n[a] - 1)
        out += np.where(ok, grid[tuple(j[a] for a in reversed(range(dim)))], 0)
    return out


def features(mesh, x: np.ndarray, J: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """(N_FEAT, N) features; rows of skipped trajectories are zero.  For 2-D
    meshes the third singular value is taken as 1 (log = 0)."""
    dim = mesh.dim
    N = x.shape[1]
    v = valid.astype(bool)
    Jm = np.moveaxis(J.reshape(dim, dim, N), 2, 0)         # (N, dim, dim), row-major a*dim+b
    # a skipped trajectory's J may be non-finite, which the SVD cannot take;
    # its features are zero whatever stands in for it
    Jm = np.where(v[:, None, None], Jm, np.eye(dim))
    s = np.linalg.svd(Jm, compute_uv=False)                 # descending
    f = np.zeros((N_FEAT, N))
    for k in range(dim):
        f[k] = np.log(s[:, k])
    adet = np.abs(np.linalg.det(Jm))
    f[3] = -np.log(adet)                                    # log(n / n0) = -log|det J| (eq. FLA-COM)
    f[4] = np.log1p(neighbour_counts(mesh, x, valid))
    f[:, ~v] = 0.0
    return f


# ----------------------------------------------------------------- network
@dataclass
class Forward:
    z: np.ndarray      # (5, N) bf16-rounded inputs
    a1: np.ndarray
    h1: np.ndarray     # bf16-rounded
    a2: np.ndarray
    h2: np.ndarray
    o: np.ndarray
    g: np.ndarray      # bandwidth factor


def forward(theta: np.ndarray, f: np.ndarray, round_bf16: bool = True) -> Forward:
    """The network; round_bf16=False skips the bfloat16 roundings (used to
    check the chain rule against finite differences)."""
    rnd = bf16 if round_bf16 else (lambda t: np.asarray(t, dtype=np.float64))
    p = unpack(theta)
    z = rnd(((f - p["mu"][:, None]) / p["sd"][:, None]))
    W1, W2, w3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["w3"])
    a1 = W1 @ z + p["b1"][:, None]
    h1 = rnd(silu(a1))
    a2 = W2 @ h1 + p["b2"][:, None]
    h2 = silu(a2)
    o = w3 @ h2 + p["b3"][0]
    g = np.exp(S_MAX * np.tanh(o))
    return Forward(z, a1, h1, a2, h2, o, g)


def backward(theta: np.ndarray, fw: Forward, dL_do: np.ndarray, round_bf16: bool = True) -> np.ndarray:
    """Gradient of L with respect to the trainable entries (W1 .. b3), laid
    out as the parameter block (zeros for mu, sd)."""
    rnd = bf16 if round_bf16 else (lambda t: np.asarray(t, dtype=np.float64))
    p = unpack(theta)
    W2, w3 = rnd(p["W2"]), rnd(p["w3"])
    g = {}
    g["w3"] = fw.h2 @ dL_do
    g["b3"] = np.array([dL_do.sum()])
    d2 = np.outer(w3, dL_do) * dsilu(fw.a2)
    g["W2"] = d2 @ fw.h1.T
    g["b2"] = d2.sum(axis=1)
    d1 = (W2.T @ d2) * dsilu(fw.a1)
    g["W1"] = d1 @ fw.z.T
    g["b1"] = d1.sum(axis=1)
    g["mu"] = np.zeros(N_FEAT)
    g["sd"] = np.zeros(N_FEAT)
    return pack(g)


def dL_do_from_dL_dh(dL_dh: np.ndarray, h: np.ndarray, o: np.ndarray) -> np.ndarray:
    return dL_dh * h * S_MAX * (1.0 - np.tanh(o) ** 2)


# ----------------------------------------------------------------- loss and d/dh
def rel_l2_loss(S: np.ndarray, R: np.ndarray):
    """L = sum_k |S_k - R_k|^2 / |R_k|^2 and dL/dS."""
    nr = np.sum(R * R, axis=1, keepdims=True)
    d = S - R
    return float(np.sum(np.sum(d * d, axis=1, keepdims=True) / nr)), 2.0 * d / nr


def dL_dh(mesh, x: np.ndarray, h: np.ndarray, q: np.ndarray, valid: np.ndarray, S: np.ndarray,
          den: np.ndarray, dL_dS: np.ndarray, cutoff: float = 4.0, scale: float = 1.0,
          cell_scale: Optional[np.ndarray] = None) -> np.ndarray:
    """Analytic dL/dh_i of the estimator (binary64 inclusion test), by brute
    force over all cells for every trajectory."""
    dim = mesh.dim
    N = x.shape[1]
    M = int(np.prod(mesh.n[:dim]))
    cs = np.ones(M) if cell_scale is None else np.asarray(cell_scale, float)
    idx = np.stack(np.unravel_index(np.arange(M), tuple(mesh.n[:dim][::-1])))[::-1]   # (dim, M), axis 0 fastest
    xc = np.zeros((dim, M))
    for a in range(dim):
        w = (mesh.hi[a] - mesh.lo[a]) / mesh.n[a]
        xc[a] = mesh.lo[a] + (idx[a] + 0.5) * w
    with np.errstate(divide="ignore", invalid="ignore"):
        a_c = np.where(den > 0, -scale * cs / den, 0.0)
        Shat = np.where(den > 0, S / (-scale * cs), 0.0)        # N_kc / D_c
    b = a_c[None, :] * dL_dS                                  # (C, M)
    e = a_c * np.sum(dL_dS * Shat, axis=0)                    # (M,)
    out = np.zeros(N)
    for i in range(N):
        if not valid[i]:
            continue
        s = np.zeros(M)
        for a in range(dim):
            d = xc[a] - x[a, i]
            if mesh.periodic[a]:
                L = mesh.hi[a] - mesh.lo[a]
                d = d - L * np.rint(d / L)
            s += (d / h[i]) ** 2
        inc = s <= cutoff * cutoff
        K = np.exp(-0.5 * s[inc]) / h[i]
        G = q[:, i] @ b[:, inc] - e[inc]
        out[i] = np.sum((K / h[i]) * (s[inc] - 1.0) * G)
    return out


# ----------------------------------------------------------------- optimiser
def adam(theta: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float = 1e-3,
         b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step on the trainable entries (step counts from 1)."""
    t = theta.copy()
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    upd = lr * mh / (np.sqrt(vh) + eps)
    t[:N_TRAIN] -= upd[:N_TRAIN]
    return t, m, v
