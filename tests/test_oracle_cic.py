"""Pins of the oracle's cloud-in-cell (CIC) accumulation.

CIC shares each particle among the 2^d cell centres around it with per-axis
hat weights 1 - |d|/dx: the weights sum to one and reproduce linear
functions (the first moment sum_c W_c x_c equals the particle position), a
particle at a cell centre deposits into that cell alone, and one halfway
between two centres splits evenly.  These fix the weights independently of
how the oracle forms them."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

RHO, MU, DELTA = W.RHO_D, W.MU_AIR, W.DELTA_EVAP


def _cloud(x, r=None, v=None, ug=None):
    x = torch.as_tensor(np.asarray(x, dtype=np.float64))
    dim, N = x.shape
    v = torch.zeros((dim, N), dtype=torch.float64) if v is None else torch.as_tensor(v, dtype=torch.float64)
    ug = torch.full((dim, N), 0.1, dtype=torch.float64) if ug is None else torch.as_tensor(ug, dtype=torch.float64)
    r = torch.full((N,), 1e-5, dtype=torch.float64) if r is None else torch.as_tensor(r, dtype=torch.float64)
    return W.Trajectories(x, torch.empty(0, dtype=torch.float64), v, ug, r, 1.0)


def _weights(mesh, xp):
    """The CIC weights of one particle, read off the weight sums."""
    _, ws, out, nf = oracle.cic(mesh, _cloud(np.asarray(xp, dtype=float).reshape(-1, 1)), 1.0, RHO, MU, DELTA)
    assert out == 0 and nf == 0
    return ws


def _centres(mesh):
    ax = [(np.arange(mesh.n[a]) + 0.5) * (mesh.hi[a] - mesh.lo[a]) / mesh.n[a] + mesh.lo[a] for a in range(mesh.dim)]
    g = np.meshgrid(*ax, indexing="ij")
    return [gi.transpose(*range(mesh.dim)[::-1]).reshape(-1) for gi in g]   # linear order: axis 0 fastest


def test_centre_and_midpoint():
    mesh = W.Mesh(2, (8, 6), (0.0, 0.0), (1.0, 1.5), (False, True))
    ws = _weights(mesh, [2.5 / 8, 3.5 * 0.25])            # the centre of cell (2, 3)
    assert ws[2 + 8 * 3] == pytest.approx(1.0, abs=1e-15) and ws.sum() == pytest.approx(1.0, abs=1e-15)
    ws = _weights(mesh, [3.0 / 8, 3.5 * 0.25])            # halfway between (2, 3) and (3, 3)
    np.testing.assert_allclose(ws[[2 + 24, 3 + 24]], [0.5, 0.5], rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_weights_reproduce_linear_functions(dim):
    n = (7, 9, 5)[:dim]
    mesh = W.Mesh(dim, n, (0.0,) * dim, (1.0,) * dim, (False,) * dim)
    cx = _centres(mesh)
    rng = np.random.default_rng(dim)
    for _ in range(20):
        # interior: at least half a cell from every wall
        xp = [rng.uniform(0.5 / n[a], 1 - 0.5 / n[a]) for a in range(dim)]
        ws = _weights(mesh, xp)
        assert ws.sum() == pytest.approx(1.0, abs=1e-14)
        assert (ws >= 0).all() and np.count_nonzero(ws) <= 2 ** dim
        for a in range(dim):
            assert (ws * cx[a]).sum() == pytest.approx(xp[a], abs=1e-14)


def test_periodic_wrap_and_closed_wall():
    mesh = W.Mesh(2, (10, 10), (0.0, 0.0), (1.0, 1.0), (True, False))
    # 0.02 from lo on the periodic axis: centres 0.05 (cell 0) and -0.05 (cell 9's image)
    ws = _weights(mesh, [0.02, 0.55])
    np.testing.assert_allclose(ws[[0 + 50, 9 + 50]], [0.7, 0.3], rtol=1e-12)
    # 0.02 from the closed wall at y = 1: everything in the last row along y
    ws = _weights(mesh, [0.6, 0.98])
    np.testing.assert_allclose(ws[[5 + 90, 6 + 90]], [0.5, 0.5], rtol=1e-12)
    assert ws.sum() == pytest.approx(1.0, abs=1e-15)


def test_conservation_and_agreement_with_psicell_at_centres():
    mesh = W.Mesh(3, (6, 5, 4), (0.0, 0.0, 0.0), (1.2, 1.0, 0.8), (True, False, True))
    rng = np.random.default_rng(3)
    N = 500
    x = np.stack([rng.uniform(0, 1.2, N), rng.uniform(0, 1.0, N), rng.uniform(0, 0.8, N)])
    cl = _cloud(x, r=rng.uniform(5e-6, 20e-6, N), v=rng.normal(size=(3, N)) * 0.1)
    S, ws, out, nf = oracle.cic(mesh, cl, 7.0, RHO, MU, DELTA)
    Sp, counts, sk = oracle.psicell(mesh, cl, 7.0, RHO, MU, DELTA)
    V = 0.2 ** 3
    np.testing.assert_allclose(S.sum(axis=1) * V, Sp.sum(axis=1) * V, rtol=1e-12)   # both deposit all of phi
    assert ws.sum() == pytest.approx(N, rel=1e-14)
    # particles at cell centres: CIC is PSI-CELL
    cx = _centres(mesh)
    pick = rng.choice(mesh.cells, 60)
    xc = np.stack([cx[a][pick] for a in range(3)])
    clc = _cloud(xc, r=rng.uniform(5e-6, 20e-6, 60))
    S1, _, _, _ = oracle.cic(mesh, clc, 1.0, RHO, MU, DELTA)
    S2, _, _ = oracle.psicell(mesh, clc, 1.0, RHO, MU, DELTA)
    np.testing.assert_allclose(S1, S2, rtol=1e-12, atol=1e-14 * np.abs(S2).max())   # centres rounded to a few ulps


def test_skips():
    mesh = W.Mesh(2, (4, 4), (0.0, 0.0), (1.0, 1.0), (False, True))
    x = np.array([[0.5, 1.5, 0.5, 1.0], [0.5, 0.5, 1.7, 0.3]])   # outside x; y wraps; x == hi is inside
    r = np.array([1e-5, 1e-5, 1e-5, np.nan])
    S, ws, out, nf = oracle.cic(mesh, _cloud(x, r=r), 1.0, RHO, MU, DELTA)
    assert out == 1 and nf == 1 and ws.sum() == pytest.approx(2.0)
