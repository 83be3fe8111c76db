"""Pins of the oracle's estimator on general meshes (cells given by their
centroids and volumes) and of the per-cell App. A factor n_hat.

The kernel estimator needs nothing of a cell but the point where it is
evaluated, so: centroids placed at a Cartesian mesh's cell centres reproduce
the (separately pinned) Cartesian oracle bit for bit; a refined mesh that
keeps some coarse centres reproduces the coarse values there; a field whose
every trajectory carries the same amounts is reproduced exactly; the
minimum image across a periodic boundary gives the closed-form weight; and
n_hat = V_cell N_ref/(A_inj v_inj tau_ref) (eq. mv-scal) multiplies each
cell's terms."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

RHO, MU, DELTA = W.RHO_D, W.MU_AIR, W.DELTA_EVAP


def _terms(wl):
    return oracle.trajectory_terms(wl.traj, wl.rho_d, wl.mu, wl.delta, wl.h0)


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("dim,periodic", [(3, True), (3, False), (2, False), (2, True)])
def test_lattice_centroids_reproduce_the_cartesian_oracle(dim, periodic, f32):
    if dim == 3:
        wl = W.small_random_3d(700, 9, seed=41, periodic=periodic, h0=0.03)
    else:
        wl = W.taylor_green_2d(per_axis=24, mesh_n=18, seed=42)
        wl.mesh = W.Mesh(2, (18, 13), (0.0, 0.0), (1.0, 0.9), (periodic, periodic))
    t = _terms(wl)
    cells = W.mesh_cells(wl.mesh)
    a = oracle.nw_cells(wl.mesh, wl.traj.x, t, f32_decision=f32, scale=1.7)
    b = oracle.nw_points(cells, wl.traj.x, t, f32_decision=f32, scale=1.7)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.den, b.den) and np.array_equal(a.pairs, b.pairs)
    assert b.pairs.sum() > 0


def test_refined_mesh_keeps_coarse_values_at_shared_centres():
    """Each coarse cell split into three along every axis: the middle
    sub-cell has the coarse centre (to rounding), and the estimator there
    is the coarse value; the estimator is meshfree."""
    wl = W.small_random_3d(600, 6, seed=43, periodic=True, h0=0.05)
    t = _terms(wl)
    n = 6
    edges = []
    for a in range(3):
        e = torch.linspace(0.0, 1.0, 3 * n + 1, dtype=torch.float64)
        edges.append(e)
    fine = W.rectilinear_cells(edges, (True, True, True))
    coarse = oracle.nw_points(W.mesh_cells(wl.mesh), wl.traj.x, t)
    mid = np.arange(n) * 3 + 1
    sel = (mid[None, None, :] + 3 * n * (mid[None, :, None] + 3 * n * mid[:, None, None])).reshape(-1)
    fr = oracle.nw_points(fine, wl.traj.x, t, sel=sel)
    np.testing.assert_allclose(fr.S, coarse.S, rtol=1e-11, atol=1e-11 * np.abs(coarse.S).max())
    np.testing.assert_allclose(fr.den, coarse.den, rtol=1e-11)


def test_uniform_amounts_are_reproduced_with_sign_and_scales():
    cells = W.scattered_cells(3, 7, (0.0, 0.0, 0.0), (1.0, 1.2, 0.8), (True, False, True), seed=44)
    N = 300
    rng = np.random.default_rng(5)
    x = np.stack([rng.uniform(0, 1.0, N), rng.uniform(0, 1.2, N), rng.uniform(0, 0.8, N)])
    qv = np.array([2.5, -1.0, 0.25, 4.0])
    t = oracle.Terms(np.ones(N), rng.uniform(0.03, 0.2, N), np.ones(N), np.tile(qv[:, None], (1, N)),
                     np.ones(N, dtype=np.int32), 0)
    cs = rng.uniform(0.5, 3.0, cells.count)
    p = oracle.nw_points(cells, x, t, scale=0.6, cell_scale=cs)
    hit = p.den > 0
    assert hit.sum() > 0.9 * cells.count
    np.testing.assert_allclose(p.S[:, hit], -0.6 * cs[hit][None, :] * qv[:, None], rtol=1e-13)
    assert np.all(p.S[:, ~hit] == 0.0)


def test_minimum_image_weight_across_a_periodic_boundary():
    """One trajectory at (0.02, 0.5) with h = 0.04: a centroid at (0.97, 0.52)
    of a periodic unit box is 0.05 away along x through the boundary, and a
    closed box sees 0.95 (outside the cutoff)."""
    x = np.array([[0.02], [0.5]])
    h = 0.04
    t = oracle.Terms(np.ones(1), np.array([h]), np.ones(1), np.array([[1.0], [0.0], [0.0]]),
                     np.ones(1, dtype=np.int32), 0)
    cen = torch.tensor([[0.97, 0.5], [0.52, 0.9]], dtype=torch.float64)
    for per, expect in ((True, math.exp(-(0.05 ** 2 + 0.02 ** 2) / (2 * h * h)) / h), (False, 0.0)):
        cells = W.Cells(2, cen, torch.ones(2, dtype=torch.float64), (0.0, 0.0), (1.0, 1.0), (per, per))
        p = oracle.nw_points(cells, x, t)
        assert p.den[0] == pytest.approx(expect, rel=1e-12, abs=0.0)
        assert p.den[1] == 0.0 and p.pairs[1] == 0          # 0.4 along y: beyond 4 h


def test_nhat_is_the_cell_volume_times_the_reference_injection_rate():
    vol = np.array([1e-9, 3.5e-9, 2e-10])
    N_ref, tau_ref, A, v = 5.0e4, 2e-3, 1e-4, 3.0
    for N_fla, tau_fla in ((50.0, 0.02), (7.0, 1e-4)):
        nh = oracle.nhat_cells(vol, N_ref, tau_ref, A, v, N_fla=N_fla, tau_fla=tau_fla)
        np.testing.assert_allclose(nh, vol * N_ref / (A * v * tau_ref), rtol=1e-14)
    # the mass-flow form (eq. mv-scal-massflow) with mdot_ref = N_ref m / tau_ref
    m = 4.0 / 3.0 * math.pi * RHO * (12e-6) ** 3
    mdot = N_ref * m / tau_ref
    np.testing.assert_allclose(vol * mdot / (A * v * m), nh, rtol=1e-14)


def test_scattered_and_stretched_generators():
    c = W.scattered_cells(3, 8, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (True, True, False), seed=1)
    assert c.count == 512 and (c.volume > 0).all()
    for a in range(3):
        assert float(c.centroids[a].min()) >= 0.0 and float(c.centroids[a].max()) <= 1.0
    e = W.stretched_edges(32, 0.0, 2.0, 2.0)
    w = e[1:] - e[:-1]
    assert float(e[0]) == 0.0 and float(e[-1]) == 2.0 and (w > 0).all() and float(w.max() / w.min()) > 5
    r = W.rectilinear_cells([e, W.stretched_edges(10, -1.0, 1.0, 1.5)], (False, True))
    assert r.count == 320 and float(r.volume.sum()) == pytest.approx(4.0, rel=1e-13)
