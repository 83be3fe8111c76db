"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a closed form, a
special value, an invariant, a printed table, or agreement with an
independent method, chosen so that a plausible mistake (a dropped term, a
wrong sign or index, a transposed operand, a wrong power of h) fails one.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RHO, MU, DELTA = W.RHO_D, W.MU_AIR, W.DELTA_EVAP


class T:
    """Minimal trajectory record for hand-built cases."""

    def __init__(self, x, J=None, v=None, ug=None, r=None, n0=1.0):
        self.x = np.asarray(x, dtype=np.float64)
        dim, N = self.x.shape
        self.J = np.asarray(J, dtype=np.float64) if J is not None else \
            np.tile(np.eye(dim).reshape(-1, 1), (1, N))
        self.v = np.asarray(v, dtype=np.float64) if v is not None else np.zeros((dim, N))
        self.ug = np.asarray(ug, dtype=np.float64) if ug is not None else np.zeros((dim, N))
        self.r = np.asarray(r, dtype=np.float64) if r is not None else np.full(N, 1e-5)
        self.n0 = n0

    @property
    def dim(self):
        return self.x.shape[0]


def _terms_from(h, q, x):
    N = x.shape[1]
    return oracle.Terms(det=np.ones(N), h=np.asarray(h, float), n=np.ones(N),
                        q=np.ascontiguousarray(np.asarray(q, float)),
                        valid=np.ones(N, dtype=np.int32), skipped=0)


def _mesh(dim, n, periodic=False):
    return oracle.make_mesh(dim, [n] * dim, [0.0] * dim, [1.0] * dim, [periodic] * dim)


# ---------------------------------------------------------------- determinant
def test_det_triangular_and_permutation():
    rng = np.random.default_rng(1)
    for dim in (2, 3):
        for _ in range(20):
            A = np.triu(rng.normal(size=(dim, dim)))
            assert oracle.det(A) == pytest.approx(np.prod(np.diag(A)), rel=1e-14)
            B = np.tril(rng.normal(size=(dim, dim)))
            assert oracle.det(B) == pytest.approx(np.prod(np.diag(B)), rel=1e-14)
    # permutation matrices: sign of the permutation
    perms3 = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (1, 0, 2): -1, (0, 2, 1): -1, (2, 1, 0): -1}
    for p, s in perms3.items():
        P = np.eye(3)[list(p)]
        assert oracle.det(P) == s
    assert oracle.det(np.array([[0.0, 1.0], [1.0, 0.0]])) == -1.0


def test_det_rotation_times_stretch():
    rng = np.random.default_rng(2)
    for _ in range(50):
        a, b, c = rng.uniform(0, 2 * np.pi, 3)
        Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
        Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
        Rx = np.array([[1, 0, 0], [0, np.cos(c), -np.sin(c)], [0, np.sin(c), np.cos(c)]])
        s = rng.uniform(-3, 3, 3)
        M = Rz @ Ry @ Rx @ np.diag(s)
        assert oracle.det(M) == pytest.approx(np.prod(s), rel=1e-12, abs=1e-14)
        # the determinant of a product is the product of determinants
        N = rng.normal(size=(3, 3))
        assert oracle.det(M @ N) == pytest.approx(oracle.det(M) * oracle.det(N), rel=1e-10, abs=1e-13)


def test_det_taylor_green_closed_form():
    """det J of the Taylor-Green map with amplitude a is
    1 - (2 pi a)^2 cos(2 pi (x+y)) cos(2 pi (x-y))."""
    x0 = W.lattice(2, 16)
    _, J, _ = W.taylor_green_map(x0, 0.1)
    J = J.numpy()
    x, y = x0[0].numpy(), x0[1].numpy()
    ka = 2 * np.pi * 0.1
    ref = 1 - ka ** 2 * np.cos(2 * np.pi * (x + y)) * np.cos(2 * np.pi * (x - y))
    got = np.array([oracle.det(J[:, i].reshape(2, 2)) for i in range(x.size)])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)


def test_det_abc_lattice_mean_is_one():
    """The ABC map is a degree-one map of the periodic cube, so the lattice mean
    of det J (a midpoint rule, exact for these trigonometric polynomials) is 1."""
    x0 = W.lattice(3, 24)
    _, J, _ = W.abc_map(x0, W.ABC(amp=0.2))
    t = oracle.trajectory_terms(W.Trajectories(x0, J, x0 * 0, x0 * 0, torch.full((x0.shape[1],), 1e-5)),
                                RHO, MU, DELTA, 1.0)
    assert t.det.mean() == pytest.approx(1.0, abs=1e-12)
    assert (t.det < 0).any()  # folds are present


# ---------------------------------------------------------------- physics
def test_table1_stokes_number():
    """Eq. 5 with U/L = 1 and mu = rho_f nu gives the printed St of Table 1;
    the oracle's relaxation time tau = 2 rho_d r^2/(9 mu) equals St there."""
    with open(os.path.join(GOLDEN, "table1_parameters.json")) as f:
        t1 = json.load(f)
    for rho_d, r, nu, st in zip(t1["rho_d"], t1["r_d"], t1["nu"], t1["St"]):
        mu = t1["rho_f"] * nu
        _, _, tau, _ = oracle.droplet_phi(2, r, [0, 0], [0, 0], rho_d, mu, 0.0)
        assert tau == pytest.approx(st, rel=1e-12)


def test_drag_is_stokes_law():
    """F = m (u_g - v)/tau must equal Stokes' drag 6 pi mu r (u_g - v)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        r = rng.uniform(1e-6, 1e-4)
        v, ug = rng.normal(size=3), rng.normal(size=3)
        phi, _, _, _ = oracle.droplet_phi(3, r, v, ug, RHO, MU, 0.0)
        np.testing.assert_allclose(phi[1:], 6 * np.pi * MU * r * (ug - v), rtol=1e-12)


def test_evaporation_rate_matches_mass_derivative():
    """mdot equals d/dt of (4/3) pi rho r^3 along rdot = delta/(2r) (eq. 4),
    checked by a central difference of the droplet mass."""
    for r in (5e-6, 2e-5, 1e-3):
        delta = -3e-9
        _, _, _, mdot = oracle.droplet_phi(3, r, [0, 0, 0], [0, 0, 0], RHO, MU, delta)
        dt = 1e-6 * r * r / abs(delta)
        mass = lambda t: 4.0 / 3.0 * np.pi * RHO * (r * r + delta * t) ** 1.5  # r^2 = r0^2 + delta t
        fd = (mass(dt) - mass(-dt)) / (2 * dt)
        assert mdot == pytest.approx(fd, rel=1e-6)
        assert mdot < 0


def test_momentum_channel_includes_evaporative_term():
    """S_Mom carries F + mdot v (eq. coupling-terms-specification)."""
    r, v, ug = 1e-5, np.array([0.3, -0.2, 0.1]), np.array([0.0, 0.0, 0.0])
    phi0, _, _, _ = oracle.droplet_phi(3, r, v, ug, RHO, MU, 0.0)
    phi1, _, _, mdot = oracle.droplet_phi(3, r, v, ug, RHO, MU, -1e-9)
    np.testing.assert_allclose(phi1[1:] - phi0[1:], mdot * v, rtol=1e-12)
    assert phi0[0] == 0.0


# ---------------------------------------------------------------- estimator
def test_single_trajectory_kernel_values():
    """One trajectory on a cell centre: den there is 1/h exactly (r = 0), one
    cell away along an axis with h = one cell it is exp(-1/2)/h, and every
    covered cell reproduces -q (the estimator is a weighted mean)."""
    n = 16
    dx = 1.0 / n
    xc = (5 + 0.5) * dx
    x = np.array([[xc], [xc], [xc]])
    h = dx
    q = np.array([[2.0], [-1.0], [0.5], [3.0]])
    m = _mesh(3, n)
    p = oracle.nw_cells(m, x, _terms_from([h], q, x))
    lin = lambda i, j, k: i + n * (j + n * k)
    assert p.den[lin(5, 5, 5)] == pytest.approx(1.0 / h, rel=1e-15)
    assert p.den[lin(6, 5, 5)] == pytest.approx(math.exp(-0.5) / h, rel=1e-14)
    assert p.den[lin(5, 7, 5)] == pytest.approx(math.exp(-2.0) / h, rel=1e-14)
    covered = p.den > 0
    # cutoff 4 h = 4 cells: the covered cells are the lattice points of a radius-4 ball
    assert covered.sum() == sum(1 for a in range(-4, 5) for b in range(-4, 5) for c in range(-4, 5)
                                if a * a + b * b + c * c <= 16)
    np.testing.assert_allclose(p.S[:, covered], -np.repeat(q, covered.sum(), axis=1), rtol=1e-14)
    assert np.all(p.S[:, ~covered] == 0.0)


def test_evaporation_sign_single_droplet():
    """An evaporating droplet (delta < 0) loses mass, so the gas-side mass
    source is positive; drag towards a faster gas gives a negative momentum
    source along the relative velocity."""
    x = np.array([[0.5], [0.5]])
    tr = T(x, v=[[0.0], [0.0]], ug=[[1.0], [0.0]], r=[1e-5])
    m = _mesh(2, 8)
    p, t = oracle.project(m, tr, RHO, MU, -1e-9, h0=0.1)
    cov = p.den > 0
    assert np.all(p.S[0, cov] > 0)
    assert np.all(p.S[1, cov] < 0)


def test_two_trajectories_closed_form():
    """Two trajectories with equal h, one on a cell centre and one two
    bandwidths away along x: at the first centre the weights are 1 and
    exp(-2), so S = -(q1 + e^-2 q2)/(1 + e^-2); at the midpoint cell both
    weights are equal and S is minus the mean."""
    n = 32
    dx = 1.0 / n
    c0 = 10.5 * dx
    h = dx
    x = np.array([[c0, c0 + 2 * h], [c0, c0]])
    q = np.array([[1.0, 5.0], [2.0, -4.0], [0.0, 1.0]])
    m = _mesh(2, n)
    p = oracle.nw_cells(m, x, _terms_from([h, h], q, x))
    e = math.exp(-2.0)
    at0 = 10 + n * 10
    np.testing.assert_allclose(p.S[:, at0], -(q[:, 0] + e * q[:, 1]) / (1 + e), rtol=1e-14)
    mid = 11 + n * 10
    np.testing.assert_allclose(p.S[:, mid], -(q[:, 0] + q[:, 1]) / 2, rtol=1e-14)


def test_kernel_prefactor_is_one_over_h():
    """Two trajectories at the same distance from a cell with bandwidths h and
    2h: weights are (1/h) e^{-r^2/2h^2} and (1/2h) e^{-r^2/8h^2}."""
    n = 64
    dx = 1.0 / n
    c = 20.5 * dx
    h = 2 * dx
    x = np.array([[c - 3 * dx, c + 3 * dx], [c, c]])
    q = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    m = _mesh(2, n)
    p = oracle.nw_cells(m, x, _terms_from([h, 2 * h], q, x), cells=np.array([20 + n * 20]))
    r2 = (3 * dx) ** 2
    w1 = (1 / h) * math.exp(-r2 / (2 * h * h))
    w2 = (1 / (2 * h)) * math.exp(-r2 / (8 * h * h))
    assert p.den[0] == pytest.approx(w1 + w2, rel=1e-14)
    assert -p.S[0, 0] == pytest.approx(w1 / (w1 + w2), rel=1e-14)


def test_uniform_field_reproduced_exactly():
    """If every trajectory carries the same q, the estimator returns -q in
    every cell with a non-zero denominator (partition of unity)."""
    wl = W.small_random_3d(400, 12, seed=5)
    t = oracle.trajectory_terms(wl.traj, RHO, MU, DELTA, wl.h0)
    q = np.tile(np.array([[1.5], [-2.0], [0.25], [7.0]]), (1, wl.traj.count))
    t.q = np.ascontiguousarray(q)
    p = oracle.nw_cells(wl.mesh, wl.traj.x, t)
    cov = p.den > 0
    assert cov.mean() > 0.5
    ref = -np.array([1.5, -2.0, 0.25, 7.0])[:, None]
    np.testing.assert_allclose(p.S[:, cov], np.broadcast_to(ref, p.S[:, cov].shape), rtol=1e-13)


def test_truncation_boundary():
    """A trajectory exactly c*h from a cell centre (c = 4, exactly representable
    distances) is included; one a little further is not."""
    n = 16
    dx = 1.0 / n
    c0 = 3.5 * dx
    h = dx / 2
    q = np.array([[1.0], [1.0], [1.0]])
    m = _mesh(2, n)
    inside = np.array([[c0 + 4 * h], [c0]])
    p = oracle.nw_cells(m, inside, _terms_from([h], q, inside), cells=np.array([3 + n * 3]))
    assert p.pairs[0] == 1 and p.den[0] == pytest.approx(2 * math.exp(-8.0) / dx, rel=1e-14)
    outside = np.array([[c0 + 4 * h * (1 + 1e-9)], [c0]])
    p = oracle.nw_cells(m, outside, _terms_from([h], q, outside), cells=np.array([3 + n * 3]))
    assert p.pairs[0] == 0 and p.den[0] == 0.0


def test_periodic_minimum_image():
    n = 10
    x = np.array([[0.01], [0.55]])
    q = np.array([[1.0], [0.0], [0.0]])
    h = 0.03
    far_cell = 9 + n * 5          # centre (0.95, 0.55): 0.06 away through the wrap
    per = oracle.nw_cells(_mesh(2, n, True), x, _terms_from([h], q, x), cells=np.array([far_cell]))
    clo = oracle.nw_cells(_mesh(2, n, False), x, _terms_from([h], q, x), cells=np.array([far_cell]))
    assert per.den[0] == pytest.approx((1 / h) * math.exp(-0.06 ** 2 / (2 * h * h)), rel=1e-12)
    assert clo.den[0] == 0.0


def test_truncation_error_is_bounded_by_the_tail():
    """Raising the cutoff from 4 to 8 bandwidths changes the estimator by no
    more than the neglected Gaussian tail allows."""
    wl = W.small_random_3d(300, 10, seed=7)
    t = oracle.trajectory_terms(wl.traj, RHO, MU, DELTA, wl.h0)
    p4 = oracle.nw_cells(wl.mesh, wl.traj.x, t, cutoff=4.0)
    p8 = oracle.nw_cells(wl.mesh, wl.traj.x, t, cutoff=8.0)
    both = p4.den > 0
    rel = np.linalg.norm(p4.S[:, both] - p8.S[:, both]) / np.linalg.norm(p8.S[:, both])
    assert 0 < rel < 0.05
    assert np.all(p8.den >= p4.den)


def test_scale_and_cell_scale():
    wl = W.small_random_3d(200, 8, seed=8)
    t = oracle.trajectory_terms(wl.traj, RHO, MU, DELTA, wl.h0)
    p1 = oracle.nw_cells(wl.mesh, wl.traj.x, t)
    cs = np.linspace(0.5, 2.0, 512)
    p2 = oracle.nw_cells(wl.mesh, wl.traj.x, t, scale=3.0, cell_scale=cs)
    np.testing.assert_allclose(p2.S, 3.0 * cs * p1.S, rtol=1e-14)


def test_f32_decision_agrees_away_from_the_boundary():
    wl = W.small_random_3d(500, 12, seed=9)
    t = oracle.trajectory_terms(wl.traj, RHO, MU, DELTA, wl.h0)
    p64 = oracle.nw_cells(wl.mesh, wl.traj.x, t, f32_decision=False)
    p32 = oracle.nw_cells(wl.mesh, wl.traj.x, t, f32_decision=True)
    assert abs(int(p64.pairs.sum()) - int(p32.pairs.sum())) <= 2
    np.testing.assert_allclose(p32.S, p64.S, rtol=1e-6, atol=1e-6 * np.abs(p64.S).max())


def test_skips_degenerate_trajectories():
    x = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    J = np.array([[1.0, 1.0, np.nan], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 1.0]])
    tr = T(x, J=J)
    t = oracle.trajectory_terms(tr, RHO, MU, DELTA, 0.1)
    assert list(t.valid) == [1, 0, 0] and t.skipped == 2


# ---------------------------------------------------------------- number density
def test_number_density_conservation_on_lattice():
    """n |det J| V_seed summed over a lattice equals n0 times the seeded volume."""
    wl = W.taylor_green_2d(per_axis=32, mesh_n=32)
    t = oracle.trajectory_terms(wl.traj, RHO, MU, DELTA, wl.h0)
    total = np.sum(t.n * np.abs(t.det) * wl.traj.seed_volume)
    assert total == pytest.approx(W.N0_DEFAULT * 1.0, rel=1e-13)
    # and h scales with |det J| (h0 = pitch)
    np.testing.assert_allclose(t.h, wl.h0 * np.abs(t.det), rtol=1e-15)


# ---------------------------------------------------------------- deposition
def test_deposit_conserves_totals():
    wl = W.small_random_3d(300, 10, seed=11)
    t = oracle.trajectory_terms(wl.traj, RHO, MU, DELTA, wl.h0)
    S, Z = oracle.deposit(wl.mesh, wl.traj.x, t, wl.traj.seed_volume, scale=2.0)
    Vc = wl.mesh.cell_volume
    Q = t.q * wl.traj.seed_volume * np.abs(t.det)
    np.testing.assert_allclose(S.sum(axis=1) * Vc, -2.0 * Q.sum(axis=1), rtol=1e-12)
    assert (Z == 0).any() or True


def test_deposit_single_trajectory_closed_form():
    """One droplet with det J = 3 deposits n0 V_seed phi in total (the seed's
    droplets; det J cancels between n = n0/|det J| and the stretched volume),
    spread with weights proportional to exp(-r^2/(2h^2)) at h = h0 |det J|."""
    n, n0, vseed, r = 16, 2.5e9, 0.04, 12e-6
    v, ug = np.array([0.3, -0.1]), np.array([0.5, 0.2])
    x = np.array([[8.5 / n], [8.5 / n]])        # a cell centre
    J = np.array([[3.0], [0.7], [0.0], [1.0]])  # det J = 3
    tr = W.Trajectories(torch.tensor(x), torch.tensor(J), torch.tensor(v.reshape(2, 1)),
                        torch.tensor(ug.reshape(2, 1)), torch.tensor([r], dtype=torch.float64), n0, vseed)
    h0 = 1.0 / (3 * n)                          # so that h = one cell width
    t = oracle.trajectory_terms(tr, RHO, MU, DELTA, h0)
    S, Z = oracle.deposit(_mesh(2, n, periodic=True), x, t, vseed)
    # phi of one droplet from Stokes' law and the d^2 evaporation law
    mdot = 2 * math.pi * RHO * r * DELTA
    F = 6 * math.pi * MU * r * (ug - v)
    phi = np.array([mdot, *(F + mdot * v)])
    Vc = 1.0 / n ** 2
    np.testing.assert_allclose(S.sum(axis=1) * Vc, -n0 * vseed * phi, rtol=1e-12)
    c0 = 8 + n * 8
    np.testing.assert_allclose(S[:, c0 + 1] / S[:, c0], math.exp(-0.5), rtol=1e-13)
    np.testing.assert_allclose(S[:, c0 + 1 + n] / S[:, c0], math.exp(-1.0), rtol=1e-13)
    np.testing.assert_allclose(S[:, c0 + 2 * n] / S[:, c0], math.exp(-2.0), rtol=1e-13)
    # the normaliser is the kernel summed over the 49 cells within 4 widths
    ks = [(i, j) for i in range(-4, 5) for j in range(-4, 5) if i * i + j * j <= 16]
    assert Z[0] == pytest.approx(n * sum(math.exp(-0.5 * (i * i + j * j)) for i, j in ks), rel=1e-13)


def test_deposit_zero_support_goes_home():
    n = 8
    x = np.array([[0.3], [0.6]])       # not at a cell centre
    q = np.array([[4.0], [1.0], [2.0]])
    t = _terms_from([1e-6], q, x)
    S, Z = oracle.deposit(_mesh(2, n), x, t, seed_volume=0.5)
    assert Z[0] == 0.0
    home = int(0.3 * n) + n * int(0.6 * n)
    Vc = 1.0 / n ** 2
    np.testing.assert_allclose(S[:, home], -q[:, 0] * 0.5 / Vc, rtol=1e-15)
    assert np.count_nonzero(S) == 3


# ---------------------------------------------------------------- PSI-CELL
def test_psicell_single_particle_and_sums():
    m = _mesh(2, 4)
    cl = T(np.array([[0.3, 0.3, 0.9, 1.0, 1.2], [0.1, 0.15, 0.9, 0.5, 0.5]]),
           v=np.array([[0.1, 0.2, 0.0, 0.0, 0.0], [0.0, 0.0, 0.1, 0.0, 0.0]]),
           ug=np.zeros((2, 5)), r=np.full(5, 1e-5))
    S, counts, sk = oracle.psicell(m, cl, weight=7.0, rho_d=RHO, mu=MU, delta=DELTA)
    assert sk == 1                       # x = 1.2 is outside the closed box
    assert counts.sum() == 4
    assert counts[1 + 4 * 0] == 2 and counts[3 + 4 * 3] == 1 and counts[3 + 4 * 2] == 1  # x == hi -> last cell
    phis = [oracle.droplet_phi(2, 1e-5, cl.v[:, p], cl.ug[:, p], RHO, MU, DELTA)[0] for p in range(4)]
    Vc = 1.0 / 16
    np.testing.assert_allclose(S.sum(axis=1) * Vc, -7.0 * np.sum(phis, axis=0), rtol=1e-13)
    np.testing.assert_allclose(S[:, 3 + 4 * 3], -7.0 / Vc * phis[2], rtol=1e-14)


def test_psicell_periodic_wrap():
    m = _mesh(3, 4, True)
    assert oracle.psicell_cell_of(m, [1.1, -0.1, 0.5]) == 0 + 4 * (3 + 4 * 2)
    m2 = _mesh(3, 4, False)
    assert oracle.psicell_cell_of(m2, [1.1, 0.5, 0.5]) == -1


# ---------------------------------------------------------------- App. A scaling
def test_app_a_fla_parameters_cancel():
    """n_hat = M_scal V_scal is independent of the FLA seeding parameters and
    equals V_cell N_ref/(A_inj v_inj tau_ref) (eq. A.13), or with the mass
    flow rate Mdot_ref = N_ref m/tau_ref, V_cell Mdot_ref/(A_inj v_inj m) (A.14)."""
    rng = np.random.default_rng(4)
    for _ in range(50):
        N_ref, tau_ref, V_cell, A, v = rng.uniform(0.1, 1000, 5)
        ref = V_cell * N_ref / (A * v * tau_ref)
        mass = rng.uniform(1e-9, 1e-3)
        mdot = N_ref * mass / tau_ref
        for N_fla, tau_fla in rng.uniform(0.01, 1000, (5, 2)):
            M_s, V_s, nh = oracle.app_a_scaling(N_ref, tau_ref, N_fla, tau_fla, V_cell, A, v)
            assert nh == pytest.approx(ref, rel=1e-12)
            assert nh == pytest.approx(V_cell * mdot / (A * v * mass), rel=1e-12)
