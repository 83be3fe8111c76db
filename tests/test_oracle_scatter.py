"""The trajectory-centric forms of the oracle against its brute-force forms.

The brute-force forms evaluate the estimator (eqs. kernel, kernel-estimator
and coupling-terms-kernel) and the deposition at every cell over every
trajectory: they are the definition, pinned by the closed forms of
``test_oracle_pins.py``.  The scatter forms visit only the cells inside each
trajectory's cutoff box (App. B steps 1c-1d), so a wrong box bound (a cell
missed at a periodic wrap, at a closed wall, or for a support wider than the
mesh) changes a pair count.  Both forms add every cell's trajectories in
ascending order with the same per-pair arithmetic, so they must agree bit
for bit: fields, denominators, pair counts and deposition normalisers.
"""
import numpy as np
import pytest

import oracle


def _random_case(dim, n, periodic, N, seed, h_lo, h_hi, outside=0.0):
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-1.0, 1.0, dim)
    L = rng.uniform(0.5, 2.0, dim)
    mesh = oracle.make_mesh(dim, n, lo, lo + L, periodic)
    x = lo[:, None] + rng.uniform(-outside, 1.0 + outside, (dim, N)) * L[:, None]
    h = np.exp(rng.uniform(np.log(h_lo), np.log(h_hi), N))
    q = rng.normal(size=(1 + dim, N))
    valid = (rng.uniform(size=N) > 0.1).astype(np.int32)
    det = rng.choice([-1.0, 1.0], N) * rng.uniform(0.2, 3.0, N)
    t = oracle.Terms(det=det, h=h * np.where(valid > 0, 1.0, 0.0), n=np.ones(N), q=q, valid=valid, skipped=0)
    return mesh, x, t


CASES = [
    # dim, cells per axis, periodic axes, trajectories, bandwidth range, positions outside the box
    (2, (13, 9), (True, True), 300, (0.02, 0.3), 0.0),
    (2, (16, 11), (False, True), 300, (0.01, 0.5), 0.3),
    (2, (7, 23), (False, False), 200, (0.005, 2.0), 0.5),
    (3, (9, 7, 11), (True, True, True), 150, (0.02, 0.3), 0.0),
    (3, (10, 6, 8), (True, False, True), 150, (0.01, 0.8), 0.2),
    (3, (5, 8, 6), (False, False, False), 120, (0.003, 3.0), 0.4),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("f32", [False, True])
def test_scatter_equals_brute_force_on_whole_mesh(case, f32):
    dim, n, per, N, (hl, hh), out = CASES[case]
    mesh, x, t = _random_case(dim, n, per, N, 10 + case, hl, hh, out)
    cs = np.random.default_rng(case).uniform(0.5, 2.0, int(np.prod(n)))
    ref = oracle.nw_cells(mesh, x, t, None, 4.0, f32, 1.7, cs)
    got = oracle.nw_box(mesh, x, t, None, None, 4.0, f32, 1.7, cs)
    np.testing.assert_array_equal(got.cells, np.arange(int(np.prod(n))))
    assert ref.pairs.sum() > 0
    np.testing.assert_array_equal(got.pairs, ref.pairs)
    np.testing.assert_array_equal(got.den, ref.den)
    np.testing.assert_array_equal(got.S, ref.S)


@pytest.mark.parametrize("case", [0, 3, 4])
def test_scatter_on_wrapped_sub_box(case):
    """A box of cells that straddles the periodic boundary."""
    dim, n, per, N, (hl, hh), out = CASES[case]
    mesh, x, t = _random_case(dim, n, per, N, 20 + case, hl, hh, out)
    box_lo = [n[a] - 3 if per[a] else 1 for a in range(dim)]
    box_n = [5 if per[a] else n[a] - 2 for a in range(dim)]
    got = oracle.nw_box(mesh, x, t, box_lo, box_n, 4.0, True)
    # the box cells: indices box_lo .. box_lo + box_n - 1, wrapped
    axes = [np.arange(box_lo[a], box_lo[a] + box_n[a]) % n[a] for a in range(dim)]
    grid = np.meshgrid(*axes, indexing="ij")
    lin = grid[0] + n[0] * grid[1] + (n[0] * n[1] * grid[2] if dim == 3 else 0)
    cells = lin.transpose(*range(dim)[::-1]).reshape(-1)   # box order: axis 0 fastest
    np.testing.assert_array_equal(got.cells, cells)
    ref = oracle.nw_cells(mesh, x, t, cells, 4.0, True)
    np.testing.assert_array_equal(got.pairs, ref.pairs)
    np.testing.assert_array_equal(got.S, ref.S)
    np.testing.assert_array_equal(got.den, ref.den)


def test_scatter_single_trajectory_covers_the_ball():
    """One trajectory at a cell centre with h equal to the cell width: the
    covered cells are the lattice points of the radius-4 ball (257 in 2-D),
    whichever periodic image holds them."""
    for centre in ([0.5 / 32, 0.5 / 32], [15.5 / 32, 31.5 / 32]):
        mesh = oracle.make_mesh(2, (32, 32), (0, 0), (1, 1), (True, True))
        x = np.array(centre, dtype=float).reshape(2, 1)
        t = oracle.Terms(det=np.ones(1), h=np.array([1 / 32]), n=np.ones(1), q=np.ones((3, 1)),
                         valid=np.ones(1, dtype=np.int32), skipped=0)
        got = oracle.nw_box(mesh, x, t)
        assert int(got.pairs.sum()) == sum(1 for i in range(-4, 5) for j in range(-4, 5) if i * i + j * j <= 16)


def test_scatter_rejects_a_box_outside_a_closed_mesh():
    mesh, x, t = _random_case(2, (8, 8), (False, False), 10, 0, 0.05, 0.1)
    with pytest.raises(ValueError):
        oracle.nw_box(mesh, x, t, [5, 0], [4, 8])


@pytest.mark.parametrize("case", range(len(CASES)))
def test_deposit_scatter_equals_brute_force(case):
    dim, n, per, N, (hl, hh), out = CASES[case]
    mesh, x, t = _random_case(dim, n, per, N, 30 + case, hl, hh, out)
    # a few tiny bandwidths reach no cell centre: their amount goes home
    t.h[::17] = t.h[::17] * 1e-4
    for f32 in (False, True):
        S1, Z1 = oracle.deposit(mesh, x, t, 0.37, 4.0, f32, 1.3)
        S2, Z2 = oracle.deposit_scatter(mesh, x, t, 0.37, 4.0, f32, 1.3)
        assert (Z1[t.valid > 0] == 0).any()
        np.testing.assert_array_equal(Z2, Z1)
        np.testing.assert_array_equal(S2, S1)
