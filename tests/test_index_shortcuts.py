"""CPU checks of the arithmetic shortcuts the device code takes in place of
a division, each restated here in numpy binary64 and compared with the
division-based definition it replaces, on random and adversarial inputs.

* Minimum image on a periodic axis: d - L rint(d/L) without the division
  for |d| < L (csrc/internal.hpp, min_image).
* PSI-CELL cell index: floor((x - lo)/w) from a multiply by 1/w, with the
  exact quotient next to integers (csrc/psicell.hip, psi_cell).
* Support bounds of the prepass: the multiply by 1/w with the widened margin
  never gives a narrower cell range than the division with the old margin
  (csrc/prepass.hip).

These pin the reasoning; the GPU parity tests run the device code itself.
"""
import numpy as np


def _min_image_fast(d, L):
    # the device code: no division for |d| < L
    ad = np.abs(d)
    out = np.where(ad <= 0.5 * L, d, np.where(d > 0.0, d - L, d + L))
    slow = ad >= L
    out[slow] = d[slow] - L * np.rint(d[slow] / L)
    return out


def _min_image_ref(d, L):
    return d - L * np.rint(d / L)


def _adversarial_offsets(rng, L, n):
    """Offsets at, just below and just above +-L/2 and +-L, random offsets in
    (-1.5 L, 1.5 L), and offsets built as differences of cell centres and
    positions (the way the device forms them)."""
    half = 0.5 * L
    edge = np.array([half, -half, L, -L, 0.0, 1.5 * L, -1.5 * L])
    near = np.concatenate([np.nextafter(edge, np.inf), np.nextafter(edge, -np.inf), edge])
    k = np.arange(-40, 41)
    ulps = np.concatenate([half + k * np.spacing(half), -half + k * np.spacing(half)])
    rnd = rng.uniform(-1.5 * L, 1.5 * L, n)
    cells = 97
    xc = (np.arange(cells) + 0.5) * (L / cells)
    xp = rng.uniform(0.0, L, n // 4)
    diff = (xc[None, :] - xp[:, None]).ravel()
    return np.concatenate([near, ulps, rnd, diff])


def test_min_image_without_division_is_exact():
    rng = np.random.default_rng(7)
    for L in (1.0, 2.0 * np.pi, 0.3, 1e-3, 7.0 / 3.0, 123.456):
        d = _adversarial_offsets(rng, L, 200_000)
        fast = _min_image_fast(d, L)
        ref = _min_image_ref(d, L)
        assert np.array_equal(fast.view(np.int64), ref.view(np.int64)), L


def _cell_floor_fast(dx, w):
    q = dx * (1.0 / w)
    near = np.abs(q - np.rint(q)) < 1e-6 * (1.0 + np.abs(q))
    q = np.where(near, dx / w, q)
    return np.floor(q)


def test_psicell_floor_by_multiply_matches_the_quotient():
    rng = np.random.default_rng(11)
    for n_cells, lo, L in ((128, 0.0, 1.0), (37, -0.25, 1.3), (1000, 0.0, 2.0 * np.pi), (256, 3.0, 1e-2)):
        w = L / n_cells
        x = rng.uniform(lo - 0.2 * L, lo + 1.2 * L, 400_000)
        # positions on and next to cell faces, where the floor is decided
        faces = lo + np.arange(-3, n_cells + 4) * w
        x = np.concatenate([x, faces, np.nextafter(faces, np.inf), np.nextafter(faces, -np.inf)])
        dx = x - lo
        assert np.array_equal(_cell_floor_fast(dx, w), np.floor(dx / w)), (n_cells, L)


def test_support_bounds_by_multiply_never_narrower():
    rng = np.random.default_rng(13)
    for n_cells, lo, L in ((128, 0.0, 1.0), (37, -0.25, 1.3), (4096, 0.0, 2.0 * np.pi)):
        w = L / n_cells
        x = rng.uniform(lo - 3 * L, lo + 4 * L, 400_000)
        rc = rng.uniform(0.0, 20.0 * w, x.size)
        iw = 1.0 / w
        qlo, qhi = (x - rc - lo) * iw, (x + rc - lo) * iw
        flo_new = qlo - 0.5 - (1e-9 + 1e-15 * np.abs(qlo))
        fhi_new = qhi - 0.5 + (1e-9 + 1e-15 * np.abs(qhi))
        # the exact real bounds, up to the rounding of the division form
        flo_div = (x - rc - lo) / w - 0.5
        fhi_div = (x + rc - lo) / w - 0.5
        assert np.all(np.ceil(flo_new) <= np.ceil(flo_div))
        assert np.all(np.floor(fhi_new) >= np.floor(fhi_div))
