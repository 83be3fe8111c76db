"""CPU checks of the input generators (the maps stand in for the paper's
trajectory producer, so their properties are pinned here) and of the
benchmark's reading of committed counter summaries."""
import hashlib
import math
import os

import pytest
import torch

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _det3(J):
    return (J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6])
            + J[2] * (J[3] * J[7] - J[4] * J[6]))


def test_counter_uniform_is_deterministic_and_uniform():
    a = W.counter_uniform(3, 7, 200_000)
    b = W.counter_uniform(3, 7, 200_000)
    c = W.counter_uniform(3, 8, 200_000)
    assert torch.equal(a, b) and not torch.equal(a, c)
    assert 0.0 < float(a.min()) and float(a.max()) < 1.0
    # mean 1/2 and variance 1/12 within a few standard errors
    assert abs(float(a.mean()) - 0.5) < 4 * (1 / 12 / 2e5) ** 0.5
    assert abs(float(a.var()) - 1 / 12) < 2e-3
    # an offset continues the same stream
    assert torch.equal(W.counter_uniform(3, 7, 10, offset=5), a[5:15])


def test_abc_map_folds():
    """Amplitude-0.2 ABC map on the 128^3 lattice: lattice mean of det J is 1
    (degree-one map of the torus) and 32.7% of the determinants are negative
    (folds), the reading of the 3-D configuration."""
    x0 = W.lattice(3, 128)
    _, J, _ = W.abc_map(x0, W.ABC(amp=0.2))
    det = _det3(J)
    assert float(det.mean()) == pytest.approx(1.0, abs=1e-12)
    assert float((det < 0).double().mean()) == pytest.approx(0.32706, abs=2e-5)


def test_multi_vortex_map_caustics():
    """The composed map of the large configuration: degree one (lattice mean
    of det J is 1), its determinants change sign, and on the 320^3 lattice
    min |det J| is below 1e-6 (strong caustics), checked slab by slab."""
    maps = W.multi_vortex_default(0)
    x0 = W.lattice(3, 64)
    _, J, _ = W.multi_vortex_map(x0, maps)
    det = _det3(J)
    assert float(det.mean()) == pytest.approx(1.0, abs=1e-12)
    assert 0.4 < float((det < 0).double().mean()) < 0.48
    n = 320
    g = (torch.arange(n, dtype=torch.float64) + 0.5) / n
    gy, gx = torch.meshgrid(g, g, indexing="ij")
    amin = float("inf")
    for k in range(n):
        x = torch.stack([gx.reshape(-1), gy.reshape(-1), torch.full((n * n,), float(g[k]), dtype=torch.float64)])
        _, J, _ = W.multi_vortex_map(x, maps)
        amin = min(amin, float(_det3(J).abs().min()))
    assert amin < 1e-6


def test_bench_reads_the_traffic_summary():
    """bench.py reports the gather's HBM traffic only from a summary whose
    source hash matches gather.hpp and the compile-time constants in
    internal.hpp; the hash key contains a colon."""
    import bench
    path = os.path.join(ROOT, "profiles", "gather_abc128_hbm_traffic.md")
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].rsplit(":", 1)
            vals[k.strip()] = v.strip()
    key = "gather.hpp + internal.hpp sha256[:16]"
    assert key in vals and "bytes per launch (calibrated)" in vals
    h = hashlib.sha256()
    for name in ("gather.hpp", "internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2512_20829_amd", "csrc", name), "rb").read())
    got = bench.gather_traffic("abc128")
    if vals[key] == h.hexdigest()[:16]:
        assert got == float(vals["bytes per launch (calibrated)"])
    else:
        assert got is None


def test_bench_learned_crossing_interpolates_in_log_n():
    import bench
    rows = [{"trajectories": 8000, "learned": 0.5}, {"trajectories": 1000, "learned": 0.7},
            {"trajectories": 125, "learned": 0.9}]
    n, note = bench.learned_crossing(rows, 0.6)
    assert n == round(math.sqrt(8000 * 1000)) and note is None
    n, note = bench.learned_crossing(rows, 0.95)
    assert n is None and "125" in note
    n, note = bench.learned_crossing(rows, 0.4)
    assert n is None and "does not reach" in note


def test_table1_constants_match_the_printed_table():
    """The Table 1 cases the benchmark sweeps are the printed ones, and their
    relaxation time 2 rho r^2 / (9 rho_f nu) is the printed St (U/L = 1)."""
    import json
    with open(os.path.join(ROOT, "tests", "golden", "table1_parameters.json")) as f:
        t1 = json.load(f)
    assert len(W.TABLE1) == 4 and W.TABLE1_RHO_F == t1["rho_f"]
    for j, c in enumerate(W.TABLE1):
        assert (c["rho_d"], c["r_d"], c["nu"], c["St"]) == (t1["rho_d"][j], t1["r_d"][j], t1["nu"][j], t1["St"][j])
        assert c["evaporating"] == t1["columns"][j].startswith("evaporating")
        tau = 2 * c["rho_d"] * c["r_d"] ** 2 / (9 * W.TABLE1_RHO_F * c["nu"])
        assert tau == pytest.approx(c["St"], rel=1e-12)
