"""Pin of the whole plain path against an independent method: as the FLA
seeding grows, the Nadaraya-Watson source field converges towards the
PSI-CELL box-counting field of a dense cloud (the comparison the paper makes
between the two coupling methods), on the fold-free Taylor-Green map."""
import numpy as np
import pytest

import oracle
import workloads as W

RHO, MU, DELTA = W.RHO_D, W.MU_AIR, W.DELTA_EVAP


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_nw_converges_to_psicell_on_taylor_green():
    mesh_n = 32
    cloud = W.taylor_green_cloud(n_particles=400_000, seed=0)
    mesh = W.unit_mesh(2, mesh_n, False)
    Np = cloud.count
    w = W.N0_DEFAULT * 1.0 / Np
    S_psi, counts, sk = oracle.psicell(mesh, cloud, w, RHO, MU, DELTA)
    assert sk == 0 and counts.sum() == Np
    # noise floor of the reference from two independent halves
    half = Np // 2
    A = cloud.subset(np.arange(half))
    B = cloud.subset(np.arange(half, Np))
    SA, _, _ = oracle.psicell(mesh, A, 2 * w, RHO, MU, DELTA)
    SB, _, _ = oracle.psicell(mesh, B, 2 * w, RHO, MU, DELTA)
    floor2 = np.sum((SA - SB) ** 2) / (4 * np.sum(S_psi ** 2))
    errs = []
    for per_axis in (8, 16, 32, 64):
        wl = W.taylor_green_2d(per_axis=per_axis, mesh_n=mesh_n)
        p, t = oracle.project(wl.mesh, wl.traj, RHO, MU, DELTA, wl.h0)
        assert (p.den > 0).all()
        e2 = np.sum((p.S - S_psi) ** 2) / np.sum(S_psi ** 2)
        errs.append(np.sqrt(max(e2 - floor2, 0.0)))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.5 * errs[0]
