"""Pins of the learned-bandwidth oracle: bfloat16 rounding against torch's
own conversion, features against closed forms and brute-force counts, the
analytic gradients against central finite differences, and Adam's first
step against its closed form."""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.learned as LN
import workloads as W

RHO, MU, DELTA = W.RHO_D, W.MU_AIR, W.DELTA_EVAP


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 0.0, 65504.0, 1e-30]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(LN.bf16(x), ref)


def test_singular_value_and_density_features():
    rng = np.random.default_rng(1)
    N = 50
    Js, svals = [], []
    for _ in range(N):
        q1, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        q2, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        s = np.sort(rng.uniform(0.1, 3.0, 3))[::-1]
        Js.append(q1 @ np.diag(s) @ q2)
        svals.append(s)
    J = np.stack(Js).reshape(N, 9).T.copy()
    x = rng.uniform(0, 1, (3, N))
    mesh = W.unit_mesh(3, 8, True)
    f = LN.features(mesh, x, J, np.ones(N, dtype=np.int32))
    np.testing.assert_allclose(f[:3], np.log(np.array(svals)).T, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(f[3], -np.log(np.prod(svals, axis=1)), rtol=1e-10, atol=1e-12)


def test_skipped_trajectories_have_zero_features_whatever_their_J():
    """A skipped trajectory (non-finite J included) has zero features, and
    the valid trajectories' singular values and det J do not depend on it;
    only the neighbour counts see validity."""
    rng = np.random.default_rng(3)
    N = 40
    J = rng.standard_normal((9, N)) + 2.0 * np.eye(3).reshape(9, 1)
    x = rng.uniform(0, 1, (3, N))
    mesh = W.unit_mesh(3, 6, True)
    valid = np.ones(N, dtype=np.int32)
    valid[[3, 17]] = 0
    f_ok = LN.features(mesh, x, J, valid)
    Jb = J.copy()
    Jb[4, 3] = np.nan
    Jb[0, 17] = np.inf
    f_bad = LN.features(mesh, x, Jb, valid)
    assert np.all(f_bad[:, [3, 17]] == 0.0)
    np.testing.assert_array_equal(f_bad, f_ok)
    f_all = LN.features(mesh, x, J, np.ones(N, dtype=np.int32))
    v = valid == 1
    np.testing.assert_array_equal(f_bad[:4, v], f_all[:4, v])


def test_neighbour_count_brute_force():
    rng = np.random.default_rng(2)
    for periodic in (True, False):
        mesh = W.unit_mesh(3, 5, periodic)
        x = rng.uniform(0, 1, (3, 60))
        valid = (rng.uniform(size=60) > 0.1).astype(np.int32)
        got = LN.neighbour_counts(mesh, x, valid)
        cell = np.floor(x * 5).astype(int)
        for i in range(60):
            cnt = 0
            for j in range(60):
                if not valid[j]:
                    continue
                d = cell[:, j] - cell[:, i]
                if periodic:
                    d = (d + 2) % 5 - 2          # circular difference in {-2..2}
                if np.all(np.abs(d) <= 1):
                    cnt += 1
            assert got[i] == cnt


def test_zero_last_layer_gives_unit_factor():
    theta = LN.init_params(3)
    f = np.random.default_rng(3).standard_normal((5, 100))
    fw = LN.forward(theta, f)
    assert np.all(fw.g == 1.0)


def _exact_loss_of_theta(theta, f):
    return float(np.sum(LN.forward(theta, f, round_bf16=False).o ** 2))


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    theta = LN.init_params(4)
    p = LN.unpack(theta)
    p["w3"] = rng.standard_normal(64) * 0.3
    p["b1"] = rng.standard_normal(64) * 0.1
    theta = LN.pack(p)
    f = rng.standard_normal((5, 40))
    fw = LN.forward(theta, f, round_bf16=False)
    grad = LN.backward(theta, fw, 2.0 * fw.o, round_bf16=False)
    for k in list(rng.choice(LN.N_TRAIN, 40, replace=False)) + [LN.N_TRAIN - 1]:
        e = np.zeros_like(theta)
        eps = 1e-6 * max(1.0, abs(theta[k]))
        e[k] = eps
        fd = (_exact_loss_of_theta(theta + e, f) - _exact_loss_of_theta(theta - e, f)) / (2 * eps)
        assert grad[k] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def _loss_of_h(mesh, x, h, t, R, cutoff):
    terms = oracle.Terms(t.det, h, t.n, t.q, t.valid, 0)
    p = oracle.nw_cells(mesh, x, terms, cutoff=cutoff)
    return LN.rel_l2_loss(p.S, R)[0], p


def test_dL_dh_matches_finite_differences():
    """Cutoff 6 bandwidths keeps the ignored boundary term below e^-18."""
    wl = W.small_random_3d(120, 8, seed=5, periodic=True)
    t = oracle.trajectory_terms(wl.traj, RHO, MU, DELTA, wl.h0)
    x = wl.traj.x.numpy()
    rng = np.random.default_rng(5)
    R = rng.standard_normal((4, wl.mesh.cells)) * 1e-3
    cutoff = 6.0
    L0, p = _loss_of_h(wl.mesh, x, t.h, t, R, cutoff)
    _, dLdS = LN.rel_l2_loss(p.S, R)
    g = LN.dL_dh(wl.mesh, x, t.h, t.q, t.valid, p.S, p.den, dLdS, cutoff=cutoff)
    for i in rng.choice(120, 12, replace=False):
        eps = 1e-6 * t.h[i]
        hp, hm = t.h.copy(), t.h.copy()
        hp[i] += eps
        hm[i] -= eps
        fd = (_loss_of_h(wl.mesh, x, hp, t, R, cutoff)[0] - _loss_of_h(wl.mesh, x, hm, t, R, cutoff)[0]) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(L0) / t.h[i])


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(6)
    theta = LN.init_params(6)
    grad = rng.standard_normal(theta.size)
    t1, m, v = LN.adam(theta, grad, np.zeros_like(theta), np.zeros_like(theta), 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(t1[:LN.N_TRAIN] - theta[:LN.N_TRAIN], -1e-3 * np.sign(grad[:LN.N_TRAIN]),
                               rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(t1[LN.N_TRAIN:], theta[LN.N_TRAIN:])


def test_adam_bias_correction_over_three_steps():
    """Closed forms of the bias-corrected moments.  A constant gradient g gives
    m_hat = g and v_hat = g^2 at every step, so each step moves by lr sign(g).
    Gradients g, -g, g give m_hat = -(1 - b1)/(1 + b1) g at step 2 and
    (b1^2 - b1 + 1)/(1 + b1 + b1^2) g at step 3, with v_hat = g^2."""
    rng = np.random.default_rng(7)
    theta = LN.init_params(7)
    g = rng.standard_normal(theta.size)
    lr, b1, b2 = 1e-3, 0.9, 0.999
    T = slice(0, LN.N_TRAIN)
    t, m, v = theta, np.zeros_like(theta), np.zeros_like(theta)
    for step in (1, 2, 3):
        t, m, v = LN.adam(t, g, m, v, step, lr=lr, b1=b1, b2=b2, eps=0.0)
        np.testing.assert_allclose(t[T] - theta[T], -step * lr * np.sign(g[T]), rtol=1e-11, atol=1e-16)
    t, m, v = theta, np.zeros_like(theta), np.zeros_like(theta)
    t1, m, v = LN.adam(t, g, m, v, 1, lr=lr, b1=b1, b2=b2, eps=0.0)
    t2, m, v = LN.adam(t1, -g, m, v, 2, lr=lr, b1=b1, b2=b2, eps=0.0)
    np.testing.assert_allclose(t2[T] - t1[T], lr * (1 - b1) / (1 + b1) * np.sign(g[T]), rtol=1e-10, atol=1e-17)
    t3, m, v = LN.adam(t2, g, m, v, 3, lr=lr, b1=b1, b2=b2, eps=0.0)
    r3 = (b1 * b1 - b1 + 1) / (1 + b1 + b1 * b1)
    np.testing.assert_allclose(t3[T] - t2[T], -lr * r3 * np.sign(g[T]), rtol=1e-10, atol=1e-17)
    np.testing.assert_array_equal(t3[LN.N_TRAIN:], theta[LN.N_TRAIN:])
