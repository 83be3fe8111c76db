"""Pins of the oracle's trajectory producer (Stokes drag, d^2-law evaporation
and the Jacobian equation, integrated by RK4 over one carrier step, with the
droplet's mass and momentum contributions summed over the substeps).

Each pin is a closed form or an independent computation: relaxation toward
a uniform gas velocity (with and without evaporation, where the relaxation
time shrinks with r^2), r^2 = r0^2 + delta t, the Jacobian of a linear flow
from the matrix exponential, the Jacobian of the ABC flow from finite
differences of the trajectory map, the velocity gradients from finite
differences of the field, and the exact identities
integral of mdot = m1 - m0, integral of (F + mdot v) = m1 v1 - m0 v0.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as W

RHO, MU = W.RHO_D, W.MU_AIR


def _state(x0, v0, r0, K0=None):
    x0 = np.asarray(x0, dtype=np.float64)
    dim, N = x0.shape
    J0 = np.tile(np.eye(dim).reshape(-1, 1), (1, N))
    K0 = np.zeros((dim * dim, N)) if K0 is None else np.asarray(K0, dtype=np.float64)
    return oracle.DropletState(x0.copy(), np.asarray(v0, dtype=np.float64).copy(), J0, K0,
                               np.asarray(r0, dtype=np.float64).copy())


def _tau(r):
    return 2.0 * RHO * r * r / (9.0 * MU)


def _mass(r):
    return 4.0 / 3.0 * math.pi * RHO * r ** 3


def test_relaxation_toward_a_uniform_gas_velocity():
    u0 = np.array([0.3, -0.2, 0.05])
    x0 = np.array([[0.1, 0.5], [0.2, 0.7], [0.9, 0.4]])
    v0 = np.array([[1.0, -0.5], [0.0, 0.25], [-0.3, 0.6]])
    r0 = np.array([10e-6, 14e-6])
    K0 = np.random.default_rng(0).normal(size=(9, 2))
    flow = oracle.make_flow(u0=u0)
    dt = 2e-3
    st, phi, valid, sk = oracle.advance(_state(x0, v0, r0, K0), flow, RHO, MU, 0.0, dt, 256)
    assert sk == 0 and valid.all()
    tau = _tau(r0)
    e = np.exp(-dt / tau)
    v = u0[:, None] + (v0 - u0[:, None]) * e
    x = x0 + u0[:, None] * dt + (v0 - u0[:, None]) * tau * (1 - e)
    np.testing.assert_allclose(st.v, v, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(st.x, x, rtol=1e-12, atol=1e-15)
    J = np.tile(np.eye(3).reshape(-1, 1), (1, 2)) + K0 * tau * (1 - e)
    np.testing.assert_allclose(st.J, J, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(st.K, K0 * e, rtol=1e-10, atol=1e-14)
    np.testing.assert_array_equal(st.r, r0)
    # no evaporation: no mass source; momentum source = m (v1 - v0) / dt
    assert np.all(phi[0] == 0.0)
    np.testing.assert_allclose(phi[1:], _mass(r0) * (v - v0) / dt, rtol=1e-9)


def test_evaporating_relaxation_and_the_d2_law():
    """r^2 = r0^2 + delta t; with tau = 2 rho r^2/(9 mu) shrinking,
    v - u0 = (v0 - u0) ((r0^2 + delta t)/r0^2)^(-9 mu / (2 rho delta))."""
    delta = -1e-9
    u0 = np.array([0.2, 0.1])
    x0 = np.array([[0.5], [0.5]])
    v0 = np.array([[0.9], [-0.4]])
    r0 = np.array([10e-6])
    dt = 2e-3
    st, phi, valid, sk = oracle.advance(_state(x0, v0, r0), oracle.make_flow(u0=u0), RHO, MU, delta, dt, 256)
    r1 = math.sqrt(r0[0] ** 2 + delta * dt)
    assert st.r[0] == pytest.approx(r1, rel=1e-13)
    p = -9.0 * MU / (2.0 * RHO * delta)
    v1 = u0 + (v0[:, 0] - u0) * ((r0[0] ** 2 + delta * dt) / r0[0] ** 2) ** p
    np.testing.assert_allclose(st.v[:, 0], v1, rtol=1e-9)
    m0, m1 = _mass(r0[0]), _mass(r1)
    assert phi[0, 0] * dt == pytest.approx(m1 - m0, rel=1e-10)
    np.testing.assert_allclose(phi[1:, 0] * dt, m1 * st.v[:, 0] - m0 * v0[:, 0], rtol=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
def test_jacobian_of_a_linear_flow_is_the_matrix_exponential(dim):
    rng = np.random.default_rng(dim)
    r0 = 12e-6
    tau = _tau(r0)
    G = rng.normal(size=(dim, dim)) * 0.3 / tau
    u0 = rng.normal(size=3) * 0.2
    x0 = rng.uniform(size=(dim, 1))
    v0 = rng.normal(size=(dim, 1)) * 0.3
    K0 = rng.normal(size=(dim * dim, 1)) * 50.0
    dt = 3e-3
    st, phi, valid, sk = oracle.advance(_state(x0, v0, [r0], K0), oracle.make_flow(u0=u0, G=G), RHO, MU, 0.0,
                                        dt, 256)
    I = np.eye(dim)
    A = np.block([[np.zeros((dim, dim)), I], [G / tau, -I / tau]])
    JK = scipy.linalg.expm(A * dt) @ np.vstack([I, K0[:, 0].reshape(dim, dim)])
    np.testing.assert_allclose(st.J[:, 0].reshape(dim, dim), JK[:dim], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(st.K[:, 0].reshape(dim, dim), JK[dim:], rtol=1e-8, atol=1e-9)
    Aa = np.zeros((2 * dim + 1, 2 * dim + 1))
    Aa[:2 * dim, :2 * dim] = A
    Aa[dim:2 * dim, -1] = u0[:dim] / tau
    xv = scipy.linalg.expm(Aa * dt) @ np.concatenate([x0[:, 0], v0[:, 0], [1.0]])
    np.testing.assert_allclose(st.x[:, 0], xv[:dim], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(st.v[:, 0], xv[dim:2 * dim], rtol=1e-9, atol=1e-12)


def _abc_flow():
    return oracle.make_flow(oracle.FLOW_ABC, U=0.2, k=1.0, abc=(1.0, 0.8, 1.2), phase=(0.3, 1.1, 2.0))


def test_flow_gradients_match_finite_differences():
    for dim, flow in ((2, oracle.make_flow(oracle.FLOW_TAYLOR_GREEN, U=0.1, k=1.0, u0=(0.05, 0.0, 0.0))),
                      (3, _abc_flow())):
        rng = np.random.default_rng(dim)
        for _ in range(5):
            x = rng.uniform(size=dim)
            u, gu = oracle.flow_eval(dim, flow, x)
            eps = 1e-6
            for b in range(dim):
                e = np.zeros(dim)
                e[b] = eps
                fd = (oracle.flow_eval(dim, flow, x + e)[0] - oracle.flow_eval(dim, flow, x - e)[0]) / (2 * eps)
                np.testing.assert_allclose(gu[:, b], fd, rtol=1e-8, atol=1e-9)
            assert abs(np.trace(gu)) < 1e-12          # both fields are divergence-free


def test_jacobian_of_the_abc_flow_matches_finite_differences_of_the_map():
    """J(t) = dx(t)/dx0 for droplets seeded with the gas velocity (v0 = u(x0),
    so dv0/dx0 = grad u(x0)), against central differences of the end
    positions over perturbed seeds; with evaporation."""
    flow = _abc_flow()
    rng = np.random.default_rng(5)
    x0 = rng.uniform(size=3)
    r0, dt, delta, sub = 9e-6, 4e-3, -1e-9, 128

    def seed(x):
        u, gu = oracle.flow_eval(3, flow, x)
        return _state(x.reshape(3, 1), u.reshape(3, 1), [r0], gu.reshape(9, 1))

    st, _, _, _ = oracle.advance(seed(x0), flow, RHO, MU, delta, dt, sub)
    eps = 1e-6
    for b in range(3):
        e = np.zeros(3)
        e[b] = eps
        xp = oracle.advance(seed(x0 + e), flow, RHO, MU, delta, dt, sub)[0].x[:, 0]
        xm = oracle.advance(seed(x0 - e), flow, RHO, MU, delta, dt, sub)[0].x[:, 0]
        np.testing.assert_allclose(st.J[:, 0].reshape(3, 3)[:, b], (xp - xm) / (2 * eps), rtol=1e-7, atol=1e-8)


def test_contributions_are_the_droplet_mass_and_momentum_changes():
    """d(m)/dt = mdot and d(m v)/dt = F + mdot v, so the summed
    contributions over a step are m1 - m0 and m1 v1 - m0 v0 in any flow."""
    flow = _abc_flow()
    rng = np.random.default_rng(7)
    N = 20
    x0 = rng.uniform(size=(3, N))
    v0 = rng.normal(size=(3, N)) * 0.2
    r0 = rng.uniform(6e-6, 20e-6, N)
    dt = 3e-3
    st, phi, valid, sk = oracle.advance(_state(x0, v0, r0), flow, RHO, MU, -2e-9, dt, 128)
    assert sk == 0
    m0, m1 = _mass(r0), _mass(st.r)
    np.testing.assert_allclose(phi[0] * dt, m1 - m0, rtol=1e-9)
    np.testing.assert_allclose(phi[1:] * dt, m1 * st.v - m0 * v0, rtol=1e-8, atol=1e-9 * np.abs(m0 * v0).max())


def test_droplets_that_evaporate_within_the_step_are_skipped():
    x0 = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    v0 = np.zeros((2, 3))
    r0 = np.array([10e-6, 1e-6, float("nan")])
    # delta dt = -2e-12: the 1 um droplet (r^2 = 1e-12) vanishes
    st, phi, valid, sk = oracle.advance(_state(x0, v0, r0), oracle.make_flow(), RHO, MU, -1e-9, 2e-3, 16)
    assert valid.tolist() == [1, 0, 0] and sk == 2
    assert np.all(phi[:, 1:] == 0.0) and st.r[1] == 1e-6
    t = oracle.state_terms(st, phi, valid, 1e10, 0.01)
    assert t.valid.tolist() == [1, 0, 0] and t.skipped == 2
    assert t.h[0] == pytest.approx(0.01) and t.q[0, 0] == pytest.approx(1e10 * phi[0, 0])
