"""Parity of the learned-bandwidth kernels with the FP64 oracle.

Each side runs its own chain from the same seeded inputs (trajectories,
parameters, reference field); no GPU output feeds the oracle.

Tolerances: features to 1e-6 (the GPU forms singular values with the
closed-form 3x3 eigen-solution, the oracle with LAPACK); network outputs to
2e-3 absolute + relative, because a pre-activation that lands within one
binary32 rounding of a bf16 rounding boundary may round the other way on the
other side (a one-ulp bf16 step is 2^-8 relative); gradients through the
estimator to 1e-6 relative L2 on the binary64 path and 1e-5 on the binary32
one (binary32 per-cell planes); network gradients, alone and through the
whole chain, to 1e-3 relative L2 (bf16 inputs; deltas carried as bf16 hi +
lo pairs).  The measured errors are printed: about 6e-8 and 2e-6 for the
estimator backward, 3e-6 for the network backward and 1e-5 through the
chain."""
import numpy as np
import pytest
import torch

import oracle
import oracle.learned as LN
import workloads as W
from helpers import as_precision, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_20829_amd as F
    c = F.Context(0)
    yield c
    c.close()


def _theta(seed, f=None, last=0.3):
    rng = np.random.default_rng(seed)
    mu = sd = None
    if f is not None:
        mu, sd = f.mean(axis=1), f.std(axis=1) + 1e-3
    th = LN.init_params(seed, mu, sd)
    p = LN.unpack(th)
    p["w3"] = rng.standard_normal(64) * last
    p["b1"] = rng.standard_normal(64) * 0.1
    p["b2"] = rng.standard_normal(64) * 0.1
    p["b3"] = np.array([0.05])
    return LN.pack(p).astype(np.float32).astype(np.float64)


def _traj_struct(tr, prec):
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    return F.make_trajectories(tr.x.to(DEV), tr.J.to(DEV), tr.v.to(DEV, dt), tr.ug.to(DEV, dt), tr.r.to(DEV, dt),
                               tr.n0, tr.seed_volume)


def _gpu_forward(ctx, wl, theta, prec="f32"):
    import paper_2512_20829_amd as F
    st, keep = _traj_struct(wl.traj, prec)
    N = wl.traj.count
    th = torch.tensor(theta, dtype=torch.float32, device=DEV)
    hf = torch.empty(N, dtype=torch.float32, device=DEV)
    z = torch.empty(5 * N, dtype=torch.float32, device=DEV)
    o = torch.empty(N, dtype=torch.float32, device=DEV)
    fr = torch.empty(5 * N, dtype=torch.float32, device=DEV)
    ctx.bandwidth_forward(F.mesh_of(wl.mesh), st, th, hf, z, o, fr)
    torch.cuda.synchronize()
    return (hf.cpu().double().numpy(), z.cpu().double().numpy().reshape(5, N), o.cpu().double().numpy(),
            fr.cpu().double().numpy().reshape(5, N))


def _oracle_forward(wl, theta, prec="f32"):
    tr = as_precision(wl.traj, prec)
    t = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
    f = LN.features(wl.mesh, tr.x.numpy(), tr.J.numpy(), t.valid)
    return LN.forward(theta, f), f, t


@pytest.mark.parametrize("dim", [3, 2])
def test_features_and_network_forward(ctx, dim):
    if dim == 3:
        wl = W.small_random_3d(3000, 16, seed=21)
    else:
        wl = W.taylor_green_2d(per_axis=48, mesh_n=40)
    _, f0, _ = _oracle_forward(wl, LN.init_params(0))
    theta = _theta(21, f0)
    hf, z, o, fr = _gpu_forward(ctx, wl, theta)
    fw, f, t = _oracle_forward(wl, theta)
    v = t.valid == 1
    np.testing.assert_allclose(fr[:, v], f[:, v], rtol=1e-6, atol=1e-6)
    assert np.mean(z[:, v] == fw.z[:, v]) > 0.999
    err = np.abs(o - fw.o)
    assert np.all(err[v] <= 2e-3 * (1 + np.abs(fw.o[v]))), err.max()
    assert np.median(err[v]) <= 1e-5
    np.testing.assert_allclose(hf[v], fw.g[v], rtol=4e-3)
    assert np.all(hf[~v] == 1.0)


def test_zero_last_layer_reproduces_the_plain_projection_bitwise(ctx):
    from helpers import gpu_run
    wl = W.small_random_3d(4000, 20, seed=22)
    theta = LN.init_params(22)                       # w3 = 0, b3 = 0  ->  g = 1 exactly
    hf, _, _, _ = _gpu_forward(ctx, wl, theta)
    assert np.all(hf == 1.0)
    S0, d0, _ = gpu_run(ctx, wl, prec="f32")
    S1, d1, _ = gpu_run(ctx, wl, prec="f32", h_factor=torch.tensor(hf, dtype=torch.float32))
    assert np.array_equal(S0, S1) and np.array_equal(d0, d1)


def _gpu_chain(ctx, wl, theta, R, prec):
    """forward network -> projection -> loss -> estimator backward -> network backward"""
    import paper_2512_20829_amd as F
    dt = torch.float64 if prec == "f64" else torch.float32
    st, keep = _traj_struct(wl.traj, prec)
    N, M = wl.traj.count, wl.mesh.cells
    mesh = F.mesh_of(wl.mesh)
    th = torch.tensor(theta, dtype=torch.float32, device=DEV)
    hf = torch.empty(N, dtype=torch.float32, device=DEV)
    z = torch.empty(5 * N, dtype=torch.float32, device=DEV)
    o = torch.empty(N, dtype=torch.float32, device=DEV)
    ctx.bandwidth_forward(mesh, st, th, hf, z, o)
    p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, h_factor=hf)
    Sm, Sv, den = F.alloc_fields(M, 3, dt, DEV)
    ctx.project_sources(mesh, st, p, Sm, Sv, den)
    Rt = [torch.tensor(R[k], dtype=dt, device=DEV) for k in range(4)]
    G = [torch.empty(M, dtype=dt, device=DEV) for _ in range(4)]
    res = ctx.rel_l2_loss(4, M, F.FLA_F64 if prec == "f64" else F.FLA_F32, [Sm, *Sv], Rt, G)
    dlogh = torch.empty(N, dtype=torch.float32, device=DEV)
    ctx.project_backward(mesh, st, p, Sm, Sv, den, G[0], G[1:], dlogh)
    grad = torch.empty(F.MLP_PARAMS, dtype=torch.float32, device=DEV)
    ctx.bandwidth_backward(3, th, N, z, o, dlogh, grad)
    torch.cuda.synchronize()
    return (res.cpu().numpy(), dlogh.cpu().double().numpy(), grad.cpu().double().numpy(),
            torch.stack([Sm, *Sv]).double().cpu().numpy())


def _oracle_chain(wl, theta, R, prec):
    fw, f, t = _oracle_forward(wl, theta, prec)
    tr = as_precision(wl.traj, prec)
    t2 = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0, h_factor=fw.g)
    p = oracle.nw_cells(wl.mesh, tr.x, t2, cutoff=wl.cutoff, f32_decision=(prec == "f32"))
    L, dLdS = LN.rel_l2_loss(p.S, R)
    dh = LN.dL_dh(wl.mesh, tr.x.numpy(), t2.h, t2.q, t2.valid, p.S, p.den, dLdS, cutoff=wl.cutoff)
    dlogh = dh * t2.h
    grad = LN.backward(theta, fw, LN.dL_do_from_dL_dh(dh, t2.h, fw.o))
    return L, dlogh, grad, p.S


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_gradient_chain_matches_oracle(ctx, prec):
    wl = W.small_random_3d(700, 12, seed=23)
    _, f0, _ = _oracle_forward(wl, LN.init_params(0))
    theta = _theta(23, f0, last=0.2)
    rng = np.random.default_rng(23)
    Lr, _, _, Sr = _oracle_chain(wl, theta, np.ones((4, wl.mesh.cells)), prec)
    R = Sr * (1.0 + 0.3 * rng.standard_normal(Sr.shape))        # a perturbed reference field
    res, dlogh, grad, S = _gpu_chain(ctx, wl, theta, R, prec)
    L, dlogh_ref, grad_ref, S_ref = _oracle_chain(wl, theta, R, prec)
    eS, ed, eg = rel_l2(S, S_ref), rel_l2(dlogh, dlogh_ref), rel_l2(grad[:LN.N_TRAIN], grad_ref[:LN.N_TRAIN])
    print(f"[gradient-chain] {prec}: S {eS:.2e} loss {abs(res[0] / L - 1):.2e} dL/dlog h {ed:.2e} "
          f"dL/dtheta {eg:.2e}", flush=True)
    assert eS < 1e-4
    assert res[0] == pytest.approx(L, rel=1e-4)
    assert ed < 1e-3
    assert eg < 1e-3
    assert np.all(grad[LN.N_TRAIN:] == 0.0)


def test_estimator_backward_with_shared_factors(ctx):
    """With the bandwidth factors of a fixed, seeded vector (no network), the
    estimator backward matches the oracle to FP32 accuracy."""
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(600, 12, seed=24)
    N, M = wl.traj.count, wl.mesh.cells
    rng = np.random.default_rng(24)
    hf = np.exp(0.3 * rng.standard_normal(N)).astype(np.float32).astype(np.float64)
    for prec in ("f32", "f64"):
        dt = torch.float64 if prec == "f64" else torch.float32
        tr = as_precision(wl.traj, prec)
        t = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0, h_factor=hf)
        p = oracle.nw_cells(wl.mesh, tr.x, t, cutoff=wl.cutoff, f32_decision=(prec == "f32"))
        R = p.S * (1.0 + 0.2 * rng.standard_normal(p.S.shape))
        L, dLdS = LN.rel_l2_loss(p.S, R)
        ref = LN.dL_dh(wl.mesh, tr.x.numpy(), t.h, t.q, t.valid, p.S, p.den, dLdS, cutoff=wl.cutoff) * t.h
        st, keep = _traj_struct(wl.traj, prec)
        mesh = F.mesh_of(wl.mesh)
        hft = torch.tensor(hf, dtype=torch.float32, device=DEV)
        prm = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff, h_factor=hft)
        Sm, Sv, den = F.alloc_fields(M, 3, dt, DEV)
        ctx.project_sources(mesh, st, prm, Sm, Sv, den)
        Rt = [torch.tensor(R[k], dtype=dt, device=DEV) for k in range(4)]
        G = [torch.empty(M, dtype=dt, device=DEV) for _ in range(4)]
        res = ctx.rel_l2_loss(4, M, F.FLA_F64 if prec == "f64" else F.FLA_F32, [Sm, *Sv], Rt, G)
        out = torch.empty(N, dtype=torch.float32, device=DEV)
        ctx.project_backward(mesh, st, prm, Sm, Sv, den, G[0], G[1:], out)
        torch.cuda.synchronize()
        assert float(res[0]) == pytest.approx(L, rel=1e-5 if prec == "f32" else 1e-10)
        e = rel_l2(out.cpu().double().numpy(), ref)
        print(f"[estimator-backward] {prec}: rel L2 {e:.2e}", flush=True)
        assert e < (1e-5 if prec == "f32" else 1e-6)


def test_network_backward_and_adam(ctx):
    import paper_2512_20829_amd as F
    wl = W.small_random_3d(5000, 16, seed=25)
    _, f0, _ = _oracle_forward(wl, LN.init_params(0))
    theta = _theta(25, f0)
    hf, z, o, _ = _gpu_forward(ctx, wl, theta)
    fw, _, t = _oracle_forward(wl, theta)
    N = wl.traj.count
    rng = np.random.default_rng(25)
    dlogh = (rng.standard_normal(N) * (t.valid == 1)).astype(np.float32).astype(np.float64)
    th = torch.tensor(theta, dtype=torch.float32, device=DEV)
    grad = torch.empty(F.MLP_PARAMS, dtype=torch.float32, device=DEV)
    ctx.bandwidth_backward(3, th, N, torch.tensor(z.reshape(-1), dtype=torch.float32, device=DEV),
                           torch.tensor(o, dtype=torch.float32, device=DEV),
                           torch.tensor(dlogh, dtype=torch.float32, device=DEV), grad)
    torch.cuda.synchronize()
    ref = LN.backward(theta, fw, dlogh * LN.S_MAX * (1 - np.tanh(fw.o) ** 2))
    g = grad.cpu().double().numpy()
    eg = rel_l2(g[:LN.N_TRAIN], ref[:LN.N_TRAIN])
    print(f"[network-backward] rel L2 {eg:.2e}", flush=True)
    assert eg < 1e-3
    # Adam on a seeded gradient
    gs = rng.standard_normal(F.MLP_PARAMS).astype(np.float32).astype(np.float64)
    m = torch.zeros(F.MLP_PARAMS, dtype=torch.float32, device=DEV)
    v = torch.zeros_like(m)
    th2 = th.clone()
    ctx.adam_step(th2, m, v, torch.tensor(gs, dtype=torch.float32, device=DEV), 1, lr=1e-3)
    torch.cuda.synchronize()
    t1, m1, v1 = LN.adam(theta, gs, np.zeros_like(theta), np.zeros_like(theta), 1, lr=1e-3)
    np.testing.assert_allclose(th2.cpu().double().numpy(), t1, rtol=1e-6, atol=1e-9)
    # steps 2 and 3 with new gradients: the bias corrections 1 - b^step
    tk, mk, vk = t1, m1, v1
    for step in (2, 3):
        gk = rng.standard_normal(F.MLP_PARAMS).astype(np.float32).astype(np.float64)
        ctx.adam_step(th2, m, v, torch.tensor(gk, dtype=torch.float32, device=DEV), step, lr=1e-3)
        torch.cuda.synchronize()
        tk, mk, vk = LN.adam(tk, gk, mk, vk, step, lr=1e-3)
        np.testing.assert_allclose(th2.cpu().double().numpy(), tk, rtol=1e-6, atol=1e-9)
        # moments of the trainable entries (binary32 on the GPU: an absolute floor for cancellation)
        T = slice(0, LN.N_TRAIN)
        np.testing.assert_allclose(m.cpu().double().numpy()[T], mk[T], rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(v.cpu().double().numpy()[T], vk[T], rtol=1e-5, atol=1e-9)


@pytest.mark.slow
@pytest.mark.timeout(400)
def test_learned_form_full_size(ctx):
    """The learned form on the 128^3 / 2M-trajectory ABC evaluation case:
    features, network output and factor of every trajectory against the
    oracle, then the projection with the oracle's factors on 256 sampled
    cells (the factors are an input of the projection)."""
    from helpers import gpu_run, oracle_run
    wl = W.abc_lattice_3d()
    print(f"[case] learned full size N={wl.traj.count}", flush=True)
    _, f0, _ = _oracle_forward(wl, LN.init_params(0))
    theta = _theta(23, f0)
    hf, z, o, fr = _gpu_forward(ctx, wl, theta)
    fw, f, t = _oracle_forward(wl, theta)
    _check_large_forward(theta, hf, z, o, fr, fw, f, t)
    g32 = torch.tensor(fw.g, dtype=torch.float32)
    S, den, st = gpu_run(ctx, wl, prec="f32", count_pairs=False, h_factor=g32)
    cells = np.sort(np.random.default_rng(2).choice(wl.mesh.cells, 256, replace=False))
    oracle.set_threads(16)
    ref, _ = oracle_run(wl, prec="f32", cells=cells, h_factor=g32)
    for k in range(ref.S.shape[0]):
        assert rel_l2(S[k, cells], ref.S[k]) <= 1e-5, k
    assert rel_l2(den[cells], ref.den) <= 1e-5


def test_forward_ragged_steps_with_invalid_trajectories(ctx):
    """700,001 random trajectories (more than one wave step of the network
    kernel, the last one partial), every 997th with a non-finite J entry:
    features, network output and factor against the oracle, and factor 1
    for the invalid ones."""
    wl = W.small_random_3d(700_001, 64, seed=31)
    bad = np.arange(5, wl.traj.count, 997)
    wl.traj.J[4, torch.from_numpy(bad)] = float("nan")
    print(f"[case] learned ragged N={wl.traj.count}, {bad.size} invalid", flush=True)
    _, f0, _ = _oracle_forward(wl, LN.init_params(0))
    theta = _theta(31, f0)
    hf, z, o, fr = _gpu_forward(ctx, wl, theta)
    fw, f, t = _oracle_forward(wl, theta)
    assert np.all(t.valid[bad] == 0) and int(np.sum(t.valid == 0)) == bad.size
    _check_large_forward(theta, hf, z, o, fr, fw, f, t)
    assert np.all(hf[bad] == 1.0) and np.all(o[bad] == 0.0)
    assert np.all(np.isnan(fr[:, bad])) and np.all(z[:, bad] == 0.0)


def _check_large_forward(theta, hf, z, o, fr, fw, f, t):
    """Features, bf16 inputs, network output and factor of a large forward
    against the oracle, within the bound of first-layer bf16 flips."""
    v = t.valid == 1
    np.testing.assert_allclose(fr[:, v], f[:, v], rtol=1e-6, atol=1e-6)
    assert np.mean(z[:, v] == fw.z[:, v]) > 0.999
    err = np.abs(o - fw.o)
    # The GPU forms first-layer pre-activations in binary32 (MFMA), the
    # oracle in binary64, and both round the activations to bf16: where a
    # value lies within one binary32 rounding of a bf16 midpoint the two
    # sides round it to neighbouring bf16 values, one ulp (at most 2^-7 of
    # the magnitude) apart.  Per trajectory, the output can then differ by at
    # most the effect of every first-layer activation moving by one ulp,
    # propagated through the oracle's second and output layers (linearised,
    # with a 1.5 margin for the change of the SiLU slope), plus binary32
    # rounding.  Such flips are rare: few outputs leave the 2e-3 band.
    p = LN.unpack(theta)
    W2, w3 = LN.bf16(p["W2"]), LN.bf16(p["w3"])
    do_dh1 = (w3[:, None] * LN.dsilu(fw.a2)).T @ W2
    bound = 1.5 * 2.0 ** -7 * np.sum(np.abs(fw.h1.T) * np.abs(do_dh1), axis=1) + 1e-5 * (1 + np.abs(fw.o))
    assert np.all(err[v] <= bound[v]), (err[v] - bound[v]).max()
    assert np.mean(err[v] > 2e-3 * (1 + np.abs(fw.o[v]))) <= 1e-4
    assert np.median(err[v]) <= 1e-5
    # the factor g = exp(s_max tanh o) moves by s_max sech^2(o) |do| relative
    # to itself, so the same bound carries over (plus binary32 rounding of
    # tanh and exp)
    smax = np.log(4.0)
    gbound = smax * (1.0 - np.tanh(fw.o) ** 2) * bound + 1e-6
    assert np.all(np.abs(hf[v] - fw.g[v]) <= gbound[v] * fw.g[v]), \
        (np.abs(hf[v] - fw.g[v]) / fw.g[v] - gbound[v]).max()
    assert np.mean(np.abs(hf[v] - fw.g[v]) > 4e-3 * fw.g[v]) <= 1e-4
