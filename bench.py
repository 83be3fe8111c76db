#!/usr/bin/env python3
"""Benchmark of the FLA source projection on one MI355X.

Workload: the 3-D ABC-map case -- 128^3 periodic mesh on the unit cube,
2,097,152 lattice trajectories deformed by an ABC map of amplitude 0.2 (with
folds), radius lognormal(ln 10 um, 0.3), h0 = 1/128, cutoff 4 bandwidths,
binary32 kernel evaluation with binary64 det J.  Inputs are synthetic and
generated on the GPU before timing; they are resident in HBM when the timed
region starts.

One step = one fla_project_sources call: prepass (det J, n, h, physics,
keys), key sort and bucket bounds, record permutation, and the gather with
its fused epilogue.  Printed as one JSON line (rank 0):
  value        mesh cells per second (M / step time)
  pairs_per_s  included trajectory-cell pairs per second
  roofline     the gather kernel, timed with HIP events on the library's
               stream: algorithmic flops per launch / average launch time
  large        the 256^3 multi-vortex case (32.8M trajectories, caustics):
               plain and learned throughput, plain / learned / deposition
               errors against a 1.68G-particle PSI-CELL reference
  cpu_baseline the FP64 oracle on a bounded sample of the same workload
  batch        64 uneven snapshots (32^3..128^3 meshes, 10k..2M trajectories)
               through fla_project_batch: graph replays, direct launches and
               one single call per snapshot, after the batch autotuner
  psicell      PSI-CELL accumulation of a 200M-particle cloud (context)
  learned_vs_plain  the learned bandwidth network trained on 500 generated
               64^3 snapshots (200k trajectories, 50M-particle PSI-CELL each),
               then plain, learned and deposition errors on the 128^3 case at
               2M..125k lattice trajectories against the 200M-particle
               reference, and cells/s of both forms
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "mesh cells/s + traj-cell pairs/s; learned vs plain form at fixed rel L2 error"
# Algorithmic work of one included (cell, trajectory) pair in 3-D with C = 4
# channels, evaluated directly from the kernel and estimator definitions:
# 3 offsets, |d|^2 (3 mul + 2 add), scaling by 1/(2h^2) (1), exp (1), the
# denominator add (1) and 4 numerator multiply-adds (8) = 19 flops.
FLOPS_PER_PAIR_3D = 19
# Non-packed fp32 vector peak: 256 CUs x 64 lanes x 2.4 GHz x 2 flops/FMA.
# The library is compiled with packed fp32 instructions disabled, so the
# packed figure (157.3 TFLOP/s) is out of reach by construction.
ALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 * 2 / 1e12
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gather_traffic():
    """HBM bytes per gather launch from the committed counter summary, or None
    when the gather source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gather_abc128_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2512_20829_amd", "csrc", "gather.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].rsplit(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("gather.hip sha256[:16]") != digest:
        return None
    try:
        return float(vals["bytes per launch (calibrated)"])
    except (KeyError, ValueError):
        return None


def _psicell_reference(ctx, F, W, torch, mesh, abc, n_particles, seed, params, dev):
    """Dense PSI-CELL reference as the mean of two independent half clouds,
    with the per-channel noise floor |A - B|^2 / (4 |R|^2)."""
    halves = []
    for h in range(2):
        cl = W.abc_cloud(n_particles // 2, seed=seed, device=dev, abc=abc, jacobian=False, offset=h * (n_particles // 2))
        st, keep = F.make_trajectories(cl.x, None, cl.v.float(), cl.ug.float(), cl.r.float(), 1.0)
        Sm, Sv, _ = F.alloc_fields(mesh.cells, mesh.dim, torch.float32, dev, den=False)
        ctx.psicell_accumulate(F.mesh_of(mesh), st, W.N0_DEFAULT / (n_particles // 2), params, Sm, Sv)
        halves.append([Sm, *Sv])
        del cl, st, keep
    ref = [(a + b) * 0.5 for a, b in zip(*halves)]
    floor = [float(((a - b) ** 2).double().sum() / (4 * (r.double() ** 2).sum())) for a, b, r in zip(*halves, ref)]
    return ref, floor


def _psicell_reference_chunked(ctx, F, torch, mesh, cloud_fn, n_particles, chunk, params, dev):
    """Dense PSI-CELL reference as the mean of two independent half clouds,
    each accumulated in chunks of at most `chunk` particles (cloud_fn(n,
    offset) draws particles offset..offset+n-1 of one seeded stream), with
    the per-channel noise floor |A - B|^2 / (4 |R|^2)."""
    import workloads as W
    half = n_particles // 2
    halves = []
    for h in range(2):
        acc, done = None, 0
        while done < half:
            n = min(chunk, half - done)
            cl = cloud_fn(n, h * half + done)
            st, keep = F.make_trajectories(cl.x, None, cl.v.float(), cl.ug.float(), cl.r.float(), 1.0)
            del cl
            Sm, Sv, _ = F.alloc_fields(mesh.cells, mesh.dim, torch.float32, dev, den=False)
            ctx.psicell_accumulate(F.mesh_of(mesh), st, W.N0_DEFAULT / half, params, Sm, Sv)
            part = [t.double() for t in (Sm, *Sv)]
            acc = part if acc is None else [a + b for a, b in zip(acc, part)]
            del st, keep, Sm, Sv, part
            done += n
        halves.append(acc)
    ref = [((a + b) * 0.5).float() for a, b in zip(*halves)]
    floor = [float(((a - b) ** 2).sum() / ((a + b) ** 2).sum()) for a, b in zip(*halves)]
    del halves
    torch.cuda.empty_cache()
    return ref, floor


def large_section(ctx, args, dev, model):
    """The 256^3 multi-vortex case with strong caustics: 32.8M lattice
    trajectories (320^3), plain throughput, and the plain, learned (the
    network trained on the 64^3 ABC snapshots, if available) and deposition
    errors against a chunked PSI-CELL reference, at 320^3, 256^3 and 200^3
    trajectories."""
    import numpy as np
    import torch

    import paper_2512_20829_amd as F
    import workloads as W
    from paper_2512_20829_amd import train as T

    t0 = time.time()
    mesh = W.unit_mesh(3, 256, True)
    p = F.Params(rho_d=W.RHO_D, mu=W.MU_AIR, delta=W.DELTA_EVAP, h0=1.0 / 320, cutoff=4.0)
    ref, floor = _psicell_reference_chunked(
        ctx, F, torch, mesh, lambda n, off: W.multi_vortex_cloud(n, seed=0, device=dev, offset=off),
        args.large_particles, 200_000_000, p, dev)
    log(f"large: PSI-CELL reference of {args.large_particles} particles in {time.time() - t0:.1f} s; "
        f"noise floor {[round(math.sqrt(f), 4) for f in floor]}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows, perf = [], None
    for pa in (320, 256, 200):
        wl = W.multi_vortex_lattice_3d(per_axis=pa, mesh_n=256, device=dev)
        tr = wl.traj
        st, keep = F.make_trajectories(tr.x, tr.J, tr.v.float(), tr.ug.float(), tr.r.float(), tr.n0, tr.seed_volume)
        wl.traj = None
        del tr
        prm = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
        snap = T.Snapshot(wl.mesh, st, keep, pa ** 3, prm, ref)
        M = wl.mesh.cells
        Sm, Sv, den = F.alloc_fields(M, 3, torch.float32, dev)
        out = {"trajectories": pa ** 3}
        if pa == 320:
            counted = F.Params(**{**prm.__dict__, "count_pairs": True})
            ctx.project_sources(F.mesh_of(wl.mesh), st, counted, Sm, Sv, den)
            torch.cuda.synchronize()
            stt = ctx.stats()
            reps = 3
            forms = [("plain", None)] + ([("learned", model)] if model is not None else [])
            perf = {"pairs": stt["pairs"], "skipped": stt["skipped"], "no_support": stt["no_support"],
                    "max_class": stt["max_class"]}
            for name, mdl in forms:
                ctx.project_sources(F.mesh_of(wl.mesh), st, prm, Sm, Sv)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    h = mdl.factors(snap)[0] if mdl is not None else None
                    ctx.project_sources(F.mesh_of(wl.mesh), st, F.Params(**{**prm.__dict__, "h_factor": h}), Sm, Sv)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                perf[f"ms_{name}"] = round(ms, 3)
                perf[f"cells_per_s_{name}"] = M / (ms * 1e-3)
            perf["pairs_per_s_plain"] = stt["pairs"] / (perf["ms_plain"] * 1e-3)
        helper = model if model is not None else T.BandwidthModel(ctx, T.initial_theta(0))
        forms = [("plain", None, F.FLA_NW), ("deposit", None, F.FLA_DEPOSIT)]
        if model is not None:
            forms.insert(1, ("learned", model.factors(snap)[0], F.FLA_NW))
        for name, h, mode in forms:
            q = F.Params(**{**prm.__dict__, "h_factor": h, "mode": mode})
            ctx.project_sources(F.mesh_of(wl.mesh), st, q, Sm, Sv, den)
            res, _ = helper.loss(snap, [Sm, *Sv], False)
            r = res.cpu().numpy()
            out[name] = round(float(np.mean([math.sqrt(max(r[1 + 2 * k] / r[2 + 2 * k] - floor[k], 0.0))
                                             for k in range(4)])), 5)
        rows.append(out)
        log(f"large: {out}")
        del snap, st, keep, Sm, Sv, den, wl
        torch.cuda.empty_cache()
    target = rows[0]["plain"]
    matched = [r["trajectories"] for r in rows if "learned" in r and r["learned"] <= target]
    return {"workload": "3-D multi-vortex map (two ABC maps, amplitudes 0.2 and 0.1, wavenumbers 1 and 2), "
                        "256^3 periodic mesh, 320^3 lattice trajectories, h0 = 1/320, FP32 kernel with FP64 det J",
            "performance": perf,
            "reference": {"psicell_particles": args.large_particles,
                          "noise_floor_rel_l2": [round(math.sqrt(f), 4) for f in floor]},
            "error": "mean over the 4 source fields of the noise-debiased rel L2 against dense PSI-CELL",
            "eval": rows, "plain_error_at_32.8M": target,
            "fewest_trajectories_learned_within_plain_error": min(matched) if matched else None}


def learned_vs_plain(ctx, args, dev):
    """Train the bandwidth network on the library's own projections of 64^3
    snapshots against dense PSI-CELL, then compare plain and learned forms
    (and the conservative deposition) on the 128^3 ABC case at several
    seeding densities against the 200M-particle reference."""
    import numpy as np
    import torch

    import paper_2512_20829_amd as F
    import workloads as W
    from paper_2512_20829_amd import train as T

    def snap_of(wl, ref):
        tr = wl.traj
        st, keep = F.make_trajectories(tr.x, tr.J, tr.v.float(), tr.ug.float(), tr.r.float(), tr.n0, tr.seed_volume)
        keep.append(tr)
        p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
        return T.Snapshot(wl.mesh, st, keep, tr.count, p, ref)

    t0 = time.perf_counter()
    train = []
    for s in range(args.train_snapshots):
        wl, abc = W.training_snapshot(s, n_traj=args.train_trajectories, mesh_n=64, device=dev)
        p = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
        ref, _ = _psicell_reference(ctx, F, W, torch, wl.mesh, abc, args.train_particles, 10_000 + s, p, dev)
        train.append(snap_of(wl, ref))
        if s % 100 == 99:
            log(f"training snapshots: {s + 1}")
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    wl2 = W.abc_lattice_3d(device=dev)
    p2 = F.Params(rho_d=wl2.rho_d, mu=wl2.mu, delta=wl2.delta, h0=wl2.h0, cutoff=wl2.cutoff)
    ref2, floor = _psicell_reference(ctx, F, W, torch, wl2.mesh, W.ABC(), args.psicell_particles, 0, p2, dev)
    del wl2
    theta = T.fit_standardisation(ctx, train[:16], T.initial_theta(0))
    model = T.BandwidthModel(ctx, theta, lr=1e-3)
    t0 = time.perf_counter()
    for it in range(args.train_steps):
        model.train_step(train[it % len(train)])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained {args.train_steps} steps on {len(train)} snapshots in {t_train:.1f} s (data {t_data:.1f} s)")
    del train

    def deb(res):
        r = res.cpu().numpy()
        e = [math.sqrt(max(r[1 + 2 * k] / r[2 + 2 * k] - floor[k], 0.0)) for k in range(4)]
        return float(np.mean(e))

    rows = []
    for pa in (128, 100, 80, 64, 50):
        wl = W.abc_lattice_3d(per_axis=pa, mesh_n=128, device=dev)
        sn = snap_of(wl, ref2)
        out = {"trajectories": pa ** 3}
        hf = model.factors(sn)[0]
        for name, h, mode in (("plain", None, F.FLA_NW), ("learned", hf, F.FLA_NW), ("deposit", None, F.FLA_DEPOSIT)):
            prm = F.Params(**{**sn.params.__dict__, "h_factor": h, "mode": mode})
            Sm, Sv, den = F.alloc_fields(sn.cells, 3, torch.float32, dev)
            ctx.project_sources(F.mesh_of(wl.mesh), sn.traj, prm, Sm, Sv, den)
            res, _ = model.loss(sn, [Sm, *Sv], False)
            out[name] = round(deb(res), 5)
        rows.append(out)
        if pa == 128:
            # throughput of both forms on the full workload (the learned form
            # includes the feature and network kernels)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            Sm, Sv, den = F.alloc_fields(sn.cells, 3, torch.float32, dev, den=False)
            for learned in (False, True):
                for rep in range(args.warmup + args.steps):
                    if rep == args.warmup:
                        e0.record()
                    h = model.factors(sn)[0] if learned else None
                    ctx.project_sources(F.mesh_of(wl.mesh), sn.traj, F.Params(**{**sn.params.__dict__, "h_factor": h}),
                                        Sm, Sv)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                out["cells_per_s_learned" if learned else "cells_per_s_plain"] = sn.cells / (ms * 1e-3)
        del sn, wl
    target = rows[0]["plain"]
    matched = [r["trajectories"] for r in rows if r["learned"] <= target]
    return model, {
        "train": {"snapshots": args.train_snapshots, "trajectories": args.train_trajectories, "mesh": [64, 64, 64],
                  "psicell_particles": args.train_particles, "steps": args.train_steps, "seconds": round(t_train, 2)},
        "reference": {"psicell_particles": args.psicell_particles, "noise_floor_rel_l2": [round(math.sqrt(f), 4) for f in floor]},
        "error": "mean over the 4 source fields of the noise-debiased rel L2 against dense PSI-CELL",
        "eval": rows,
        "plain_error_at_2M": target,
        "fewest_trajectories_learned_within_plain_error_at_2M": min(matched) if matched else None,
    }


def batch_section(ctx, args, dev):
    """The uneven batch: 64 snapshots, meshes 32^3..128^3, 10k..2M random
    trajectories each through ABC maps of random amplitude and phase, FP32.
    Times graph replays of fla_project_batch after the batch autotuner has
    chosen the gather plan and XCD chunk, direct launches of the same batch,
    and one fla_project_sources call per snapshot for comparison."""
    import torch

    import paper_2512_20829_amd as F
    import workloads as W

    t0 = time.time()
    wls = [W.uneven_snapshot(s, device=dev) for s in range(args.batch_snapshots)]
    meshes, trajs, keeps, outs, params = [], [], [], [], []
    for wl in wls:
        tr = wl.traj
        st, keep = F.make_trajectories(tr.x.contiguous(), tr.J.contiguous(), tr.v.to(torch.float32).contiguous(),
                                       tr.ug.to(torch.float32).contiguous(), tr.r.to(torch.float32).contiguous(),
                                       tr.n0, tr.seed_volume)
        wl.traj = None
        meshes.append(F.mesh_of(wl.mesh))
        trajs.append(st)
        keeps.append(keep)
        Sm, Sv, _ = F.alloc_fields(wl.mesh.cells, 3, torch.float32, dev, den=False)
        outs.append((Sm, Sv, None))
        params.append(F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff))
    torch.cuda.synchronize()
    N = sum(t.count for t in trajs)
    M = sum(wl.mesh.cells for wl in wls)
    log(f"batch: {len(wls)} snapshots, {N} trajectories, {M} cells (generated in {time.time() - t0:.1f} s)")

    counted = [F.Params(**{**p.__dict__, "count_pairs": True}) for p in params]
    ctx.set_batch_graph(False)
    ctx.project_batch(meshes, trajs, counted, outs)
    torch.cuda.synchronize()
    P = ctx.stats()["pairs"]
    times = ctx.autotune_batch(meshes, trajs, params, outs)
    plan, chunk = ctx.get_batch_plan(3, F.FLA_F32)
    log(f"batch autotune: plan {plan}, chunk {chunk}; gather ms {[round(t, 3) for t in times]}")

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    run = lambda: ctx.project_batch(meshes, trajs, params, outs)
    ms_direct = timed(run, args.steps)
    ctx.profile_enable(True)
    for _ in range(3):
        run()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    stages = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items() if v[1]}
    g_ms = stages["gather"]

    ctx.set_batch_graph(True)
    r0 = ctx.stats()["graph_replays"]
    ms_graph = timed(run, args.steps)
    replays = ctx.stats()["graph_replays"] - r0

    def singles():
        for m, t, p, o in zip(meshes, trajs, params, outs):
            ctx.project_sources(m, t, p, o[0], o[1])
    ctx.set_plan(3, F.FLA_F32, plan)
    ms_single = timed(singles, max(args.steps // 4, 2))
    ctx.set_plan(3, F.FLA_F32, -1)
    achieved = P * FLOPS_PER_PAIR_3D / (g_ms * 1e-3) / 1e12
    log(f"batch: graph {ms_graph:.3f} ms, direct {ms_direct:.3f} ms, 64 single calls {ms_single:.3f} ms; "
        f"stages {stages}")
    out = {"workload": "64 uneven snapshots: meshes round(32*4^u)^3 (32^3..128^3), round(1e4*200^u') random "
                       "trajectories (10k..2M), ABC amplitude U[0.05, 0.2] with random phases, h0 = N^(-1/3), FP32",
           "snapshots": len(wls), "trajectories": N, "cells": M, "pairs": P,
           "ms_graph": round(ms_graph, 4), "ms_direct": round(ms_direct, 4),
           "ms_single_calls": round(ms_single, 4), "graph_replays": replays,
           "cells_per_s": M / (ms_graph * 1e-3), "pairs_per_s": P / (ms_graph * 1e-3),
           "stage_ms": stages, "plan": plan, "chunk": chunk,
           "autotune_gather_ms": [round(t, 4) for t in times],
           "gather": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                      "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "launch_ms": g_ms,
                      "kernel": "k_gather_batch<float,3,NW>"}}
    del wls, trajs, keeps, outs
    torch.cuda.empty_cache()
    return out


def cpu_baseline(seconds: float):
    """FP64 oracle, brute force per cell, on a random sample of cells of the
    same workload; full-field time extrapolated from the sample."""
    import numpy as np
    import torch

    import oracle
    import workloads as W
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    wl = W.abc_lattice_3d(device="cpu")
    f = lambda t: t.to(torch.float32).to(torch.float64)
    tr = W.Trajectories(wl.traj.x, wl.traj.J, f(wl.traj.v), f(wl.traj.ug), f(wl.traj.r), wl.traj.n0)
    t0 = time.perf_counter()
    terms = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
    t_terms = time.perf_counter() - t0
    M = wl.mesh.cells
    rng = np.random.default_rng(0)
    probe = rng.choice(M, 4 * cores, replace=False)
    t0 = time.perf_counter()
    oracle.nw_cells(wl.mesh, tr.x, terms, probe, wl.cutoff, True)
    per_cell = (time.perf_counter() - t0) / probe.size
    n = int(min(M, max(probe.size, seconds / per_cell)))
    cells = rng.choice(M, n, replace=False)
    t0 = time.perf_counter()
    oracle.nw_cells(wl.mesh, tr.x, terms, cells, wl.cutoff, True)
    t_cells = time.perf_counter() - t0
    full = t_terms + t_cells * M / n
    return {
        "value": M / full,
        "unit": "cells/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"{n} random cells of the 128^3 mesh, each by brute force over all "
                   f"{tr.count} trajectories, plus the per-trajectory terms of all trajectories "
                   f"({t_terms:.2f} s); full field extrapolated as t_terms + t_cells*M/n = {full:.0f} s"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-psicell", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch section")
    ap.add_argument("--no-large", action="store_true", help="skip the 256^3 multi-vortex section")
    ap.add_argument("--large-particles", type=int, default=1_677_721_600)
    ap.add_argument("--batch-snapshots", type=int, default=64)
    ap.add_argument("--psicell-particles", type=int, default=200_000_000)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain section")
    ap.add_argument("--train-snapshots", type=int, default=500)
    ap.add_argument("--train-trajectories", type=int, default=200_000)
    ap.add_argument("--train-particles", type=int, default=50_000_000)
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build targets a single GPU; the projection of one snapshot runs on one "
              "MI355X and --gpus must be 1 (the multi-GPU sharding is a design note only).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2512_20829_amd as F
    import workloads as W

    dev = torch.device("cuda", 0)
    log("generating the 128^3 / 2M-trajectory ABC workload on the GPU")
    wl = W.abc_lattice_3d(device=dev)
    tr = wl.traj
    x = tr.x.contiguous()
    J = tr.J.contiguous()
    v = tr.v.to(torch.float32).contiguous()
    ug = tr.ug.to(torch.float32).contiguous()
    r = tr.r.to(torch.float32).contiguous()
    st, keep = F.make_trajectories(x, J, v, ug, r, tr.n0, tr.seed_volume)
    M = wl.mesh.cells
    mesh = F.mesh_of(wl.mesh)
    S_mass, S_mom, den = F.alloc_fields(M, 3, torch.float32, dev, den=False)
    ctx = F.Context(0)
    params = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
    counted = F.Params(**{**params.__dict__, "count_pairs": True})
    ctx.project_sources(mesh, st, counted, S_mass, S_mom)
    torch.cuda.synchronize()
    stats = ctx.stats()
    P = stats["pairs"]
    log(f"pairs per call: {P} ({P / tr.count:.1f} per trajectory); skipped {stats['skipped']}")

    for _ in range(args.warmup):
        ctx.project_sources(mesh, st, params, S_mass, S_mom)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        ctx.project_sources(mesh, st, params, S_mass, S_mom)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    g_ms = prof["gather"][0] / max(prof["gather"][1], 1)
    stages = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items() if v[1]}
    log(f"{ms_step:.3f} ms/step; stages (ms/launch): {stages}")

    achieved = P * FLOPS_PER_PAIR_3D / (g_ms * 1e-3) / 1e12
    traffic = gather_traffic()
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_gather<float,3,NW>", "launch_ms": round(g_ms, 4),
                "flops_per_pair": FLOPS_PER_PAIR_3D, "pairs_per_launch": P}

    batch = None
    if not args.no_batch:
        batch = batch_section(ctx, args, dev)

    psi = None
    if not args.no_psicell:
        Np = args.psicell_particles
        log(f"generating the {Np}-particle PSI-CELL cloud on the GPU")
        cl = W.abc_cloud(Np, seed=0, device=dev, jacobian=False)
        cv, cu, cr = (cl.v.to(torch.float32).contiguous(), cl.ug.to(torch.float32).contiguous(),
                      cl.r.to(torch.float32).contiguous())
        pst, pkeep = F.make_trajectories(cl.x.contiguous(), None, cv, cu, cr, 1.0)
        del cl
        Pm, Pv, _ = F.alloc_fields(M, 3, torch.float32, dev, den=False)
        w = W.N0_DEFAULT / Np
        ctx.psicell_accumulate(mesh, pst, w, params, Pm, Pv)
        torch.cuda.synchronize()
        reps = 3
        ctx.profile_enable(True)
        e0.record()
        for _ in range(reps):
            ctx.psicell_accumulate(mesh, pst, w, params, Pm, Pv)
        e1.record()
        torch.cuda.synchronize()
        psi_ms = e0.elapsed_time(e1) / reps
        pp = ctx.profile_read()["psicell"]
        ctx.profile_enable(False)
        psi = {"particles": Np, "ms": round(psi_ms, 3),
               "particles_per_s": Np / (psi_ms * 1e-3),
               # inputs: x in binary64 (24 B), v, u_g, r in binary32 (28 B)
               "hbm_gbs_input": round(Np * 52 / (psi_ms * 1e-3) / 1e9, 1),
               # the four passes move 140 B per particle: count 24 in + 4 out,
               # scatter 32 in + 20 out, tiles 20 in + 20 out, reduce 20 in
               "hbm_gbs_algorithmic": round(Np * 140 / (psi_ms * 1e-3) / 1e9, 1),
               "frac_of_hbm_peak": round(Np * 140 / (psi_ms * 1e-3) / 8.0e12, 3),
               "psicell_over_fla_time": round(psi_ms / ms_step, 3),
               "paper_context": "paper: FLA 32 CPU-h vs PSI-CELL 4030 CPU-h for the whole coupled "
                                "solver at 100x seeding, University of Brighton CPU cluster"}
        del pst, pkeep, Pm, Pv
        torch.cuda.empty_cache()
        log(f"psicell {Np}: {psi_ms:.3f} ms")

    learned, model = None, None
    if not args.no_learned:
        log("learned-vs-plain section: training the bandwidth network")
        model, learned = learned_vs_plain(ctx, args, dev)
        log(f"learned: {learned['eval']}")

    large = None
    if not args.no_large:
        log("large section: 256^3 multi-vortex case")
        large = large_section(ctx, args, dev, model)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the FP64 oracle on host cores (~{args.cpu_seconds:.0f} s)")
        cpu = cpu_baseline(args.cpu_seconds)
        log(f"oracle: {cpu['value']:.1f} cells/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": M / (ms_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3-D ABC map (amplitude 0.2, folds), 128^3 periodic mesh, 2,097,152 "
                               "lattice trajectories, FP32 kernel with FP64 det J, h0 = 1/128, cutoff 4",
                   "mesh": [128, 128, 128], "trajectories": tr.count, "mode": "NW"},
        "pairs_per_s": P / (ms_step * 1e-3),
        "pairs": P,
        "stage_ms": stages,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batch": batch,
        "psicell": psi,
        "learned_vs_plain": learned,
        "large": large,
    }
    print(json.dumps(out), flush=True)
    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibration_copy_mib} MiB done")
    ctx.close()


if __name__ == "__main__":
    main()
