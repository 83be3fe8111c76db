#!/usr/bin/env python3
"""Benchmark of the FLA source projection on one MI355X.

Headline workload: the 3-D multi-vortex case -- 256^3 periodic mesh on the
unit cube, 320^3 = 32,768,000 lattice trajectories through the composition of
two ABC maps (folds, |det J| down to ~1e-8), radius lognormal(ln 10 um, 0.3),
h0 = 1/320, cutoff 4 bandwidths, binary32 kernel evaluation with binary64
det J.  Inputs are synthetic, generated on the GPU before timing, and
resident in HBM when the timed region starts.

One step = one fla_project_sources call: prepass (det J, n, h, physics,
keys), key sort and bucket bounds, record permutation, and the gather with
its fused epilogue.  Printed as one JSON line (rank 0):
  value        mesh cells per second of the headline workload (M / step time)
  pairs_per_s  included trajectory-cell pairs per second
  roofline     the gather kernel of the headline workload, timed with HIP
               events on the library's stream: algorithmic flops per launch
               (15 per included pair) / average launch time, against the
               157.3 TFLOP/s binary32 vector peak
  cpu_baseline the FP64 oracle (trajectory-centric form) on a bounded sample
               of the headline workload, with whole-field and one-thread
               times of the 128^3 and 2-D cases beside it
  abc128       the 128^3 ABC case (2,097,152 lattice trajectories) with its
               own roofline
  tg2d_f64     the 2-D Taylor-Green case in binary64 (64^2 mesh, 4096
               trajectories) against the binary64 vector peak, and the same
               calls replayed as a HIP graph (launch-latency bound)
  batch        64 uneven snapshots (32^3..128^3 meshes, 10k..2M trajectories)
               through fla_project_batch: graph replays, direct launches and
               one single call per snapshot, after the batch autotuner
  psicell      PSI-CELL accumulation of a 200M-particle cloud on 128^3
  learned_vs_plain  the learned bandwidth network trained on 500 generated
               64^3 snapshots (200k trajectories, 50M-particle PSI-CELL each),
               then plain, learned and deposition errors on the 128^3 case
               from 2M down to 32k lattice trajectories against the
               200M-particle reference, the interpolated seeding at which the
               learned form matches the plain form's error at 2M, and the
               cells/s of both forms there
  large        errors of the plain, learned and deposition forms on the
               headline workload against a 1.68G-particle PSI-CELL reference,
               and the learned form's throughput
  table1       the four Table 1 cases through the trajectory producer: FLA
               errors against a 100x box-counted reference after 2 s of
               droplet motion in a Taylor-Green vortex, and step times
  general_mesh the estimator at the centroids of three 128^3-cell general
               meshes (uniform centroids, stretched rectilinear with n_hat
               from the cell volumes, scattered) with the 2M ABC
               trajectories, and the index build time
  producer     one carrier step of 2M droplets in the ABC flow (8 RK4
               substeps, binary64) fused with the projection
  (psicell also times the cloud-in-cell comparator on the same cloud)
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
# Algorithmic work of one included (cell, trajectory) pair, from the kernel
# and estimator definitions: in 3-D with C = 4 channels, 3 offsets, 3 squares
# and 2 additions for |d|^2, the scaling by 1/(2h^2), the denominator addition
# and 4 numerator multiply-adds (14), plus the exponential (1) = 15; in 2-D
# with C = 3 channels, 2 + 2 + 1 + 1 + 1 + 3 = 10, plus the exponential = 11.
FLOPS_PER_PAIR = {3: 15, 2: 11}
# MI355X published vector peaks (256 CUs at 2.4 GHz): binary32 157.3 TFLOP/s
# (packed), 78.6 without packed instructions; binary64 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gather_traffic(workload: str):
    """HBM bytes per gather launch on a workload from the committed counter
    summary profiles/gather_<workload>_hbm_traffic.md, or None when the gather
    source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"gather_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for name in ("gather.hpp", "internal.hpp"):     # the kernel and its compile-time constants
        h.update(open(os.path.join(ROOT, "paper_2512_20829_amd", "csrc", name), "rb").read())
    digest = h.hexdigest()[:16]
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].rsplit(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("gather.hpp + internal.hpp sha256[:16]") != digest:
        return None
    try:
        return float(vals["bytes per launch (calibrated)"])
    except (KeyError, ValueError):
        return None


def timed_projection(ctx, F, mesh, st, params, steps, warmup):
    """Counted call (pairs), warm-up, then `steps` timed calls bracketed by
    synchronisations.  Returns (ms per step from events around the loop,
    per-stage ms per launch from the library's HIP events on the same
    stream, the average gather launch in ms, stats of the counted call)."""
    import torch
    counted = F.Params(**{**params.__dict__, "count_pairs": True})
    M = int(mesh.n[0]) * int(mesh.n[1]) * (int(mesh.n[2]) if mesh.dim == 3 else 1)
    dt = torch.float64 if st.prec == F.FLA_F64 else torch.float32
    S_mass, S_mom, _ = F.alloc_fields(M, mesh.dim, dt, torch.device("cuda", 0), den=False)
    ctx.project_sources(mesh, st, counted, S_mass, S_mom)
    torch.cuda.synchronize()
    stats = ctx.stats()
    for _ in range(warmup):
        ctx.project_sources(mesh, st, params, S_mass, S_mom)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        ctx.project_sources(mesh, st, params, S_mass, S_mom)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    g_ms = prof["gather"][0] / max(prof["gather"][1], 1)
    stages = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items() if v[1]}
    return ms_step, stages, g_ms, stats


def gather_roofline(pairs, g_ms, dim, prec, workload):
    """Roofline object of the gather: ALU-bound; 15 (3-D) or 11 (2-D) flops
    per included pair over the average launch time, against the vector peak
    of the call's precision."""
    fpp = FLOPS_PER_PAIR[dim]
    achieved = pairs * fpp / (g_ms * 1e-3) / 1e12
    peak = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    r = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
         "frac": round(achieved / peak, 4), "traffic": gather_traffic(workload),
         "kernel": f"k_gather<{'double' if prec == 'f64' else 'float'},{dim},NW>", "launch_ms": round(g_ms, 4),
         "flops_per_pair": fpp, "pairs_per_launch": pairs}
    if prec == "f32":
        r["frac_of_nonpacked_78.6"] = round(achieved / FP32_NONPACKED_TFLOPS, 4)
    return r


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


def learned_crossing(rows, target):
    """Seeding at which the learned form's error equals `target`: linear in
    log N between the two sweep points (rows in descending N) that bracket
    it.  Returns (N or None, note)."""
    for a, b in zip(rows, rows[1:]):
        if "learned" in a and "learned" in b and a["learned"] <= target < b["learned"]:
            la, lb = math.log(a["trajectories"]), math.log(b["trajectories"])
            t = (target - b["learned"]) / (a["learned"] - b["learned"])
            return int(round(math.exp(lb + t * (la - lb)))), None
    if rows and "learned" in rows[-1] and rows[-1]["learned"] <= target:
        return None, (f"the learned error is within the target down to the smallest seeding tried, "
                      f"{rows[-1]['trajectories']} (an upper bound on the crossing)")
    return None, "the learned form does not reach the target within the sweep"


def large_section(ctx, args, dev, model):
    """The 256^3 multi-vortex case with strong caustics: the plain, learned
    (the network trained on the 64^3 ABC snapshots, if available) and
    deposition errors against a chunked PSI-CELL reference at 320^3 down to
    16^3 lattice trajectories, the seeding at which the learned
    form matches the plain form's error at 320^3, and the learned form's
    throughput at 320^3 (the plain form's is the headline line)."""
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
    for pa in (320, 256, 200, 160, 128, 100, 80, 64, 50, 40, 32, 25, 20, 16):
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
        if pa == 320 and model is not None:
            # the plain form is the headline line; the learned form includes
            # the feature and network kernels
            reps = 3
            ctx.project_sources(F.mesh_of(wl.mesh), st, prm, Sm, Sv)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                h = model.factors(snap)[0]
                ctx.project_sources(F.mesh_of(wl.mesh), st, F.Params(**{**prm.__dict__, "h_factor": h}), Sm, Sv)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            perf = {"ms_learned": round(ms, 3), "cells_per_s_learned": M / (ms * 1e-3)}
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
    crossing, note = learned_crossing(rows, target)
    return {"workload": "3-D multi-vortex map (two ABC maps, amplitudes 0.2 and 0.1, wavenumbers 1 and 2), "
                        "256^3 periodic mesh, 320^3 lattice trajectories, h0 = 1/320, FP32 kernel with FP64 det J",
            "learned_performance": perf,
            "reference": {"psicell_particles": args.large_particles,
                          "noise_floor_rel_l2": [round(math.sqrt(f), 4) for f in floor]},
            "error": "mean over the 4 source fields of the noise-debiased rel L2 against dense PSI-CELL",
            "eval": rows, "plain_error_at_32.8M": target,
            "learned_matches_plain_at_32.8M_with_trajectories": crossing, "crossing_note": note}


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

    def time_forms(sn, mesh):
        """cells/s of the plain and learned forms (the learned form includes
        the feature and network kernels) on one snapshot."""
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        Sm, Sv, den = F.alloc_fields(sn.cells, 3, torch.float32, dev, den=False)
        out = {}
        for learned in (False, True):
            for rep in range(args.warmup + args.steps):
                if rep == args.warmup:
                    e0.record()
                h = model.factors(sn)[0] if learned else None
                ctx.project_sources(F.mesh_of(mesh), sn.traj, F.Params(**{**sn.params.__dict__, "h_factor": h}),
                                    Sm, Sv)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            out["cells_per_s_learned" if learned else "cells_per_s_plain"] = sn.cells / (ms * 1e-3)
        return out

    rows = []
    for pa in (128, 100, 80, 64, 50, 40, 32):
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
        out.update({k: float(f"{v:.4g}") for k, v in time_forms(sn, wl.mesh).items()})
        rows.append(out)
        del sn, wl
    target = rows[0]["plain"]
    crossing, note = learned_crossing(rows, target)
    at_crossing = None
    if crossing is not None:
        pa = max(2, int(round(crossing ** (1.0 / 3.0))))
        wl = W.abc_lattice_3d(per_axis=pa, mesh_n=128, device=dev)
        sn = snap_of(wl, ref2)
        hf = model.factors(sn)[0]
        prm = F.Params(**{**sn.params.__dict__, "h_factor": hf})
        Sm, Sv, den = F.alloc_fields(sn.cells, 3, torch.float32, dev)
        ctx.project_sources(F.mesh_of(wl.mesh), sn.traj, prm, Sm, Sv, den)
        res, _ = model.loss(sn, [Sm, *Sv], False)
        at_crossing = {"lattice_trajectories": pa ** 3, "learned": round(deb(res), 5), **time_forms(sn, wl.mesh)}
        del sn, wl
    return model, {
        "train": {"snapshots": args.train_snapshots, "trajectories": args.train_trajectories, "mesh": [64, 64, 64],
                  "psicell_particles": args.train_particles, "steps": args.train_steps, "seconds": round(t_train, 2)},
        "reference": {"psicell_particles": args.psicell_particles, "noise_floor_rel_l2": [round(math.sqrt(f), 4) for f in floor]},
        "error": "mean over the 4 source fields of the noise-debiased rel L2 against dense PSI-CELL",
        "eval": rows,
        "plain_error_at_2M": target,
        "learned_matches_plain_at_2M_with_trajectories": crossing,
        "crossing_note": note,
        "at_crossing": at_crossing,
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
    achieved = P * FLOPS_PER_PAIR[3] / (g_ms * 1e-3) / 1e12
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
           "gather": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "launch_ms": g_ms,
                      "frac_of_nonpacked_78.6": round(achieved / FP32_NONPACKED_TFLOPS, 4),
                      "kernel": "k_gather_batch<float,3,NW>"}}
    del wls, trajs, keeps, outs
    torch.cuda.empty_cache()
    return out


def table1_section(ctx, args, dev):
    """The four Table 1 cases as a second workload.  Monodisperse droplets of
    each case start at rest on the periodic unit square in the steady
    Taylor-Green vortex of amplitude 1 m/s (U/L = 1 s^-1, so the relaxation
    time equals the case's St) and are advanced by fla_advance_project over
    2 s in 100 carrier steps (8 RK4 substeps each); evaporating cases lose
    half of r^2 over the run (delta = -r0^2/(4 s)).  FLA: a 64^2 lattice of
    droplets, projected every step on the 64^2 mesh.  Reference: 100 times as
    many droplets at random positions, advanced by the same producer, each
    step's rates box-counted (FLA_DEPOSIT with a vanishing bandwidth puts a
    droplet's whole n0 V_seed phibar into its cell, which is PSI-CELL with
    statistical weight n0 V_seed), as two independent half clouds for the
    noise floor.  Reported per case: the noise-debiased errors of the FLA
    estimator and deposition forms against the reference after 2 s, and the
    time per carrier step of the FLA and reference runs."""
    import numpy as np
    import torch

    import paper_2512_20829_amd as F
    import workloads as W

    mesh_w = W.unit_mesh(2, 64, True)
    mesh = F.mesh_of(mesh_w)
    M = mesh_w.cells
    flow = F.make_flow(F.FLA_FLOW_TAYLOR_GREEN, U=1.0, k=1.0)
    T, nsteps, sub = 2.0, 100, 8
    dt = T / nsteps
    n_fla = 64
    n_cloud = 100 * n_fla * n_fla
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = []
    for j, case in enumerate(W.TABLE1):
        mu = W.TABLE1_RHO_F * case["nu"]
        delta = -case["r_d"] ** 2 / (4.0 * T) if case["evaporating"] else 0.0
        prm = dict(rho_d=case["rho_d"], mu=mu, delta=delta, cutoff=4.0)

        def run(d, h0, mode, field_planes, last_extra=None):
            """Advance d for nsteps, projecting every step; returns ms per step."""
            t = [d.x.to(dev).contiguous(), d.v.to(dev).contiguous(), d.J.to(dev).contiguous(),
                 d.dJ.to(dev).contiguous(), d.r.to(dev).contiguous()]
            st, keep = F.make_droplets(*t, n0=d.n0, seed_volume=d.seed_volume)
            p = F.Params(h0=h0, mode=mode, **prm)
            step = F.make_step(dt, sub, True)
            torch.cuda.synchronize()
            e0.record()
            for it in range(nsteps):
                if it == nsteps - 1 and last_extra is not None:
                    # the same final step, in the other mode, without updating the state
                    ctx.advance_project(mesh, st, flow, F.make_step(dt, sub, False),
                                        F.Params(h0=h0, mode=last_extra[0], **prm), F.FLA_F64,
                                        last_extra[1][0], last_extra[1][1:])
                ctx.advance_project(mesh, st, flow, step, p, F.FLA_F64, field_planes[0], field_planes[1:])
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / nsteps

        planes = lambda: [torch.zeros(M, dtype=torch.float64, device=dev) for _ in range(3)]
        fla_nw, fla_dep = planes(), planes()
        ms_fla = run(W.table1_droplets(j, n_fla, device=dev), 1.0 / n_fla, F.FLA_NW, fla_nw,
                     (F.FLA_DEPOSIT, fla_dep))
        halves, ms_ref = [], 0.0
        for h in range(2):
            d = W.table1_droplets(j, n_cloud // 2, seed=7 + j, device=dev, lattice_seeding=False,
                                  offset=h * (n_cloud // 2))
            pl = planes()
            ms_ref += run(d, 1e-12, F.FLA_DEPOSIT, pl)
            halves.append(pl)
        ref = [(a + b) * 0.5 for a, b in zip(*halves)]
        chans = range(3) if case["evaporating"] else range(1, 3)
        floor = {k: float(((halves[0][k] - halves[1][k]) ** 2).sum() / (4 * (ref[k] ** 2).sum())) for k in chans}

        def deb(S):
            e = []
            for k in chans:
                e2 = float(((S[k] - ref[k]) ** 2).sum() / (ref[k] ** 2).sum())
                e.append(math.sqrt(max(e2 - floor[k], 0.0)))
            return round(float(np.mean(e)), 5)

        row = {"case": case["case"], "St": case["St"], "delta": delta, "rho_d": case["rho_d"], "r_d": case["r_d"],
               "fla_error_nw": deb(fla_nw), "fla_error_deposit": deb(fla_dep),
               "noise_floor": round(math.sqrt(float(np.mean(list(floor.values())))), 5),
               "ms_per_step_fla": round(ms_fla, 4), "ms_per_step_reference": round(ms_ref, 4),
               "reference_over_fla_time": round(ms_ref / ms_fla, 2)}
        log(f"table1: {row}")
        out.append(row)
        torch.cuda.empty_cache()
    return {"workload": "Table 1 cases: monodisperse droplets from rest in the steady Taylor-Green vortex (1 m/s, "
                        "periodic unit square, 64^2 mesh), 2 s in 100 carrier steps of 8 RK4 substeps; FLA 4096 "
                        "lattice droplets vs a 409,600-droplet box-counted reference",
            "error": "mean over the source fields (momentum only without evaporation) of the noise-debiased rel "
                     "L2 against the reference after 2 s",
            "cases": out}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(args, dev):
    """The FP64 oracle in its trajectory-centric form (each trajectory visits
    the cells of its cutoff box; OpenMP threads own planes of cells) on the
    host cores.  Headline: a slab of whole y-planes of the 256^3 multi-vortex
    case, all trajectories, sized to about args.cpu_seconds; the rate is the
    sample's cells over its time plus the trajectory terms of all 32.8M
    trajectories, as cells/s over the whole field.  Beside it, with no
    extrapolation: the whole 128^3 field on all threads and the whole 2-D
    Taylor-Green field; and one-thread rates (a y-slab of the 128^3 case,
    the whole 2-D field)."""
    import torch

    import oracle
    import workloads as W
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    threads = oracle.num_threads()
    f = lambda t: t.to(torch.float32).to(torch.float64)

    def host(tr, prec):
        g = f if prec == "f32" else (lambda t: t)
        return W.Trajectories(tr.x.cpu(), tr.J.cpu(), g(tr.v.cpu()), g(tr.ug.cpu()), g(tr.r.cpu()), tr.n0,
                              tr.seed_volume)

    def run(wl, tr, terms, box_lo=None, box_n=None):
        t0 = time.perf_counter()
        p = oracle.nw_box(wl.mesh, tr.x, terms, box_lo, box_n, wl.cutoff, wl.precision == "f32")
        return time.perf_counter() - t0, p

    # headline: 256^3 multi-vortex, y-slab sample
    wl = W.multi_vortex_lattice_3d(device=dev)
    tr = host(wl.traj, "f32")
    wl.traj = None
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    terms = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
    t_terms = time.perf_counter() - t0
    n = wl.mesh.n
    t1, _ = run(wl, tr, terms, [0, 0, 0], [n[0], 1, n[2]])
    k = int(max(1, min(n[1] - 1, args.cpu_seconds / max(t1, 1e-3))))
    t_box, p = run(wl, tr, terms, [0, 1, 0], [n[0], k, n[2]])
    B = n[0] * k * n[2]
    M = wl.mesh.cells
    full = t_terms + t_box * M / B
    pairs_sample = int(p.pairs.sum())
    del tr, terms, p, wl
    out = {
        "value": M / full,
        "unit": "cells/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{k} whole y-planes ({B} cells, {pairs_sample} included pairs) of the 256^3 multi-vortex "
                   f"field, by the FP64 oracle's trajectory-centric form over all 32,768,000 trajectories on "
                   f"{threads} threads: {t_box:.1f} s, plus {t_terms:.1f} s for the terms of every trajectory; "
                   f"value = M / (t_terms + t_sample * M / cells)"),
        "cpu_model": _cpu_model(),
        "affinity_cores": cores,
    }
    # 128^3 ABC: whole field on all threads (no extrapolation), and one thread on a y-slab
    wl = W.abc_lattice_3d(device="cpu")
    tr = host(wl.traj, "f32")
    terms = oracle.trajectory_terms(tr, wl.rho_d, wl.mu, wl.delta, wl.h0)
    t_all, p = run(wl, tr, terms)
    out["abc128_whole_field"] = {"seconds": round(t_all, 2), "cells_per_s": wl.mesh.cells / t_all,
                                 "pairs": int(p.pairs.sum()), "threads": threads}
    oracle.set_threads(1)
    t1, p1 = run(wl, tr, terms, [0, 0, 0], [128, 2, 128])
    out["abc128_one_thread"] = {"seconds": round(t1, 2), "cells": 128 * 2 * 128,
                                "cells_per_s": 128 * 2 * 128 / t1, "pairs": int(p1.pairs.sum()),
                                "sample": "2 whole y-planes of the 128^3 field"}
    # 2-D Taylor-Green in binary64: whole field, one thread and all threads
    wl2 = W.taylor_green_2d()
    tr2 = host(wl2.traj, "f64")
    terms2 = oracle.trajectory_terms(tr2, wl2.rho_d, wl2.mu, wl2.delta, wl2.h0)
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        run(wl2, tr2, terms2)
    t_one = (time.perf_counter() - t0) / reps
    oracle.set_threads(cores)
    t0 = time.perf_counter()
    for _ in range(reps):
        run(wl2, tr2, terms2)
    t_many = (time.perf_counter() - t0) / reps
    out["tg2d_f64_whole_field"] = {"one_thread_s": round(t_one, 5), "cells_per_s_one_thread": wl2.mesh.cells / t_one,
                                   "all_threads_s": round(t_many, 5),
                                   "cells_per_s_all_threads": wl2.mesh.cells / t_many}
    return out


def projection_section(ctx, args, dev, wl, prec, traffic_name, graph=False):
    """Timed fla_project_sources on one workload (inputs on the GPU), its
    rates and the gather's roofline.  With graph, also the time per call of
    the same calls replayed as a HIP graph (fla_set_graph; profiling off),
    beside the direct calls without profiling."""
    import torch

    import paper_2512_20829_amd as F
    tr = wl.traj
    dt = torch.float64 if prec == "f64" else torch.float32
    st, keep = F.make_trajectories(tr.x.contiguous(), tr.J.contiguous(), tr.v.to(dt).contiguous(),
                                   tr.ug.to(dt).contiguous(), tr.r.to(dt).contiguous(), tr.n0, tr.seed_volume)
    wl.traj = None
    del tr
    mesh = F.mesh_of(wl.mesh)
    params = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
    ms, stages, g_ms, stats = timed_projection(ctx, F, mesh, st, params, args.steps, args.warmup)
    M = wl.mesh.cells
    P = stats["pairs"]
    extra = {}
    if graph:
        dt = torch.float64 if prec == "f64" else torch.float32
        Sm, Sv, _ = F.alloc_fields(M, wl.mesh.dim, dt, dev, den=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def loop():
            for _ in range(3):
                ctx.project_sources(mesh, st, params, Sm, Sv)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                ctx.project_sources(mesh, st, params, Sm, Sv)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / args.steps

        ms_direct = loop()
        ctx.set_graph(True)
        r0 = ctx.stats()["graph_replays"]
        ms_graph = loop()
        replays = ctx.stats()["graph_replays"] - r0
        ctx.set_graph(False)
        extra = {"ms_per_step_direct_unprofiled": round(ms_direct, 4), "ms_per_step_graph": round(ms_graph, 4),
                 "cells_per_s_graph": M / (ms_graph * 1e-3), "graph_replays": replays}
    del st, keep
    torch.cuda.empty_cache()
    return {"ms_per_step": round(ms, 4), "cells_per_s": M / (ms * 1e-3), "pairs_per_s": P / (ms * 1e-3),
            "pairs": P, "trajectories": stats["trajectories"], "skipped": stats["skipped"],
            "max_class": stats["max_class"], "stage_ms": stages,
            "roofline": gather_roofline(P, g_ms, wl.mesh.dim, prec, traffic_name), **extra}


def general_mesh_section(ctx, args, dev, cartesian_ms):
    """fla_project_cells on the 2M-trajectory ABC workload over three
    general meshes of 128^3 cells: the uniform mesh's centroids (same pairs
    as the Cartesian path), a rectilinear mesh stretched toward every wall
    and a scattered (jittered, shuffled) mesh; n_hat from the cell volumes
    on the stretched mesh.  Times the index build once and the projection
    per call (inputs resident on the GPU)."""
    import time

    import torch

    import paper_2512_20829_amd as F
    import workloads as W
    wl = W.abc_lattice_3d(device=dev)
    tr = wl.traj
    st, keep = F.make_trajectories(tr.x.contiguous(), tr.J.contiguous(), tr.v.float().contiguous(),
                                   tr.ug.float().contiguous(), tr.r.float().contiguous(), tr.n0, tr.seed_volume)
    params = F.Params(rho_d=wl.rho_d, mu=wl.mu, delta=wl.delta, h0=wl.h0, cutoff=wl.cutoff)
    counted = F.Params(**{**params.__dict__, "count_pairs": True})
    inj = F.make_injection(2.0e5, 1.0e-3, 2.5e-3, 4.0)
    meshes = [("uniform_centroids", W.mesh_cells(wl.mesh), None),
              ("stretched_rectilinear", W.rectilinear_cells([W.stretched_edges(128, 0.0, 1.0, 1.5)] * 3,
                                                            (True,) * 3), inj),
              ("scattered", W.scattered_cells(3, 128, (0.0,) * 3, (1.0,) * 3, (True,) * 3, seed=3), None)]
    rows = {}
    for name, cells, j in meshes:
        cs, ck = F.cells_of(cells, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ix = ctx.cell_index(cs)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        M = cells.count
        Sm, Sv, _ = F.alloc_fields(M, 3, torch.float32, dev, den=False)
        ctx.project_cells(ix, st, counted, Sm, Sv, injection=j)
        torch.cuda.synchronize()
        stats = ctx.stats()
        for _ in range(args.warmup):
            ctx.project_cells(ix, st, params, Sm, Sv, injection=j)
        ctx.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            ctx.project_cells(ix, st, params, Sm, Sv, injection=j)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        g_ms = prof["gather"][0] / max(prof["gather"][1], 1)
        P = stats["pairs"]
        fpp = FLOPS_PER_PAIR[3]
        ach = P * fpp / (g_ms * 1e-3) / 1e12
        nb, nwork = ix.shape()
        rows[name] = {"cells": M, "buckets": list(nb), "work_items": nwork, "index_build_ms": round(build_ms, 2),
                      "ms_per_step": round(ms, 3), "cells_per_s": M / (ms * 1e-3), "pairs": P,
                      "pairs_per_s": P / (ms * 1e-3), "n_hat": j is not None,
                      "stage_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items() if v[1]},
                      "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4), "traffic": None,
                                   "kernel": "k_cells_gather<float,3>", "launch_ms": round(g_ms, 4),
                                   "flops_per_pair": fpp,
                                   "frac_of_nonpacked_78.6": round(ach / FP32_NONPACKED_TFLOPS, 4)},
                      "over_cartesian_time": round(ms / cartesian_ms, 2) if cartesian_ms else None}
        log(f"general mesh {name}: {ms:.3f} ms/step, {P:.4g} pairs, index {build_ms:.1f} ms")
        ix.close()
        del Sm, Sv
    # the stretched mesh again as a rectilinear Cartesian mesh (per-axis edges
    # in fla_mesh): the separable gather of fla_project_sources
    edges = [W.stretched_edges(128, 0.0, 1.0, 1.5).to(dev) for _ in range(3)]
    mesh = F.mesh_of(W.unit_mesh(3, 128, True), edges=edges)
    ms, stages, g_ms, stats = timed_projection(ctx, F, mesh, st, params, args.steps, args.warmup)
    P = stats["pairs"]
    ach = P * FLOPS_PER_PAIR[3] / (g_ms * 1e-3) / 1e12
    rows["stretched_rectilinear_cartesian"] = {
        "cells": 128 ** 3, "ms_per_step": round(ms, 3), "cells_per_s": 128 ** 3 / (ms * 1e-3), "pairs": P,
        "pairs_per_s": P / (ms * 1e-3), "stage_ms": stages, "entry": "fla_project_sources with fla_mesh.edges",
        "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / FP32_PEAK_TFLOPS, 4), "traffic": None, "kernel": "k_gather<float,3,NW>",
                     "launch_ms": round(g_ms, 4), "flops_per_pair": FLOPS_PER_PAIR[3],
                     "frac_of_nonpacked_78.6": round(ach / FP32_NONPACKED_TFLOPS, 4)},
        "over_cartesian_time": round(ms / cartesian_ms, 2) if cartesian_ms else None}
    log(f"general mesh stretched, rectilinear path: {ms:.3f} ms/step, {P:.4g} pairs")
    del st, keep
    torch.cuda.empty_cache()
    return rows


def producer_section(ctx, args, dev):
    """fla_advance_project on 2,097,152 droplets (128^3 lattice, lognormal
    radii, random initial velocities) in the ABC flow on the 128^3 periodic
    mesh: one carrier step of 2 ms in 8 RK4 substeps (binary64) fused with
    the record emission, then the projection (binary32 kernel).  The state
    is not written back, so every call advances the same droplets."""
    import torch

    import paper_2512_20829_amd as F
    import workloads as W
    d = W.seed_droplets(3, 128, seed=0, device=dev)
    mesh_w = W.unit_mesh(3, 128, True)
    mesh = F.mesh_of(mesh_w)
    N = d.x.shape[1]
    phibar = torch.empty((4, N), dtype=torch.float64, device=dev)
    dr, keep = F.make_droplets(d.x, d.v, d.J, d.dJ, d.r, d.n0, d.seed_volume, phibar=phibar)
    flow = F.make_flow(F.FLA_FLOW_ABC, U=0.2, k=1.0)
    step = F.make_step(2e-3, 8, update_state=False)
    p = F.Params(rho_d=W.RHO_D, mu=W.MU_AIR, delta=W.DELTA_EVAP, h0=1.0 / 128)
    Sm, Sv, _ = F.alloc_fields(mesh_w.cells, 3, torch.float32, dev, den=False)
    for _ in range(max(args.warmup, 1)):
        ctx.advance_project(mesh, dr, flow, step, p, F.FLA_F32, Sm, Sv)
    ctx.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        ctx.advance_project(mesh, dr, flow, step, p, F.FLA_F32, Sm, Sv)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    stages = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items() if v[1]}
    prod_ms = stages.get("prepass")
    return {"droplets": N, "substeps": 8, "ms_per_step": round(ms, 4), "stage_ms": stages,
            "producer_ms": prod_ms,
            "droplet_substeps_per_s": N * 8 / (prod_ms * 1e-3) if prod_ms else None,
            "note": "producer_ms is the fused kernel (RK4 of the droplet state, Jacobian and sources, then the "
                    "records); the rest of the step is the projection of the advanced droplets"}


def learned_kernels_section(ctx, args, dev):
    """Times of the learned-bandwidth calls alone: the forward (features and
    network) and the network backward on the 2M-trajectory 128^3 ABC case,
    and the library's whole training step on 64^3 training snapshots."""
    import numpy as np
    import torch

    import paper_2512_20829_amd as F
    import workloads as W
    from paper_2512_20829_amd import train as T
    wl = W.abc_lattice_3d(device=dev)
    tr = wl.traj
    st, keep = F.make_trajectories(tr.x.contiguous(), tr.J.contiguous(), tr.v.float().contiguous(),
                                   tr.ug.float().contiguous(), tr.r.float().contiguous(), tr.n0, tr.seed_volume)
    N = tr.count
    th = T.initial_theta(0)
    th[64 * 5 + 64 + 64 * 64 + 64:64 * 5 + 64 + 64 * 64 + 128] = np.random.default_rng(1).uniform(-0.2, 0.2, 64)
    theta = torch.tensor(th, dtype=torch.float32, device=dev)     # a non-zero output layer
    hf = torch.empty(N, dtype=torch.float32, device=dev)
    z = torch.empty(5 * N, dtype=torch.float32, device=dev)
    o = torch.empty(N, dtype=torch.float32, device=dev)
    mesh = F.mesh_of(wl.mesh)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    fwd = timed(lambda: ctx.bandwidth_forward(mesh, st, theta, hf, z, o), 20)
    dl = torch.randn(N, dtype=torch.float32, device=dev) * 1e-3
    grad = torch.empty(theta.numel(), dtype=torch.float32, device=dev)
    bwd = timed(lambda: ctx.bandwidth_backward(3, theta, N, z, o, dl, grad), 10)
    del st, keep, hf, z, o, dl
    snaps = []
    for s in range(4):
        w2, abc = W.training_snapshot(s, n_traj=args.train_trajectories, mesh_n=64, device=dev)
        p = F.Params(rho_d=w2.rho_d, mu=w2.mu, delta=w2.delta, h0=w2.h0, cutoff=w2.cutoff)
        ref, _ = _psicell_reference(ctx, F, W, torch, w2.mesh, abc, args.train_particles, 10_000 + s, p, dev)
        t2 = w2.traj
        s2, k2 = F.make_trajectories(t2.x, t2.J, t2.v.float(), t2.ug.float(), t2.r.float(), t2.n0, t2.seed_volume)
        k2.append(t2)
        snaps.append(T.Snapshot(w2.mesh, s2, k2, t2.count, p, ref))
    model = T.BandwidthModel(ctx, T.fit_standardisation(ctx, snaps, T.initial_theta(0)), lr=1e-3)
    it = [0]

    def step():
        model.train_step(snaps[it[0] % len(snaps)])
        it[0] += 1

    train = timed(step, 20)
    return {"trajectories": N, "forward_ms": round(fwd, 4), "network_backward_ms": round(bwd, 4),
            "train_step_ms_64cubed_200k": round(train, 4)}


def psicell_section(ctx, args, dev, fla_ms):
    import torch

    import paper_2512_20829_amd as F
    import workloads as W
    Np = args.psicell_particles
    log(f"generating the {Np}-particle PSI-CELL cloud on the GPU")
    mesh_w = W.unit_mesh(3, 128, True)
    M = mesh_w.cells
    mesh = F.mesh_of(mesh_w)
    cl = W.abc_cloud(Np, seed=0, device=dev, jacobian=False)
    cv, cu, cr = (cl.v.to(torch.float32).contiguous(), cl.ug.to(torch.float32).contiguous(),
                  cl.r.to(torch.float32).contiguous())
    pst, pkeep = F.make_trajectories(cl.x.contiguous(), None, cv, cu, cr, 1.0)
    del cl
    Pm, Pv, _ = F.alloc_fields(M, 3, torch.float32, dev, den=False)
    w = W.N0_DEFAULT / Np
    params = F.Params(rho_d=W.RHO_D, mu=W.MU_AIR, delta=W.DELTA_EVAP, h0=1.0 / 128)
    ctx.psicell_accumulate(mesh, pst, w, params, Pm, Pv)
    torch.cuda.synchronize()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.psicell_accumulate(mesh, pst, w, params, Pm, Pv)
    e1.record()
    torch.cuda.synchronize()
    psi_ms = e0.elapsed_time(e1) / reps
    # the cloud-in-cell comparator on the same cloud
    ctx.cic_accumulate(mesh, pst, w, params, Pm, Pv)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.cic_accumulate(mesh, pst, w, params, Pm, Pv)
    e1.record()
    torch.cuda.synchronize()
    cic_ms = e0.elapsed_time(e1) / reps
    del pst, pkeep, Pm, Pv
    torch.cuda.empty_cache()
    # algorithmic bytes: x in binary64 (24 B) and v, u_g, r in binary32
    # (28 B) per particle read once, 4 binary32 fields of 16 B per cell written
    alg = Np * 52 + M * 16
    return {"particles": Np, "ms": round(psi_ms, 3), "particles_per_s": Np / (psi_ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": round(alg / (psi_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg / (psi_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": psicell_traffic(), "algorithmic_bytes": alg,
                         "note": "achieved counts 52 B per particle in and 16 B per cell out; traffic is the "
                                 "counted bytes of the passes (records written and re-read)"},
            "cic": {"ms": round(cic_ms, 3), "particles_per_s": Np / (cic_ms * 1e-3),
                    "frac_of_hbm_by_algorithmic_bytes": round(alg / (cic_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "psicell_over_fla_time": round(psi_ms / fla_ms, 3) if fla_ms else None,
            "paper_context": "paper: FLA 32 CPU-h vs PSI-CELL 4030 CPU-h for the whole coupled "
                             "solver at 100x seeding, University of Brighton CPU cluster"}


def psicell_traffic():
    """Counted HBM bytes of one PSI-CELL call on the 200M-particle cloud from
    the committed counter summary, or None when psicell.hip changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "psicell_200m_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2512_20829_amd", "csrc", "psicell.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].rsplit(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("psicell.hip sha256[:16]") != digest:
        return None
    try:
        return float(vals["bytes per call (calibrated)"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only-headline", action="store_true", help="time the headline workload only")
    ap.add_argument("--only", choices=["headline", "abc128", "tg2d", "psicell", "table1", "cells", "batch", "learned",
                                       "producer"],
                    default=None,
                    help="time one projection workload only (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-psicell", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch section")
    ap.add_argument("--no-large", action="store_true", help="skip the 256^3 error section")
    ap.add_argument("--large-particles", type=int, default=1_677_721_600)
    ap.add_argument("--batch-snapshots", type=int, default=64)
    ap.add_argument("--psicell-particles", type=int, default=200_000_000)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain section")
    ap.add_argument("--no-table1", action="store_true", help="skip the Table 1 sweep")
    ap.add_argument("--no-cells", action="store_true", help="skip the general-mesh section")
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
    if args.only_headline:
        args.only = "headline"

    import torch

    import paper_2512_20829_amd as F
    import workloads as W

    dev = torch.device("cuda", 0)
    ctx = F.Context(0)
    head = abc = tg = None
    if args.only in (None, "headline"):
        log("headline: generating the 256^3 / 32.8M-trajectory multi-vortex workload on the GPU")
        head = projection_section(ctx, args, dev, W.multi_vortex_lattice_3d(device=dev), "f32", "multivortex256")
        log(f"headline: {head['ms_per_step']:.3f} ms/step; stages {head['stage_ms']}")
    if args.only in (None, "abc128"):
        log("abc128: the 128^3 / 2M-trajectory ABC workload")
        abc = projection_section(ctx, args, dev, W.abc_lattice_3d(device=dev), "f32", "abc128")
        log(f"abc128: {abc['ms_per_step']:.3f} ms/step; stages {abc['stage_ms']}")
    if args.only in (None, "tg2d"):
        log("tg2d_f64: the 2-D Taylor-Green workload in binary64")
        a2 = argparse.Namespace(**{**vars(args), "steps": max(args.steps, 200)})
        tg = projection_section(ctx, a2, dev, W.taylor_green_2d(device=dev), "f64", "tg2d", graph=True)
        log(f"tg2d_f64: {tg['ms_per_step']:.4f} ms/step ({tg['ms_per_step_graph']:.4f} as graph replays)")

    batch = psi = learned = large = cpu = None
    if args.only == "psicell":
        psi = psicell_section(ctx, args, dev, None)
        print(json.dumps({"psicell": psi}), flush=True)
        if args.calibration_copy_mib > 0:
            n = args.calibration_copy_mib * (1 << 20) // 4
            a = torch.ones(n, dtype=torch.float32, device=dev)
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
        ctx.close()
        return
    if args.only in ("batch", "learned", "producer"):
        sec = {"batch": batch_section, "learned": learned_kernels_section,
               "producer": producer_section}[args.only](ctx, args, dev)
        print(json.dumps({args.only: sec}), flush=True)
        ctx.close()
        return
    if args.only == "cells":
        print(json.dumps({"general_mesh": general_mesh_section(ctx, args, dev, None)}), flush=True)
        ctx.close()
        return
    if args.only == "table1":
        print(json.dumps({"table1": table1_section(ctx, args, dev)}), flush=True)
        ctx.close()
        return
    table1 = cells = producer = None
    if args.only is None:
        if not args.no_table1:
            table1 = table1_section(ctx, args, dev)
        if not args.no_cells:
            cells = general_mesh_section(ctx, args, dev, abc["ms_per_step"])
        producer = producer_section(ctx, args, dev)
        log(f"producer: {producer['ms_per_step']:.3f} ms/step; stages {producer['stage_ms']}")
        if not args.no_batch:
            batch = batch_section(ctx, args, dev)
        if not args.no_psicell:
            psi = psicell_section(ctx, args, dev, abc["ms_per_step"])
            log(f"psicell: {psi['ms']:.3f} ms")
        model = None
        if not args.no_learned:
            log("learned-vs-plain section: training the bandwidth network")
            model, learned = learned_vs_plain(ctx, args, dev)
            log(f"learned: {learned['eval']}")
        if not args.no_large:
            log("large section: errors on the 256^3 multi-vortex case")
            large = large_section(ctx, args, dev, model)
        if not args.no_cpu_baseline:
            log(f"timing the FP64 oracle on host cores (~{args.cpu_seconds:.0f} s sample + whole fields)")
            cpu = cpu_baseline(args, dev)
            log(f"oracle: {cpu['value']:.1f} cells/s on {cpu['cores']} threads")

    main_sec = head or abc or tg
    name = {"headline": "multi-vortex 256^3", "abc128": "ABC 128^3", "tg2d": "Taylor-Green 2-D FP64"}[args.only or "headline"]
    workload_configs = {
        "headline": {"workload": "3-D multi-vortex map (two ABC maps, amplitudes 0.2 and 0.1, wavenumbers 1 and 2; "
                                 "folds, |det J| down to ~1e-8), 256^3 periodic mesh, 32,768,000 lattice "
                                 "trajectories (320^3), FP32 kernel with FP64 det J, h0 = 1/320, cutoff 4",
                     "mesh": [256, 256, 256], "trajectories": 320 ** 3, "mode": "NW"},
        "abc128": {"workload": "3-D ABC map (amplitude 0.2, folds), 128^3 periodic mesh, 2,097,152 lattice "
                               "trajectories, FP32 kernel with FP64 det J, h0 = 1/128, cutoff 4",
                   "mesh": [128, 128, 128], "trajectories": 128 ** 3, "mode": "NW"},
        "tg2d": {"workload": "2-D Taylor-Green map (amplitude 0.1), 64^2 mesh on the unit square, 4096 lattice "
                             "trajectories, FP64, h0 = 1/64, cutoff 4",
                 "mesh": [64, 64], "trajectories": 64 ** 2, "mode": "NW"},
    }
    out = {
        "metric": METRIC,
        "value": main_sec["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_sec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_sec is tg else "f32",
        "data": "synthetic",
        "config": workload_configs[args.only or "headline"],
        "pairs_per_s": main_sec["pairs_per_s"],
        "pairs": main_sec["pairs"],
        "max_class": main_sec["max_class"],
        "stage_ms": main_sec["stage_ms"],
        "roofline": main_sec["roofline"],
        "cpu_baseline": cpu,
        "abc128": abc if main_sec is not abc else None,
        "tg2d_f64": tg if main_sec is not tg else None,
        "batch": batch,
        "psicell": psi,
        "learned_vs_plain": learned,
        "large": large,
        "table1": table1,
        "general_mesh": cells,
        "producer": producer,
    }
    log(f"main line: {name}")
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
