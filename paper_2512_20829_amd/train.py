"""Training and evaluation of the learned bandwidth correction on the GPU.

One training step is one library call, fla_mlp_train_step (all arithmetic
in the library's kernels, one stream): features + network -> h factors ->
estimator projection -> relative-L2 loss against the reference field and
dL/dS -> estimator backward (dL/dlog h) -> network backward (dL/dtheta) ->
Adam.  The feature standardisation is fla_bandwidth_standardise.

The reference field of a snapshot is the PSI-CELL accumulation of a dense
particle cloud drawn from the same flow map, computed by the same library.
Snapshots are produced by a caller-supplied function, so that this module
holds no workload definition.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np
import torch

from . import (FLA_F32, FLA_F64, MLP_PARAMS, MLP_TRAINABLE, Context, Params, alloc_fields, make_trajectories,
               mesh_of)

DEV = torch.device("cuda", 0)


@dataclass
class Snapshot:
    """Device-resident inputs of one training or evaluation snapshot."""
    mesh: object              # object with dim, n, lo, hi, periodic
    traj: object              # fla_trajectories struct
    keep: list                # tensors kept alive for traj
    count: int
    params: Params            # physics and kernel parameters (h_factor filled per step)
    ref: List[torch.Tensor]   # reference field planes (PSI-CELL of a dense cloud)
    prec: int = FLA_F32

    @property
    def cells(self) -> int:
        c = 1
        for k in self.mesh.n[: self.mesh.dim]:
            c *= k
        return c


class BandwidthModel:
    """FP32 master parameters, Adam moments and the training step."""

    def __init__(self, ctx: Context, theta: np.ndarray, lr: float = 1e-3):
        self.ctx = ctx
        self.theta = torch.tensor(np.asarray(theta, dtype=np.float32), device=DEV)
        assert self.theta.numel() == MLP_PARAMS
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.step_count = 0
        self.lr = lr

    def state_dict(self) -> dict:
        return {"theta": self.theta.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "step": self.step_count, "lr": self.lr}

    def load_state_dict(self, d: dict):
        self.theta.copy_(torch.tensor(d["theta"], device=DEV))
        self.m.copy_(torch.tensor(d["m"], device=DEV))
        self.v.copy_(torch.tensor(d["v"], device=DEV))
        self.step_count = int(d["step"])
        self.lr = float(d["lr"])

    # -- one snapshot ---------------------------------------------------------------------
    def _buffers(self, snap: Snapshot):
        N, M = snap.count, snap.cells
        dt = torch.float64 if snap.prec == FLA_F64 else torch.float32
        return (torch.empty(N, dtype=torch.float32, device=DEV), torch.empty(5 * N, dtype=torch.float32, device=DEV),
                torch.empty(N, dtype=torch.float32, device=DEV), dt)

    def factors(self, snap: Snapshot):
        hf, z, o, _ = self._buffers(snap)
        self.ctx.bandwidth_forward(mesh_of(snap.mesh), snap.traj, self.theta, hf, z, o)
        return hf, z, o

    def project(self, snap: Snapshot, hf: Optional[torch.Tensor]):
        dt = torch.float64 if snap.prec == FLA_F64 else torch.float32
        p = Params(**{**snap.params.__dict__, "h_factor": hf})
        Sm, Sv, den = alloc_fields(snap.cells, snap.mesh.dim, dt, DEV)
        self.ctx.project_sources(mesh_of(snap.mesh), snap.traj, p, Sm, Sv, den)
        return [Sm, *Sv], den, p

    def loss(self, snap: Snapshot, S, want_grad: bool):
        C = 1 + snap.mesh.dim
        G = [torch.empty_like(S[0]) for _ in range(C)] if want_grad else None
        res = self.ctx.rel_l2_loss(C, snap.cells, snap.prec, S, snap.ref, G)
        return res, G

    def train_step(self, snap: Snapshot) -> torch.Tensor:
        """One step through fla_mlp_train_step; returns the loss terms."""
        res = torch.empty(1 + 2 * (1 + snap.mesh.dim), dtype=torch.float64, device=DEV)
        self.step_count += 1
        p = Params(**{**snap.params.__dict__, "h_factor": None})
        self.ctx.mlp_train_step(mesh_of(snap.mesh), snap.traj, p, snap.ref, self.theta, self.m, self.v,
                                self.step_count, lr=self.lr, loss=res)
        return res

    def train_step_composed(self, snap: Snapshot) -> torch.Tensor:
        """The same step as six separate library calls."""
        hf, z, o = self.factors(snap)
        S, den, p = self.project(snap, hf)
        res, G = self.loss(snap, S, True)
        dlogh = torch.empty(snap.count, dtype=torch.float32, device=DEV)
        self.ctx.project_backward(mesh_of(snap.mesh), snap.traj, p, S[0], S[1:], den, G[0], G[1:], dlogh)
        self.ctx.bandwidth_backward(snap.mesh.dim, self.theta, snap.count, z, o, dlogh, self.grad)
        self.step_count += 1
        self.ctx.adam_step(self.theta, self.m, self.v, self.grad, self.step_count, lr=self.lr)
        return res

    def evaluate(self, snap: Snapshot, learned: bool = True) -> float:
        hf = self.factors(snap)[0] if learned else None
        S, _, _ = self.project(snap, hf)
        res, _ = self.loss(snap, S, False)
        return float(res[0])


def fit_standardisation(ctx: Context, snaps: List[Snapshot], theta: np.ndarray) -> np.ndarray:
    """Set mu, sd of the parameter block to the mean and spread of the raw
    features over the valid trajectories of the given snapshots
    (fla_bandwidth_standardise)."""
    th = torch.tensor(np.asarray(theta, dtype=np.float32), device=DEV)
    ctx.bandwidth_standardise([mesh_of(s.mesh) for s in snaps], [s.traj for s in snaps], th)
    return th.cpu().numpy().astype(np.float64)


def initial_theta(seed: int = 0) -> np.ndarray:
    """Random hidden layers (He scaling), zero biases, zero output layer: the
    initial factor is exactly 1 (the plain rule of eq. smoothing-length)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 5)) * math.sqrt(2.0 / 5)
    W2 = rng.standard_normal((64, 64)) * math.sqrt(2.0 / 64)
    return np.concatenate([W1.reshape(-1), np.zeros(64), W2.reshape(-1), np.zeros(64), np.zeros(64), np.zeros(1),
                           np.zeros(5), np.ones(5)]).astype(np.float32).astype(np.float64)
