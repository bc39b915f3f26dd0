"""Training pipeline of the learned proposal: generate training pairs with a
scaling-based schedule, train the per-edge network on the GPU, hand the
parameters to an estimator.

Host orchestration only: recording, the forward / backward passes and the
optimiser all run in the HIP library (perm_est_record, perm_est_mlp_*).
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import MLP_NPARAM, PermEstBatch, ProposalNet, preset
from .inputs import SparseMatrix, network_params


def init_params(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Initial parameters (float32, packed layout) from the seeded generator."""
    p = network_params(seed, scale)
    assert p.size == MLP_NPARAM
    return p.astype(np.float32)


def teacher_schedule():
    """The plain scaled method: shared initial filter, K0 = 100 outer SK
    iterations, one local SK repair per step (Eq. (local)), no inner
    filter; its proposal of Eq. (q) at every recorded step is the training
    target."""
    return preset("local_nodm")


MIX_ALPHA = 0.01  # uniform share mixed into the learned proposal


def record_pairs(mats: List[SparseMatrix], n_traj: int = 4, seed: int = 1, stride: int = 1,
                 device: int = 0) -> Dict:
    """Training pairs from the teacher schedule over a batch of matrices.

    A step records at most 64 pairs and the buffer is sized for 12 per step
    on average; a claim that does not fit is dropped, which can only happen
    once fewer than 64 slots are left.  If the recording got that close to
    full it is repeated with four times the room (so that the set of groups,
    and with the trainer's canonical order the trained network, does not
    depend on which claims won); `complete` says whether every group fit."""
    steps = sum(int(M.n) for M in mats) * n_traj
    group_cap = int(min((1 << 31) - 1, steps // stride + 64))
    bt = PermEstBatch(mats, device=device)
    t = time.perf_counter()
    per_step = 12
    while True:
        rec_cap = int(min((1 << 31) - 1, per_step * steps // stride + 64))
        rec = bt.record(n_traj, seed, teacher_schedule(), rec_cap=rec_cap, group_cap=group_cap, stride=stride)
        rec["complete"] = rec["n_records"] + 64 <= rec_cap
        if rec["complete"] or per_step >= 64 or rec_cap == (1 << 31) - 1:
            break
        per_step = min(64, per_step * 4)
    rec["seconds"] = time.perf_counter() - t
    bt.close()
    return rec


def train(rec: Dict, *, epochs: int = 4, batch_groups: int = 1024, lr: float = 2e-3, seed: int = 0,
          init: Optional[np.ndarray] = None, device: int = 0) -> Tuple["object", Dict]:
    """Train the network on a recording; returns (float32 device tensor of
    the parameters, info)."""
    net = ProposalNet(init if init is not None else init_params(seed), device=device)
    l0, _ = net.loss_grad(rec)
    t = time.perf_counter()
    losses = net.train(rec, epochs=epochs, batch_groups=batch_groups, lr=lr, seed=seed)
    secs = time.perf_counter() - t
    params = net.params()
    net.close()
    return params, {"loss_initial": l0, "loss_per_epoch": losses, "train_seconds": secs,
                    "n_records": rec["n_records"], "n_groups": rec["n_groups"]}


def train_proposal(mats: List[SparseMatrix], *, n_traj: int = 4, stride: int = 1, epochs: int = 4,
                   batch_groups: int = 1024, lr: float = 2e-3, seed: int = 1, device: int = 0):
    """Record teacher pairs on `mats` and train; returns (params, info)."""
    rec = record_pairs(mats, n_traj=n_traj, seed=seed, stride=stride, device=device)
    params, info = train(rec, epochs=epochs, batch_groups=batch_groups, lr=lr, seed=seed, device=device)
    info["record_seconds"] = rec["seconds"]
    info["recording_complete"] = rec["complete"]
    return params, info
