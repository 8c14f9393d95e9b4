"""Training and evaluation workflow of the learned Newton guess.

Everything numerical runs in the library's kernels (single-substep solves
of the plain FP64 integrator, feature/target extraction, BF16-MFMA training
and inference); this module only sequences the calls and moves tensors.

Training pairs: (y_n, h) -> Phi_h(y_n), one backward-Euler substep of the
plain solver, for y_n drawn from the combustion-network cell distribution
and from states part-way along their trajectories, with h log-uniform in
[1e-10, 1e-4] s.  Cells whose substep fails (status 2) are dropped.
"""
from __future__ import annotations

import numpy as np

import synthetic as sy

from . import (KR_FIXED_STEP, GuessModel, Network, chem_integrate, default_options,
               guess_options)

H_RANGE = (1e-10, 1e-4)


def single_step_pairs(knet: Network, model: GuessModel, desc, n: int, salt: int,
                      traj_fraction: float = 0.5, stream=None):
    """(X, Y, kept) for n sampled cells: raw features and targets of one
    plain BE substep each (device tensors, failed cells removed)."""
    import torch
    dev = torch.device("cuda")
    cs = sy.cells_h_o_n(desc, n, 1, salt=salt)
    states = torch.tensor(cs.n, device=dev)
    T = torch.tensor(cs.T, device=dev)
    # part of the cells first move along their own trajectories
    n_traj = int(n * traj_fraction)
    if n_traj:
        adv = torch.tensor(sy.log_uniform(n_traj, 1e-10, 1e-6, 1, salt + 100), device=dev)
        sub_n = states[:, :n_traj]
        chem_integrate(knet, sub_n, T[:n_traj], dt=adv, rtol=1e-6, stream=stream)
    h = torch.tensor(sy.log_uniform(n, *H_RANGE, 1, salt + 200), device=dev)
    before = states.clone()
    Tb = T.clone()
    status = torch.empty(n, dtype=torch.int32, device=dev)
    chem_integrate(knet, states, T, dt=h, rtol=1e-6,
                   opts=default_options(mode=KR_FIXED_STEP, n_fixed=1), status=status, stream=stream)
    X = model.features(before, Tb, dt=h, stream=stream)
    Y = model.targets(before, Tb, states, T, stream=stream)
    keep = status == 0
    return X[keep].contiguous(), Y[keep].contiguous(), keep


def train(model: GuessModel, X, Y, steps: int, batch: int = 4096, lr: float = 1e-3,
          lr_min: float = 1e-5, seed: int = 1, chunk: int = 500, log=None):
    """Adam with cosine decay over `steps` (run in chunks so that progress
    can be reported); returns the list of (step, loss)."""
    model.fit_normalization(X, Y)
    hist = []
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        # one cosine schedule over the whole run, split into chunks
        a = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * done / max(steps - 1, 1)))
        b = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * (done + k - 1) / max(steps - 1, 1)))
        loss = model.train(X, Y, k, batch=batch, lr=float(a), lr_min=float(b), seed=seed + done)
        done += k
        hist.append((done, loss))
        if log:
            log(f"guess training step {done}/{steps}: loss {loss:.4e}")
    return hist


def newton_counts(knet: Network, model: GuessModel | None, desc, n: int, salt: int,
                  h=None, stream=None, precision: int = 0):
    """Single-substep solves of n held-out cells with and without the guess
    (precision: KR_FP64 or KR_FP32LU_REFINE): returns dict(status,
    cell_stats, counters, states, T) for the run."""
    import torch
    dev = torch.device("cuda")
    cs = sy.cells_h_o_n(desc, n, 1, salt=salt)
    states = torch.tensor(cs.n, device=dev)
    T = torch.tensor(cs.T, device=dev)
    if h is None:
        h = torch.tensor(sy.log_uniform(n, *H_RANGE, 1, salt + 200), device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    stats = torch.zeros((n, 4), dtype=torch.int32, device=dev)
    counters = torch.zeros(8, dtype=torch.int64, device=dev)
    if model is not None:
        guess = model.predict(states, T, dt=h, stream=stream)
        opts = guess_options(guess, counters, mode=KR_FIXED_STEP, n_fixed=1, precision=precision)
    else:
        opts = default_options(mode=KR_FIXED_STEP, n_fixed=1, precision=precision)
        opts.counters = counters.data_ptr()
    chem_integrate(knet, states, T, dt=h, rtol=1e-6, opts=opts, status=status, cell_stats=stats,
                   stream=stream)
    return {"status": status, "cell_stats": stats, "counters": counters, "states": states, "T": T,
            "h": h, "cells": cs}
