"""Training the learned restart proposal on the filter's own posterior samples.

Pairs come from plain-restart runs of the filter (GpuFilter with
collect_pairs=True) on observation paths disjoint from the evaluation paths:
the estimate x_hat at one restart, and the sample mean and variance of the
resampled nodes at the next restart.  Training runs on the
GPU through yy_proposal_train_step (forward, Gaussian NLL, backward and Adam
in libyy's kernels); the trained parameter vector is then given to the
filters that use the proposal (each creates its own network on its context).
"""
from __future__ import annotations

import dataclasses

import torch

from . import yy
from .filter import GpuFilter
from .workloads import Workload, simulate


COLLECT_R_FACTOR = 4.0   # collection runs use a plain box this many times wider than R


def collect_pairs(w: Workload, seeds, prec: str | None = None, device: int = 0,
                  r_factor: float = COLLECT_R_FACTOR):
    """Runs plain-restart filters on the observation paths of `seeds`, with the plain box widened
    to r_factor * R so that the next restart's samples are not cut off by the box they were
    drawn in; returns the stacked training pairs (x_hat, mu, var) as device tensors [N x r]."""
    wc = dataclasses.replace(w, R=w.R * r_factor)
    xs_all, mus, vars_ = [], [], []
    for sd in seeds:
        xs, dys = simulate(wc, seed=sd)
        f = GpuFilter(wc, prec=prec, device=device, collect_pairs=True)
        try:
            f.set_observations(dys)
            f.init()
            for k in range(1, w.K + 1):
                f.step(k)
            torch.cuda.synchronize(f.dev)
            xs_all.append(f.pair_x[:f.npairs].clone())
            mus.append(f.pair_mu[:f.npairs].clone())
            vars_.append(f.pair_var[:f.npairs].clone())
        finally:
            f.close()
    return torch.cat(xs_all), torch.cat(mus), torch.cat(vars_)


def train(w: Workload, X, MU, VAR, hidden: int = 256, steps: int = 1000, lr: float = 1e-3, seed: int = 0,
          device: int = 0, log_every: int = 0):
    """Trains a fresh network (default initialisation keyed by `seed`) on all pairs for `steps`
    full-batch Adam steps.  Returns (parameter vector [P] float32 on the device, losses)."""
    dev = torch.device("cuda", device)
    ctx = yy.yy_create(device, torch.cuda.current_stream(dev))
    p = None
    try:
        p = yy.yy_proposal_create(ctx, w.r, hidden, seed, None)
        B = X.shape[0]
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        losses = []
        for t in range(steps):
            yy.yy_proposal_train_step(p, B, X.contiguous(), MU.contiguous(), VAR.contiguous(), w.R, lr, True,
                                      loss=loss, r=w.r)
            if log_every and (t % log_every == 0 or t == steps - 1):
                losses.append((t, float(loss.item())))
        params = torch.empty(yy.yy_proposal_num_params(p), dtype=torch.float32, device=dev)
        yy.yy_proposal_get_params(p, params)
        torch.cuda.synchronize(dev)
        return params, losses
    finally:
        if p is not None:
            yy.yy_proposal_destroy(p)
        yy.yy_destroy(ctx)
