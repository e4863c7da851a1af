"""Many independent filter runs stepped together on the GPU (libyy's yy_batch_* calls).

Each step launches the pairwise kernel once for all runs (work items in
decreasing-cost order); the step loop can be captured once into a HIP graph
and replayed.  Runs are Workload descriptions with their own observation paths.
"""
from __future__ import annotations

import numpy as np
import torch

from . import yy
from .workloads import Workload


class Batch:
    def __init__(self, workloads: list[Workload], dys_list, prec: str = "bf16x3g", max_split: int = 0,
                 device: int = 0, stream=None):
        if len({tuple(w.scales) for w in workloads}) != 1:
            raise ValueError("all runs of a batch share the kernel scales")
        self.dev = torch.device("cuda", device)
        # a stream of its own (default priority): graph capture needs a created stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.dev)
        torch.cuda.current_stream(self.dev).synchronize()
        self.ctx = yy.yy_create(device, self.stream)
        self.workloads = list(workloads)
        self.models = [yy.Model(w.r, w.m, w.drift, w.A, w.obs, w.H, w.h_shift, w.q, w.rho2, device=self.dev)
                       for w in workloads]
        self.dys = [torch.as_tensor(np.ascontiguousarray(d), dtype=torch.float64, device=self.dev).reshape(-1)
                    for d in dys_list]
        self.scales = yy.Scales(workloads[0].scales)
        runs = [(m, w.n, w.dt, w.box_half, w.R, w.restart_every, w.K, w.seed, d)
                for m, w, d in zip(self.models, workloads, self.dys)]
        self.b = yy.yy_batch_create(self.ctx, runs, self.scales, prec, max_split)

    def close(self):
        if getattr(self, "b", None) is not None:
            yy.yy_batch_destroy(self.b)
            self.b = None
        if getattr(self, "ctx", None) is not None:
            yy.yy_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        yy.yy_batch_step(self.b)

    def reset(self):
        yy.yy_batch_reset(self.b)

    def run_graph(self, k_end: int):
        yy.yy_batch_run_graph(self.b, k_end)

    def tune(self, reps: int = 3, forms: bool = False, dense: bool = False) -> int:
        """Each run's pairwise form -- against the vector-ALU form (forms=True) and, in a BF16X3P
        batch, against the split form on every tile (dense=True) -- then the source splits; returns
        the split bound."""
        return yy.yy_batch_tune(self.b, reps, (1 if forms else 0) | (2 if dense else 0))

    @property
    def k(self) -> int:
        return yy.yy_batch_step_count(self.b)

    def run_form(self, run: int) -> str:
        """Run `run`'s pairwise form: the batch's matrix-core form, "fp32" on the vector ALUs, or in a
        BF16X3P batch "bf16x3g" (no screen, every tile)."""
        return yy.yy_batch_run_form(self.b, run)

    def set_run_form(self, run: int, prec: str):
        yy.yy_batch_set_run_form(self.b, run, prec)

    def screen_count(self, run: int):
        """(flagged tiles, tiles) of run `run`'s last screen (screened forms only)."""
        return yy.yy_batch_screen_count(self.b, run)

    def results(self, run: int):
        w = self.workloads[run]
        mean = torch.empty(w.K * w.r, dtype=torch.float64, device=self.dev)
        lz = torch.empty(w.K, dtype=torch.float64, device=self.dev)
        ess = torch.empty(w.K, dtype=torch.float64, device=self.dev)
        yy.yy_batch_results(self.b, run, mean, lz, ess)
        return mean.reshape(w.K, w.r), lz, ess
