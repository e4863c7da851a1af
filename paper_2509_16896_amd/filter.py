"""The filter's time loop on the GPU, built on the libyy calls (Sec. 2.2.2 procedure, Sec. 6 restart).

Per step k: yy_propagate -> yy_loglik_update -> yy_normalise_moments, and every
``restart_every`` steps yy_restart (resampling, new box around the estimate,
the reference codes mapped into it, the re-centred prior) followed by a
normalisation.  The initial state is the restart map with centre 0 and
half-width ``box_half``: nodes in [-box_half, box_half]^r carrying the N(0, I)
log-density.  All buffers are allocated once; no call reads back to the host
inside the loop.
"""
from __future__ import annotations

import numpy as np
import torch

from . import yy
from .workloads import Workload


class GpuFilter:
    def __init__(self, w: Workload, prec: str | None = None, device: int = 0, stream=None,
                 want_cov: bool = False, ess_min: float = 0.0):
        self.w = w
        self.dev = torch.device("cuda", device)
        self.prec = prec or w.precision
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.ctx = yy.yy_create(device, self.stream)
        self.model = yy.Model(w.r, w.m, w.drift, w.A, w.obs, w.H, w.h_shift, w.q, w.rho2, device=self.dev)
        self.scales = yy.Scales(w.scales)
        n, r = w.n, w.r
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.codes = torch.empty(n * r, dtype=torch.int32, device=self.dev)
        self.x = torch.empty(n * r, **f64)
        self.lo = torch.empty(r, **f64)
        self.hi = torch.empty(r, **f64)
        self.lw = [torch.empty(n, **f64), torch.empty(n, **f64)]
        self.cur = 0
        self.wts = torch.empty(n, **f64)
        self.mean = torch.zeros(r, **f64)
        self.cov = torch.empty(r * r, **f64) if want_cov else None
        self.logZ_step = torch.zeros(1, **f64)
        self.logZ_acc = torch.zeros(1, **f64)
        self.logZ_scratch = torch.zeros(1, **f64)   # restart priors do not enter logZ_acc
        self.hist = torch.zeros(max(w.K, 1), r, **f64)
        self.logZ_hist = torch.zeros(max(w.K, 1), **f64)
        self.ess_hist = torch.zeros(max(w.K, 1), **f64)
        self.ess = torch.zeros(1, **f64)
        self.idx = torch.empty(n, dtype=torch.int64, device=self.dev)
        self.zero_r = torch.zeros(r, **f64)
        self.ess_min = ess_min
        self.version = 0
        self.dys = None

    def close(self):
        if self.ctx is not None:
            yy.yy_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_observations(self, dys: np.ndarray):
        self.dys = torch.as_tensor(np.ascontiguousarray(dys), dtype=torch.float64, device=self.dev)

    def init(self):
        w = self.w
        with torch.cuda.stream(self.stream):
            self.logZ_acc.zero_()
        yy.yy_nodes_sobol(self.ctx, w.r, w.n, 0, True, w.seed, None, None, self.codes, None)
        # initial density N(0, I) on [-box_half, box_half]^r: the restart map centred at 0
        yy.yy_restart(self.ctx, w.n, w.r, self.codes, None, self.zero_r, None, 0, w.box_half, 0.0, w.seed,
                      None, self.lo, self.hi, self.x, self.lw[self.cur])
        self.version += 1
        self._normalise(want_cov=False, acc=self.logZ_scratch)

    def _normalise(self, want_cov, acc):
        w = self.w
        yy.yy_normalise_moments(self.ctx, w.n, w.r, self.x, self.lw[self.cur], self.wts, self.logZ_step,
                                acc, self.mean, self.cov if want_cov else None, self.ess)

    def step(self, k: int, restart: bool | None = None, want_cov: bool = False):
        """Filter step k (1-based) with observation increment dys[k-1]."""
        w = self.w
        src, dst = self.lw[self.cur], self.lw[1 - self.cur]
        yy.yy_propagate(self.ctx, self.model, self.scales, self.prec, w.n, self.x, self.version, self.lo,
                        self.hi, w.dt, src, dst)
        self.cur = 1 - self.cur
        yy.yy_loglik_update(self.ctx, self.model, w.n, self.x, self.dys[k - 1], w.dt, dst)
        self._normalise(want_cov, acc=self.logZ_acc)
        with torch.cuda.stream(self.stream):
            self.hist[k - 1].copy_(self.mean)
            self.logZ_hist[k - 1].copy_(self.logZ_step[0])
            self.ess_hist[k - 1].copy_(self.ess[0])
        if restart is None:
            restart = bool(w.restart_every) and k % w.restart_every == 0 and k < w.K
        if restart:
            self.restart(k)

    def restart(self, k: int):
        w = self.w
        yy.yy_restart(self.ctx, w.n, w.r, self.codes, self.wts, self.mean, self.ess, k, w.R, self.ess_min,
                      w.seed, self.idx, self.lo, self.hi, self.x, self.lw[self.cur])
        self.version += 1
        self._normalise(want_cov=False, acc=self.logZ_scratch)
