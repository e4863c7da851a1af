"""The filter's time loop on the GPU, built on the libyy calls (Sec. 2.2.2 procedure, Sec. 6 restart).

Per step k: yy_propagate -> yy_loglik_update -> yy_normalise_moments, and every
``restart_every`` steps yy_restart (resampling, new box around the estimate --
the plain box, or the learned proposal's box with the plain one as fallback --
the reference codes mapped into it, the re-centred prior) followed by a
normalisation.  Node sets are double-buffered so that a restart can read the
current nodes (the posterior samples) while it writes the new ones.  The initial state is the restart map with centre 0 and
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
                 want_cov: bool = False, ess_min: float = 0.0, proposal_params=None, hidden: int = 256,
                 cover_min: float = 0.95, collect_pairs: bool = False, one_pass: bool = True,
                 form: str = "push", div: int = 0, operator: bool = False):
        """one_pass: each step's correction and normalisation through yy_loglik_normalise (x read
        once where it can); False makes the two calls yy_loglik_update and yy_normalise_moments, the
        sequence the batched step reproduces bit for bit.  form: the first-order kernel, "push" or
        "pull" (eq. kernel, with the divergence in closed form, div = 0, or by complex step, div = 1).
        operator: predict with the stored operator (Sec. 10 offline/online split) -- built once per
        node set by yy_operator_build, applied every step by yy_operator_apply -- instead of
        yy_propagate's recomputation."""
        self.w = w
        self.one_pass = one_pass
        self.dev = torch.device("cuda", device)
        self.prec = prec or w.precision
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.ctx = yy.yy_create(device, self.stream)
        # general noise coefficients a = U U^T, b = V V^T (Sec. 7), when the workload gives them
        self.noise = None
        if w.U is not None or w.V is not None:
            self.noise = yy.yy_noise_create(self.ctx, w.r, w.U, w.m, w.V)
        self.model = yy.Model(w.r, w.m, w.drift, w.A, w.obs, w.H, w.h_shift, w.q, w.rho2, device=self.dev,
                              noise=self.noise)
        self.scales = yy.Scales(w.scales, form=form, div=div)
        n, r = w.n, w.r
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.codes = torch.empty(n * r, dtype=torch.int32, device=self.dev)
        self.xbuf = [torch.empty(n * r, **f64), torch.empty(n * r, **f64)]
        self.xi = 0
        self.lo = torch.empty(r, **f64)
        self.hi = torch.empty(r, **f64)
        self.lw = [torch.empty(n, **f64), torch.empty(n, **f64)]
        self.cur = 0
        self.wts = torch.empty(n, **f64)
        self.mean_buf = torch.zeros(r, **f64)
        self.mean = self.mean_buf   # the latest posterior mean (a history row after a step)
        self.cov = torch.empty(r * r, **f64) if want_cov else None
        self.logZ_step = torch.zeros(1, **f64)
        self.logZ_acc = torch.zeros(1, **f64)
        self.logZ_scratch = torch.zeros(1, **f64)   # restart priors do not enter logZ_acc
        self.hist = torch.zeros(max(w.K, 1), r, **f64)
        self.logZ_hist = torch.zeros(max(w.K, 1), **f64)
        self.ess_hist = torch.zeros(max(w.K, 1), **f64)
        self.ess_buf = torch.zeros(1, **f64)
        self.ess = self.ess_buf     # the latest ESS
        self.idx = torch.empty(n, dtype=torch.int64, device=self.dev)
        self.zero_r = torch.zeros(r, **f64)
        self.ess_min = ess_min
        self.version = 0
        self.dys = None
        self.use_operator = operator
        self.op = None
        self.op_version = -1
        # learned restart proposal (a network created on this context from trained parameters)
        self.proposal = None
        self.cover_min = cover_min
        if proposal_params is not None:
            self.proposal = yy.yy_proposal_create(self.ctx, r, hidden, 0, proposal_params)
        self.used = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.used_count = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.restarts = 0
        # training pairs: (estimate at a restart, sample mean / variance at the next restart)
        self.collect = collect_pairs
        npairs = max(w.K // max(w.restart_every, 1), 1)
        self.pair_x = torch.zeros(npairs, r, **f64) if collect_pairs else None
        self.pair_mu = torch.zeros(npairs, r, **f64) if collect_pairs else None
        self.pair_var = torch.zeros(npairs, r, **f64) if collect_pairs else None
        self.prev_xhat = torch.zeros(r, **f64) if collect_pairs else None
        self.npairs = 0

    @property
    def x(self):
        return self.xbuf[self.xi]

    def close(self):
        if self.proposal is not None:
            yy.yy_proposal_destroy(self.proposal)
            self.proposal = None
        if getattr(self, "op", None) is not None:
            yy.yy_operator_destroy(self.op)
            self.op = None
        if getattr(self, "noise", None) is not None:
            yy.yy_noise_destroy(self.noise)
            self.noise = None
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
        yy.yy_restart(self.ctx, w.n, w.r, self.codes, None, None, self.zero_r, None, 0, w.box_half, 0.0, w.seed,
                      None, self.lo, self.hi, self.x, self.lw[self.cur])
        self.version += 1
        self._normalise(want_cov=False, acc=self.logZ_scratch)

    def _normalise(self, want_cov, acc, moments=True, row=None):
        """Normalise the current log-weights.  With `row`, the step's mean, logZ and ESS go straight
        into that row of the histories (self.mean and self.ess then refer to it); otherwise into the
        filter's own buffers."""
        w = self.w
        if row is None:
            mean, logz, ess = self.mean_buf, self.logZ_step, self.ess_buf
        else:
            mean, logz, ess = self.hist[row], self.logZ_hist[row:row + 1], self.ess_hist[row:row + 1]
        yy.yy_normalise_moments(self.ctx, w.n, w.r, self.x, self.lw[self.cur], self.wts if moments else None,
                                logz, acc, mean if moments else None, self.cov if want_cov else None, ess)
        if moments:
            self.mean = mean
        self.ess = ess

    def step(self, k: int, restart: bool | None = None, want_cov: bool = False):
        """Filter step k (1-based) with observation increment dys[k-1]."""
        w = self.w
        src, dst = self.lw[self.cur], self.lw[1 - self.cur]
        if self.use_operator:
            if self.op_version != self.version:   # offline stage: once per node set
                self.op = yy.yy_operator_build(self.ctx, self.model, self.scales, w.n, self.x, self.version, self.lo,
                                               self.hi, w.dt, self.op)
                self.op_version = self.version
            yy.yy_operator_apply(self.op, src, dst)
        else:
            yy.yy_propagate(self.ctx, self.model, self.scales, self.prec, w.n, self.x, self.version, self.lo,
                            self.hi, w.dt, src, dst)
        self.cur = 1 - self.cur
        row = k - 1
        if self.one_pass and not want_cov:
            yy.yy_loglik_normalise(self.ctx, self.model, w.n, self.x, self.dys[row], w.dt, dst, self.wts,
                                   self.logZ_hist[row:row + 1], self.logZ_acc, self.hist[row],
                                   self.ess_hist[row:row + 1])
            self.mean, self.ess = self.hist[row], self.ess_hist[row:row + 1]
        else:
            yy.yy_loglik_update(self.ctx, self.model, w.n, self.x, self.dys[row], w.dt, dst)
            self._normalise(want_cov, acc=self.logZ_acc, row=row)
        if restart is None:
            restart = bool(w.restart_every) and k % w.restart_every == 0 and k < w.K
        if restart:
            self.restart(k)

    def restart(self, k: int):
        w = self.w
        x_cur, x_new = self.xbuf[self.xi], self.xbuf[1 - self.xi]
        yy.yy_restart(self.ctx, w.n, w.r, self.codes, x_cur, self.wts, self.mean, self.ess, k, w.R, self.ess_min,
                      w.seed, self.idx, self.lo, self.hi, x_new, self.lw[self.cur], self.proposal, self.cover_min,
                      self.used if self.proposal is not None else None)
        if self.collect:
            if self.restarts > 0 and self.npairs < self.pair_x.shape[0]:
                j = self.npairs
                yy.yy_sample_moments(self.ctx, w.n, w.r, x_cur, self.idx, self.pair_mu[j], self.pair_var[j])
                with torch.cuda.stream(self.stream):
                    self.pair_x[j].copy_(self.prev_xhat)
                self.npairs += 1
            with torch.cuda.stream(self.stream):
                self.prev_xhat.copy_(self.mean)
        if self.proposal is not None:
            with torch.cuda.stream(self.stream):
                self.used_count.add_(self.used)
        self.restarts += 1
        self.xi = 1 - self.xi
        self.version += 1
        # the new prior: normalised log-weights only (the next step recomputes the moments)
        self._normalise(want_cov=False, acc=self.logZ_scratch, moments=False)
