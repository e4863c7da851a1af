"""The oracle's filter loop (Sec. 2.2.2 procedure with the Sec. 6 local restart).

TEST INFRASTRUCTURE ONLY.  Calls the FP64 C oracle step by step:
propagate -> log-likelihood update -> normalise/moments, and every
`restart_every` steps the local resample-restart.  The initial density is
N(0, I) evaluated at the nodes (up to a constant); the restart prior is the
same density re-centred at the current estimate.
"""
from __future__ import annotations

import numpy as np

from . import (DIV_CLOSED, FORM_PUSH, OModel, codes_to_points, is_boundary, kernel_coefficients, loglik_update,
               loglik_update_ex, normalise_moments, propagate_ex, resample, restart_nodes, sobol_codes)


def model_of(w) -> OModel:
    return OModel(w.r, w.m, w.drift, w.A, w.obs, w.H, w.h_shift, w.q, w.rho2)


def initial_state(w, codes):
    """Nodes in [-box_half, box_half]^r and the N(0, I) log-density (boundary nodes -inf)."""
    lo = -w.box_half * np.ones(w.r)
    hi = w.box_half * np.ones(w.r)
    x = codes_to_points(codes, lo, hi)
    lw = -0.5 * np.sum(x * x, axis=1)
    lw[is_boundary(x, lo, hi)] = -np.inf
    return lo, hi, x, lw


def run_filter(w, dys, steps=None, codes=None, want_cov=False, form=FORM_PUSH, div_mode=DIV_CLOSED, apinv=None,
               logdet_a=0.0, bpinv=None):
    """Returns dict with per-step means, logZ, ESS, resample indices and the final state.

    form / div_mode: the first-order kernel (push form, or the pull form of eq. kernel with its
    divergence); apinv, logdet_a: general process noise (a^+, log det_+ a; default a = q I);
    bpinv: general observation noise b^+ (default b = rho2 I)."""
    model = model_of(w)
    K = w.K if steps is None else steps
    s = np.asarray(w.scales, dtype=np.float64)
    c = kernel_coefficients(s)
    if codes is None:
        codes = sobol_codes(w.r, w.n, 0, True, w.seed)
    lo, hi, x, lw = initial_state(w, codes)
    st = normalise_moments(x, lw, 0.0, want_cov=False)
    lw = st["logw"]
    logZ_acc = 0.0
    means, logZs, esss, clamps, idxs, covs = [], [], [], [], [], []
    for k in range(1, K + 1):
        lw, ncl = propagate_ex(model, s, c, x, lo, hi, w.dt, lw, form=form, div_mode=div_mode, apinv=apinv,
                               logdet_a=logdet_a)
        if bpinv is None:
            lw = loglik_update(model, x, dys[k - 1], w.dt, lw)
        else:
            lw = loglik_update_ex(model, x, dys[k - 1], w.dt, bpinv, lw)
        st = normalise_moments(x, lw, logZ_acc, want_cov=want_cov)
        if st["status"] != 0:
            raise FloatingPointError(f"all weights vanished at step {k}")
        lw, logZ_acc = st["logw"], st["logZ_acc"]
        means.append(st["mean"])
        logZs.append(st["logZ_step"])
        esss.append(st["ess"])
        clamps.append(ncl)
        if want_cov:
            covs.append(st["cov"])
        if w.restart_every and k % w.restart_every == 0 and k < K:
            idxs.append(resample(st["w"], w.seed, k))
            lo, hi, x, lw = restart_nodes(codes, st["mean"], w.R)
            lw = normalise_moments(x, lw, 0.0, want_cov=False)["logw"]
    return dict(means=np.array(means), logZ=np.array(logZs), ess=np.array(esss),
                clamps=np.array(clamps), resample_idx=idxs, x=x, logw=lw, lo=lo, hi=hi,
                covs=np.array(covs) if want_cov else None)
