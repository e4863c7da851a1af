"""yy_normalise_moments_noalloc (the normalisation with its partial sums in a static device array)
against yy_normalise_moments (partial sums in the context's allocated scratch), through the C ABI.

Both run the same kernels with the same block count, so every output must be bit-identical.  Two
calls in a row, the second with a smaller input (the static array keeps the first call's partial
sums, which the second must not see), then a call with the covariance, and the limits: r above the
array's maximum and a covariance without the caller's weights are refused before anything runs.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

yy = pytest.importorskip("paper_2509_16896_amd.yy")


def _inputs(n, r, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, r))
    lw = rng.standard_normal(n) * 30.0 - 500.0
    lw[rng.random(n) < 0.05] = -np.inf
    return x, lw


def _run(fn, ctx, x, lw, want_w=True, want_cov=False):
    n, r = x.shape
    d = dict(dtype=torch.float64, device="cuda")
    xd = torch.as_tensor(np.ascontiguousarray(x).reshape(-1), **d)
    lwd = torch.as_tensor(lw, **d)
    w = torch.full((n,), np.nan, **d) if want_w else None
    lz = torch.zeros(1, **d)
    acc = torch.full((1,), 2.5, **d)
    mean = torch.full((r,), np.nan, **d)
    cov = torch.full((r * r,), np.nan, **d) if want_cov else None
    ess = torch.zeros(1, **d)
    fn(ctx, n, r, xd, lwd, w, lz, acc, mean, cov, ess)
    torch.cuda.synchronize()
    out = dict(logw=lwd, logZ=lz, acc=acc, mean=mean, ess=ess)
    if want_w:
        out["w"] = w
    if want_cov:
        out["cov"] = cov
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_noalloc_normalisation_equals_the_allocating_call():
    stream = torch.cuda.current_stream()
    ctx = yy.yy_create(0, stream)
    try:
        # first call: large input; second: smaller n and r, so stale partial sums of the first
        # call sit in the static array beyond the second call's range
        for n, r, seed in ((70001, 1000, 1), (3001, 37, 2), (1, 2, 3)):
            x, lw = _inputs(n, r, seed)
            ref = _run(yy.yy_normalise_moments, ctx, x, lw)
            got = _run(yy.yy_normalise_moments_noalloc, ctx, x, lw)
            print(f"n={n} r={r}: logZ {got['logZ'][0]:.6f}, ess {got['ess'][0]:.4f}", flush=True)
            _same(got, ref)
            assert np.all(np.isfinite(got["mean"]))
        # with the covariance (the caller's weights) and without the weights array
        x, lw = _inputs(5000, 64, 4)
        _same(_run(yy.yy_normalise_moments_noalloc, ctx, x, lw, want_cov=True),
              _run(yy.yy_normalise_moments, ctx, x, lw, want_cov=True))
        _same(_run(yy.yy_normalise_moments_noalloc, ctx, x, lw, want_w=False),
              _run(yy.yy_normalise_moments, ctx, x, lw, want_w=False))
        # limits: refused on the host, nothing launched
        x, lw = _inputs(64, yy_max_r() + 1, 5)
        with pytest.raises(yy.YYError) as e:
            _run(yy.yy_normalise_moments_noalloc, ctx, x, lw)
        assert e.value.status == yy.YY_ERR_UNSUPPORTED
        x, lw = _inputs(64, 8, 6)
        with pytest.raises(yy.YYError) as e:
            _run(yy.yy_normalise_moments_noalloc, ctx, x, lw, want_w=False, want_cov=True)
        assert e.value.status == yy.YY_ERR_ARG
    finally:
        yy.yy_destroy(ctx)


def yy_max_r():
    return 1024   # YY_NOALLOC_MAX_R in include/yy.h
