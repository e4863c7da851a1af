"""The paper's large-scale cubic sensor test (its drift with the bidiagonal A and
A1, h = (x - 100)^3, unit noise) through the library against the oracle's filter:
short runs at the paper's r = 10 and r = 50 sizes, and longer ones -- all 1000
steps at r = 10, 200 steps at r = 100 and 40 steps at r = 300 -- held to the
"same error" bar (posterior means within 1e-3, RMSE to the true path within 1 %)."""
import numpy as np
import pytest
import torch

from oracle import filter as ofilter
from paper_2509_16896_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r,prec", [(10, "fp32"), (50, "fp32"), (50, "bf16x3p"), (50, "bf16x3s")])
def test_paper_large_scale_short_run(r, prec):
    from paper_2509_16896_amd.filter import GpuFilter
    w = W.shrink(W.paper_e1(r), K=20)
    xs, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys)
    f = GpuFilter(w, prec=prec)
    try:
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        torch.cuda.synchronize()
        got = f.hist.cpu().numpy()
    finally:
        f.close()
    err = float(np.max(np.abs(got - ref["means"])))
    print(f"r={r} [{prec}]: max |mean - oracle| = {err:.3g}, RMSE to truth {W.rmse(got, xs[1:]):.3f} "
          f"(oracle {W.rmse(ref['means'], xs[1:]):.3f})")
    assert np.all(np.isfinite(got))
    assert err <= 1e-5


@pytest.mark.parametrize("r,K,prec", [(10, 1000, "fp32"), (100, 200, "bf16x3p"), (300, 40, "bf16x3p")])
def test_paper_large_scale_long_run(r, K, prec):
    from paper_2509_16896_amd.filter import GpuFilter
    w = W.shrink(W.paper_e1(r), K=K)
    xs, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys)
    f = GpuFilter(w, prec=prec)
    try:
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        torch.cuda.synchronize()
        got = f.hist.cpu().numpy()
    finally:
        f.close()
    err = float(np.max(np.abs(got - ref["means"])))
    rg, ro = W.rmse(got, xs[1:]), W.rmse(ref["means"], xs[1:])
    print(f"r={r} K={K} [{prec}]: max |mean - oracle| = {err:.3g}, RMSE {rg:.4f} (oracle {ro:.4f})")
    assert np.all(np.isfinite(got))
    assert err <= 1e-3
    assert abs(rg - ro) <= 0.01 * ro
