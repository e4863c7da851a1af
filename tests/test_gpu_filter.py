"""End-to-end parity: the GPU filter loop against the oracle's filter loop on the same
seeded workload (nodes, observations, restarts), posterior means to 1e-5 absolute."""
import numpy as np
import pytest
import torch

from oracle import filter as ofilter
from paper_2509_16896_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run_gpu(w, dys, prec):
    from paper_2509_16896_amd.filter import GpuFilter
    f = GpuFilter(w, prec=prec)
    f.set_observations(dys)
    f.init()
    for k in range(1, w.K + 1):
        f.step(k)
    torch.cuda.synchronize()
    out = dict(means=f.hist.cpu().numpy(), logZ=f.logZ_hist.cpu().numpy(), ess=f.ess_hist.cpu().numpy())
    f.close()
    return out


CASES = {
    "cubic_r2_n1024_K20": (W.shrink(W.cubic_r2(), K=20), "fp32"),
    # the plain cubic-sensor configuration in full: r=2, n=1024 on [-4,4]^2, 100 steps, scales {1,2}
    "cubic_r2_n1024_K100_full": (W.cubic_r2(), "fp32"),
    "linear_r10_n2048_K10_restart": (W.shrink(W.linear_r10(), n=2048, K=10), "fp32"),
    "cubic_r20_n1024_K6_restart_s124": (W.shrink(W.cubic_r100(), r=20, n=1024, K=6), "fp32"),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_filter_matches_oracle(name):
    w, prec = CASES[name]
    xs, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys)
    got = _run_gpu(w, dys, prec)
    err = np.max(np.abs(got["means"] - ref["means"]))
    print(f"{name}: max |mean - oracle| = {err:.3g}; RMSE gpu {W.rmse(got['means'], xs[1:]):.5f} "
          f"oracle {W.rmse(ref['means'], xs[1:]):.5f}")
    assert err <= 1e-5
    assert np.allclose(got["logZ"], ref["logZ"], rtol=1e-6, atol=1e-4)
    assert np.allclose(got["ess"], ref["ess"], rtol=1e-4)
