"""End-to-end pin of the oracle filter: the linear-Gaussian case (Sec. 11.3 benchmark structure).

With one kernel scale, no restart and a box far wider than the posterior, the
push-form prediction is the Kalman prediction density and the Ito-corrected
update is the Gaussian likelihood, so the filter's posterior mean converges
to the discrete Kalman filter's mean as the node set is refined.
"""
import numpy as np

from oracle import filter as ofilter
from oracle.kalman import kalman_bucy, kalman_filter
from paper_2509_16896_amd import workloads as W


def _linear_workload(r, n, K, half, dt, q, rho2, A):
    return W.Workload(f"linear_r{r}", r=r, n=n, dt=dt, K=K, drift=W.F_LINEAR, obs=W.H_IDENTITY, q=q,
                      rho2=rho2, scales=(1.0,), box_half=half, restart_every=0, R=half, seed=3, A=A)


def test_r1_matches_kalman_filter(oracle_lib):
    w = _linear_workload(1, 2048, 60, 6.0, 0.01, 1.0, 1.0, np.array([[-0.5]]))
    xs, dys = W.simulate(w)
    out = ofilter.run_filter(w, dys)
    km, kP = kalman_filter(w.A, np.eye(1), w.q, w.rho2, w.dt, dys, np.zeros(1), np.eye(1))
    assert np.max(np.abs(out["means"] - km)) < 2e-5


def test_r2_matches_kalman_filter(oracle_lib):
    # 2-D Sobol quadrature of a Gaussian kernel is far less accurate than the 1-D grid of the r = 1
    # case, so this pin uses a wide kernel (dt = 0.5) and checks the error shrinks as n grows.
    A = np.array([[-0.5, 0.2], [-0.1, -0.3]])
    errs = []
    for n in (1024, 4096):
        w = _linear_workload(2, n, 20, 5.0, 0.5, 1.0, 0.5, A)
        xs, dys = W.simulate(w)
        out = ofilter.run_filter(w, dys)
        km, kP = kalman_filter(A, np.eye(2), w.q, w.rho2, w.dt, dys, np.zeros(2), np.eye(2))
        errs.append(np.max(np.abs(out["means"] - km)))
    assert errs[1] < 3e-3 and errs[1] < errs[0], errs


def test_kalman_bucy_is_the_continuous_limit():
    # the discrete filter and the continuous Kalman-Bucy filter agree to O(dt)
    A = np.array([[-0.5]])
    w = _linear_workload(1, 16, 400, 6.0, 0.005, 1.0, 1.0, A)
    xs, dys = W.simulate(w)
    km, _ = kalman_filter(A, np.eye(1), 1.0, 1.0, w.dt, dys, np.zeros(1), np.eye(1))
    kb = kalman_bucy(A, np.eye(1), 1.0, 1.0, w.dt, dys, np.zeros(1), np.eye(1))
    assert np.max(np.abs(km - kb)) < 0.02
