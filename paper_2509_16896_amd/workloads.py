"""Seeded synthetic workloads: model parameters, true trajectories and observation increments.

This module is shared by the GPU path's tests/benchmark and by the oracle's
tests.  It holds none of the filter's arithmetic: it only draws the inputs the
filter consumes (Sec. 11: truth and observations are simulated by the
Euler-Maruyama scheme with the filter's step dt) and describes the workload
shapes.  It imports neither the GPU binding nor the oracle.

Euler-Maruyama alignment (the paper only says the SDEs are discretised with
step dt): x_k = x_{k-1} + f(x_{k-1}) dt + sqrt(q dt) xi_k and
dy_k = h(x_k) dt + sqrt(rho2 dt) eta_k, so dy_k observes the post-step state.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

F_ZERO, F_COS, F_LINEAR, F_PAPER_SINMIX = 0, 1, 2, 3
H_IDENTITY, H_CUBE, H_LINEAR = 0, 1, 2


@dataclasses.dataclass
class Workload:
    name: str
    r: int
    n: int
    dt: float
    K: int
    drift: int
    obs: int
    q: float
    rho2: float
    scales: tuple
    box_half: float          # half-width of the initial box (centred at 0) or the restart box
    restart_every: int       # 0 = never restart
    R: float                 # restart half-width
    seed: int = 0
    h_shift: float = 0.0
    A: np.ndarray | None = None
    H: np.ndarray | None = None
    precision: str = "bf16x3"
    U: np.ndarray | None = None   # general process-noise coefficient (a = U U^T), else sqrt(q) I
    V: np.ndarray | None = None   # general observation-noise coefficient (b = V V^T), else sqrt(rho2) I

    @property
    def m(self) -> int:
        return self.r if self.H is None else self.H.shape[0]


def linear_drift_matrix(r: int, seed: int = 0) -> np.ndarray:
    """A = -0.5 I + 0.1 G / sqrt(r), G_ij ~ N(0, 1) (linear-Gaussian workload)."""
    g = np.random.default_rng(seed).standard_normal((r, r))
    return -0.5 * np.eye(r) + 0.1 * g / math.sqrt(r)


def cubic_r2() -> Workload:
    """Plain cubic sensor r=2: f=cos, h=x^3, unit noise, n=1024 on [-4,4]^2, dt=0.01, 100 steps, scales {1,2}."""
    return Workload("cubic_r2_n1024", r=2, n=1024, dt=0.01, K=100, drift=F_COS, obs=H_CUBE, q=1.0,
                    rho2=1.0, scales=(1.0, 2.0), box_half=4.0, restart_every=0, R=4.0, seed=0,
                    precision="fp32")


def linear_r10() -> Workload:
    """Linear-Gaussian r=10: f=Ax, h=x, noise covariances 0.1 I, n=4096, dt=0.01, 200 steps."""
    return Workload("linear_r10_n4096", r=10, n=4096, dt=0.01, K=200, drift=F_LINEAR, obs=H_IDENTITY,
                    q=0.1, rho2=0.1, scales=(1.0,), box_half=3.0, restart_every=2, R=0.75, seed=0,
                    A=linear_drift_matrix(10, 0), precision="fp32")


def cubic_r100() -> Workload:
    """Cubic sensor r=100, noise std 0.3, n=16384, dt=0.005, 100 steps, scales {1,2,4}."""
    return Workload("cubic_r100_n16384", r=100, n=16384, dt=0.005, K=100, drift=F_COS, obs=H_CUBE,
                    q=0.09, rho2=0.09, scales=(1.0, 2.0, 4.0), box_half=0.3, restart_every=2, R=0.3,
                    seed=0)


def cubic_r1000() -> Workload:
    """Cubic sensor r=1000, noise std 0.3, n=65536, dt=0.005, 50 steps, scales {1,2,4}."""
    return Workload("cubic_r1000_n65536", r=1000, n=65536, dt=0.005, K=50, drift=F_COS, obs=H_CUBE,
                    q=0.09, rho2=0.09, scales=(1.0, 2.0, 4.0), box_half=0.3, restart_every=2, R=0.3,
                    seed=0)


# (r, n) pairs of the paper's large-scale test
PAPER_E1_SIZES = ((10, 100), (50, 300), (100, 500), (300, 800), (600, 1000), (1000, 2000))


def paper_e1(r: int, seed: int = 0) -> Workload:
    """The paper's large-scale cubic sensor test: f = sin(x)(Ax) + sin(2x)(A1 x) with its bidiagonal A and
    A1, h = (x - 100)^3, unit noise, dt = 0.01, 1000 steps, restarts of half-width 0.3 every 2 steps, n as
    the paper pairs it with r; scales {1,2,4} and an initial box of half-width 3 around the prior N(0, I).
    The chosen form BF16X3P where r >= 32; below that the matrix cores would pad every K stage to 32
    coordinates, and the plain FP32 form on the vector ALUs is both exact and faster."""
    n = dict(PAPER_E1_SIZES)[r]
    return Workload(f"paper_e1_r{r}_n{n}", r=r, n=n, dt=0.01, K=1000, drift=F_PAPER_SINMIX, obs=H_CUBE, q=1.0,
                    rho2=1.0, scales=(1.0, 2.0, 4.0), box_half=3.0, restart_every=2, R=0.3, seed=seed,
                    h_shift=100.0, precision="bf16x3p" if r >= 32 else "fp32")


def batch_runs(count: int = 64, seed: int = 0):
    """Batch of independent cubic-sensor runs: r ~ U{10..200}, n = 2^U{11..15}, dt=0.01, 100 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        r = int(rng.integers(10, 201))
        n = int(2 ** rng.integers(11, 16))
        out.append(Workload(f"batch{b}_r{r}_n{n}", r=r, n=n, dt=0.01, K=100, drift=F_COS, obs=H_CUBE,
                            q=0.09, rho2=0.09, scales=(1.0, 2.0, 4.0), box_half=0.3, restart_every=2,
                            R=0.3, seed=b))
    return out


def shrink(w: Workload, *, n=None, K=None, r=None, name=None) -> Workload:
    """Same workload family at a smaller size (for tests)."""
    kw = dataclasses.asdict(w)
    if r is not None and r != w.r:
        kw["r"] = r
        if w.A is not None:
            kw["A"] = linear_drift_matrix(r, w.seed)
    if n is not None:
        kw["n"] = n
    if K is not None:
        kw["K"] = K
    kw["name"] = name or f"{w.name}_mini"
    return Workload(**kw)


def _drift_np(w: Workload, x: np.ndarray) -> np.ndarray:
    if w.drift == F_ZERO:
        return np.zeros_like(x)
    if w.drift == F_COS:
        return np.cos(x)
    if w.drift == F_PAPER_SINMIX:
        nxt = np.concatenate([x[..., 1:], np.zeros_like(x[..., :1])], axis=-1)   # x_{k+1}, 0 past the last
        return np.sin(x) * (-0.5 * x + 0.1 * nxt) + np.sin(2.0 * x) * (-0.3 * x + 0.3 * nxt)
    return x @ w.A.T


def _obs_np(w: Workload, x: np.ndarray) -> np.ndarray:
    if w.obs == H_IDENTITY:
        return x.copy()
    if w.obs == H_CUBE:
        return (x - w.h_shift) ** 3
    return x @ w.H.T


def simulate(w: Workload, seed: int | None = None):
    """True states x_0..x_K and observation increments dy_1..dy_K (arrays [K+1, r], [K, m])."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    x = rng.standard_normal(w.r)  # x_0 ~ N(0, I)
    xs = [x.copy()]
    dys = []
    sq, so = math.sqrt(w.q * w.dt), math.sqrt(w.rho2 * w.dt)
    sdt = math.sqrt(w.dt)
    for _ in range(w.K):
        xi = rng.standard_normal(w.r)
        x = x + _drift_np(w, x[None, :])[0] * w.dt + (sq * xi if w.U is None else sdt * (w.U @ xi))
        eta = rng.standard_normal(w.m)
        dy = _obs_np(w, x[None, :])[0] * w.dt + (so * eta if w.V is None else sdt * (w.V @ eta))
        xs.append(x.copy())
        dys.append(dy)
    return np.array(xs), np.array(dys)


def random_logw(n: int, seed: int, spread: float = 5.0) -> np.ndarray:
    """Seeded log-weights for per-call parity cases (finite, spread over `spread` nats)."""
    return -spread * np.random.default_rng(seed + 7919).random(n)


def rmse(xhat: np.ndarray, xtrue: np.ndarray) -> float:
    """RMSE = sqrt( sum_k |xhat_k - x_k|^2 / (K r) ) (Sec. 11, error metrics)."""
    d = np.asarray(xhat) - np.asarray(xtrue)
    return float(math.sqrt(np.sum(d * d) / d.size))


def mean_error(xhat: np.ndarray, xtrue: np.ndarray) -> float:
    """ME = (1/K) sum_k sqrt(|xhat_k - x_k|^2 / r) (Sec. 11, error metrics)."""
    d = np.asarray(xhat) - np.asarray(xtrue)
    return float(np.mean(np.sqrt(np.sum(d * d, axis=1) / d.shape[1])))
