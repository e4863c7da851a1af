"""Discrete Kalman filter: the closed-form limit of the filter on a linear-Gaussian model.

TEST INFRASTRUCTURE ONLY (used by the oracle's pins and the statistical checks).

For dx = A x dt + sqrt(q) dV, dy = H x dt + sqrt(rho2) dW discretised by
Euler-Maruyama with step dt (state x_k = (I + dt A) x_{k-1} + N(0, q dt I),
observation increment dy_k = dt H x_k + N(0, rho2 dt I)), the push-form kernel
of the filter at a single scale is exactly the Kalman prediction density and
the Ito-corrected update is exactly the Gaussian likelihood of dy_k, so the
filter's posterior mean converges to the Kalman filter's mean as the node set
is refined (Sec. 11.3 compares against the Kalman-Bucy filter for this reason).
"""
from __future__ import annotations

import numpy as np


def kalman_filter(A, H, q, rho2, dt, dys, m0, P0):
    """Returns (means [K, r], covariances [K, r, r]) after each update."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    H = np.atleast_2d(np.asarray(H, dtype=np.float64))
    r = A.shape[0]
    Phi = np.eye(r) + dt * A
    Q = q * dt * np.eye(r)
    Hd = dt * H
    Rm = rho2 * dt * np.eye(H.shape[0])
    m = np.asarray(m0, dtype=np.float64).reshape(r).copy()
    P = np.asarray(P0, dtype=np.float64).reshape(r, r).copy()
    means, covs = [], []
    for dy in np.atleast_2d(np.asarray(dys, dtype=np.float64)):
        m = Phi @ m
        P = Phi @ P @ Phi.T + Q
        S = Hd @ P @ Hd.T + Rm
        K = np.linalg.solve(S, Hd @ P).T
        m = m + K @ (dy - Hd @ m)
        P = (np.eye(r) - K @ Hd) @ P
        P = 0.5 * (P + P.T)
        means.append(m.copy())
        covs.append(P.copy())
    return np.array(means), np.array(covs)


def kalman_bucy(A, H, q, rho2, dt, dys, m0, P0, substeps: int = 8):
    """Continuous-time Kalman-Bucy filter driven by the increments dy_k.

    dm = A m dt + P H^T rho2^-1 (dy - H m dt), dP/dt = A P + P A^T + q I - P H^T H P / rho2,
    the Riccati equation integrated with classical RK4 on `substeps` sub-steps per dt and the
    mean equation with the increment spread evenly over the sub-steps.
    """
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    H = np.atleast_2d(np.asarray(H, dtype=np.float64))
    r = A.shape[0]
    m = np.asarray(m0, dtype=np.float64).reshape(r).copy()
    P = np.asarray(P0, dtype=np.float64).reshape(r, r).copy()
    h = dt / substeps

    def ric(P):
        return A @ P + P @ A.T + q * np.eye(r) - P @ H.T @ H @ P / rho2

    means = []
    for dy in np.atleast_2d(np.asarray(dys, dtype=np.float64)):
        for _ in range(substeps):
            gain = P @ H.T / rho2
            m = m + h * (A @ m) + gain @ (dy / substeps - h * (H @ m))
            k1 = ric(P)
            k2 = ric(P + 0.5 * h * k1)
            k3 = ric(P + 0.5 * h * k2)
            k4 = ric(P + h * k3)
            P = P + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        means.append(m.copy())
    return np.array(means)
