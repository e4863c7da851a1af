"""FP64 oracle of the learned restart proposal.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain NumPy in double
precision, one function per step, no blocking or fusion.

The paper places every restart box at the current estimate with a fixed
half-width R (Sec. 6).  The learned proposal replaces the fixed box by one
predicted from the estimate, with the plain box as fallback:

* network: x_hat (r) -> Linear(r, H) -> GELU -> Linear(H, H) -> GELU ->
  Linear(H, 2r) -> (delta, u); GELU is the exact erf form x * Phi(x);
* proposed box: centre x_hat + delta, half-width R * exp(u) per coordinate;
  the box is read as +-KAPPA standard deviations of a diagonal Gaussian,
  s = (R / KAPPA) * exp(u);
* training loss: the Gaussian negative log-likelihood of the posterior
  samples the filter produces at the next restart, written with their
  per-coordinate sample mean mu and variance v (an exact identity for a
  diagonal Gaussian), with a variance floor V0_FRAC * (R / KAPPA)^2 and the
  constant (1/2) log(2 pi) dropped, averaged over coordinates and pairs;
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction;
* checks before the learned box is used: coverage of the current posterior
  samples (fraction of sample coordinates inside the box) at least
  cover_min; their mean log-density under the learned box's Gaussian at
  least that under the plain box's; the effective sample size of the new
  nodes' prior weights at least ess_min.  Otherwise the plain box is used.

Parameter vector layout (FP32 on the GPU, FP64 here): W1 [H x r] row-major,
b1 [H], W2 [H x H], b2 [H], W3 [2r x H], b3 [2r].

Parity status: pinned (tests/test_oracle_proposal.py): GELU against
scipy's normal CDF and its symmetry identity; the loss against the
brute-force Gaussian log-density of explicit samples (scipy); the analytic
backward against central finite differences; Adam's first step in closed
form and convergence on a quadratic; checks against direct counts, scipy
log-densities and the closed-form ESS of equal weights.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

KAPPA = 3.0          # box half-width = KAPPA standard deviations
V0_FRAC = 0.01       # variance floor, as a fraction of (R / KAPPA)^2
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def num_params(r: int, H: int) -> int:
    return H * r + H + H * H + H + 2 * r * H + 2 * r


def unpack(p: np.ndarray, r: int, H: int):
    """Views of the flat parameter vector: W1, b1, W2, b2, W3, b3."""
    o = 0
    out = []
    for shape in [(H, r), (H,), (H, H), (H,), (2 * r, H), (2 * r,)]:
        size = int(np.prod(shape))
        out.append(p[o:o + size].reshape(shape))
        o += size
    assert o == p.size
    return out


def gelu(x):
    """GELU, exact form: x * Phi(x) = x/2 * (1 + erf(x / sqrt 2))."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(p, xhat, r, H):
    """Network outputs [B x 2r] (delta then u) and the intermediate values for the backward."""
    W1, b1, W2, b2, W3, b3 = unpack(p, r, H)
    z1 = xhat @ W1.T + b1
    a1 = gelu(z1)
    z2 = a1 @ W2.T + b2
    a2 = gelu(z2)
    out = a2 @ W3.T + b3
    return out, (xhat, z1, a1, z2, a2)


def loss_and_dout(out, xhat, mu, var, R):
    """Mean Gaussian NLL per coordinate and pair, and its gradient w.r.t. the outputs."""
    B, r2 = out.shape
    r = r2 // 2
    delta, u = out[:, :r], out[:, r:]
    s0 = R / KAPPA
    s2 = (s0 * np.exp(u)) ** 2
    e = mu - xhat - delta
    A = var + V0_FRAC * s0 * s0 + e * e
    terms = A / (2.0 * s2) + np.log(s0) + u
    loss = terms.sum() / (B * r)
    dout = np.empty_like(out)
    dout[:, :r] = -e / s2 / (B * r)
    dout[:, r:] = (1.0 - A / s2) / (B * r)
    return loss, dout


def backward(p, cache, dout, r, H):
    """Gradient of the loss w.r.t. the flat parameter vector, given d loss / d outputs."""
    W1, b1, W2, b2, W3, b3 = unpack(p, r, H)
    xhat, z1, a1, z2, a2 = cache
    g = np.zeros_like(p)
    gW1, gb1, gW2, gb2, gW3, gb3 = unpack(g, r, H)
    gW3[...] = dout.T @ a2
    gb3[...] = dout.sum(axis=0)
    da2 = dout @ W3
    dz2 = da2 * gelu_grad(z2)
    gW2[...] = dz2.T @ a1
    gb2[...] = dz2.sum(axis=0)
    da1 = dz2 @ W2
    dz1 = da1 * gelu_grad(z1)
    gW1[...] = dz1.T @ xhat
    gb1[...] = dz1.sum(axis=0)
    return g


def loss_grad(p, xhat, mu, var, R, r, H):
    out, cache = forward(p, xhat, r, H)
    loss, dout = loss_and_dout(out, xhat, mu, var, R)
    return loss, backward(p, cache, dout, r, H)


def adam_step(p, g, m, v, t, lr):
    """One Adam update (t = 1 for the first step); returns new (p, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * g
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * g * g
    mh = m / (1.0 - ADAM_B1 ** t)
    vh = v / (1.0 - ADAM_B2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


def learned_box(out_row, xhat, R):
    """Centre and half-width of the proposed box from one output row."""
    r = xhat.size
    return xhat + out_row[:r], R * np.exp(out_row[r:])


def sample_moments(x, idx):
    """Per-coordinate mean and (1/n) variance of the resampled nodes x[idx] (two passes)."""
    y = x[idx]
    mu = y.mean(axis=0)
    return mu, ((y - mu) ** 2).mean(axis=0)


def coverage(x, idx, centre, half):
    """Fraction of sample coordinates inside the box."""
    y = x[idx]
    return float(np.mean(np.abs(y - centre) <= half))


def mean_log_density(x, idx, centre, half):
    """Mean over samples of the diagonal Gaussian log-density with s = half / KAPPA."""
    y = x[idx]
    s = half / KAPPA
    z = (y - centre) / s
    per = -0.5 * z * z - np.log(s) - 0.5 * math.log(2.0 * math.pi)
    return float(per.sum(axis=1).mean())


def prior_ess(lw):
    """(sum w)^2 / sum w^2 of the weights exp(lw) over finite entries."""
    f = lw[np.isfinite(lw)]
    if f.size == 0:
        return 0.0
    m = f.max()
    e = np.exp(f - m)
    return float(e.sum() ** 2 / (e * e).sum())


def learned_restart(p, r, H, x_cur, idx, xhat, R, codes, cover_min, ess_min, codes_to_points, is_boundary):
    """The learned restart's box decision.  Returns (used, lo, hi, x_new, lw_new)."""
    out, _ = forward(p, xhat[None, :], r, H)
    c, hw = learned_box(out[0], xhat, R)
    ok = (coverage(x_cur, idx, c, hw) >= cover_min and
          mean_log_density(x_cur, idx, c, hw) >= mean_log_density(x_cur, idx, xhat, R * np.ones(r)))

    def place(lo, hi):
        xn = codes_to_points(codes, lo, hi)
        lw = -0.5 * np.sum((xn - xhat) ** 2, axis=1)
        lw[is_boundary(xn, lo, hi)] = -np.inf
        return xn, lw

    if ok:
        lo, hi = c - hw, c + hw
        xn, lw = place(lo, hi)
        if prior_ess(lw) >= ess_min:
            return True, lo, hi, xn, lw
    lo, hi = xhat - R, xhat + R
    xn, lw = place(lo, hi)
    return False, lo, hi, xn, lw
