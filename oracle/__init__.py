"""FP64 CPU oracle of the improved Yau-Yau filter step (arXiv 2509.16896).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_2509_16896_amd``) never imports, links or runs it, and the two
share no code: the oracle is plain C in double precision (``yyo.c``) plus the
Kalman filter in ``kalman.py``; this module only marshals numpy arrays into it.

Every function below mirrors one C function; see ``yyo.h`` for the passage of
the paper each one follows.

Parity status of the oracle's functions and the tests that pin each one:

* SplitMix64 -- pinned: the published reference outputs for states 0 and
  1234567 (test_oracle_bruteforce.py::test_splitmix64_published_outputs).
* Sobol codes / points -- pinned: van der Corput closed form, Pascal matrix
  of the second dimension, scipy's unscrambled Sobol for dimensions 1-2,
  (0,m,2)-net and dyadic stratification invariants (test_oracle_sobol.py).
* kernel coefficients -- pinned: the printed alpha, beta, gamma of
  Theorem thm:2ndorderkernel; exact closed form for scales {1,2,4}
  (test_oracle_coefficients.py).
* propagation -- pinned: 50-digit linear-domain double sums for n <= 64,
  r in {1, 3}, one to three signed scales, boundary nodes, -inf weights and
  clamped rows (test_oracle_bruteforce.py::test_prediction_equals_50_digit_double_sum);
  linearity in the weights with three signed scales (::test_linearity_...);
  second-order consistency with scales {1,2,4} and first-order with one
  (::test_three_scales_are_second_order_consistent,
  test_oracle_propagate.py::test_first_order_consistency); single-source
  closed form with scipy's Gaussian log-density, mass conservation
  (test_oracle_propagate.py); Kalman filter limit end to end
  (test_oracle_kalman.py).
* log-likelihood update -- pinned: Gaussian likelihood closed form, Ito
  unbiasedness by Monte Carlo (test_oracle_update.py).
* normalisation / moments -- pinned: numpy weighted average / covariance,
  scipy's logsumexp, shift invariance (test_oracle_update.py).
* resampling -- pinned: exhaustive search with exact integers
  (test_oracle_bruteforce.py::test_resampling_equals_exhaustive_search),
  systematic-resampling count bounds and monotone ancestors
  (test_oracle_update.py).
* restart -- pinned: the reference set translated by the estimate and its
  mean (test_oracle_bruteforce.py::test_restart_translates_the_reference_set),
  containment and the prior's closed form (test_oracle_update.py).
* pull-form kernel (eq. kernel) -- pinned: single sources against scipy's
  Gaussian log-density centred at x_i - tau f(x_i) times exp(-tau div f(x_i))
  (test_oracle_pull_noise.py::test_pull_single_source_matches_gaussian_density);
  50-digit double sums for n <= 64 with signed scales
  (::test_pull_prediction_equals_50_digit_double_sum); first and second order
  consistency and agreement with the push form
  (::test_pull_form_consistency_orders_and_agreement_with_push).
* divergence (closed forms; the complex-step sum of Sec. 8) -- pinned:
  mpmath's 30-digit numerical derivative
  (::test_divergence_closed_form_and_complex_step_against_numerical_derivative).
* general noise a = U U^T, b = V V^T (Sec. 7) -- pinned: the Moore-Penrose
  conditions, numpy's pinv and the log pseudo-determinant of a rank-deficient a
  (::test_noise_pinv_moore_penrose_and_log_pseudo_determinant); a = q I against the
  isotropic path; single sources against scipy's full-covariance Gaussian,
  and in the range coordinates of a singular a; null-space invariance; the
  observation update against scipy's likelihood ratio with covariance b dt,
  invertible and singular (::test_general_noise_single_source_against_scipy,
  ::test_general_noise_linearity_and_pseudo_inverse_invariance,
  ::test_general_observation_noise_update).
* learned restart proposal (``proposal.py``, NumPy) -- pinned: GELU against
  scipy's normal CDF, loss against the brute-force Gaussian log-density of
  samples, backward against finite differences, Adam's closed-form first
  step, checks against direct counts (test_oracle_proposal.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libyyo.so")
_lib = None

F_ZERO, F_COS, F_LINEAR, F_PAPER_SINMIX = 0, 1, 2, 3
H_IDENTITY, H_CUBE, H_LINEAR = 0, 1, 2
FORM_PUSH, FORM_PULL = 0, 1
DIV_CLOSED, DIV_COMPLEX_STEP = 0, 1
# eigenvalues of a noise coefficient a = U U^T at or below this fraction of the largest count as zero
PINV_RTOL = 1e-10


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = [
            "gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
            os.path.join(_HERE, "yyo.c"), "-o", _LIB_PATH + ".tmp", "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Model(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_int32), ("m", ctypes.c_int32),
        ("drift", ctypes.c_int32), ("A", ctypes.c_void_p),
        ("obs", ctypes.c_int32), ("H", ctypes.c_void_p),
        ("h_shift", ctypes.c_double), ("q", ctypes.c_double), ("rho2", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.yyo_splitmix64_at.argtypes = [u64, u64]
    lib.yyo_splitmix64_at.restype = u64
    lib.yyo_primitive_poly.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)]
    lib.yyo_primitive_poly.restype = ctypes.c_int
    lib.yyo_sobol_directions.argtypes = [i32, P]
    lib.yyo_sobol_codes.argtypes = [i32, i64, i64, i32, u64, P]
    lib.yyo_codes_to_points.argtypes = [i32, i64, P, P, P, P]
    lib.yyo_is_boundary.argtypes = [i32, P, P, P]
    lib.yyo_is_boundary.restype = ctypes.c_int
    lib.yyo_kernel_coefficients.argtypes = [i32, P, P]
    lib.yyo_kernel_coefficients.restype = ctypes.c_int
    lib.yyo_drift.argtypes = [ctypes.POINTER(Model), P, P]
    lib.yyo_obs.argtypes = [ctypes.POINTER(Model), P, P]
    lib.yyo_propagate.argtypes = [ctypes.POINTER(Model), i32, P, P, i64, P, P, P, f64, P, P]
    lib.yyo_propagate.restype = i64
    lib.yyo_propagate_rows.argtypes = [ctypes.POINTER(Model), i32, P, P, i64, P, P, P, f64, P, i64, P, P]
    lib.yyo_propagate_rows.restype = i64
    lib.yyo_loglik_update.argtypes = [ctypes.POINTER(Model), i64, P, P, f64, P]
    lib.yyo_divergence.argtypes = [ctypes.POINTER(Model), P, i32, f64]
    lib.yyo_divergence.restype = f64
    lib.yyo_propagate_ex.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Kernel), i32, P, P, i64, P, P, P, f64,
                                     P, P]
    lib.yyo_propagate_ex.restype = i64
    lib.yyo_propagate_rows_ex.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Kernel), i32, P, P, i64, P, P, P,
                                          f64, P, i64, P, P]
    lib.yyo_propagate_rows_ex.restype = i64
    lib.yyo_loglik_update_ex.argtypes = [ctypes.POINTER(Model), i64, P, P, f64, P, P]
    lib.yyo_normalise_moments.argtypes = [i64, i32, P, P, P, P, P, P, P, P]
    lib.yyo_normalise_moments.restype = ctypes.c_int
    lib.yyo_resample.argtypes = [i64, P, u64, i64, P]
    lib.yyo_resample.restype = ctypes.c_int
    lib.yyo_restart_nodes.argtypes = [i64, i32, P, P, f64, P, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Kernel(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("div_mode", ctypes.c_int32), ("cs_step", ctypes.c_double),
                ("apinv", ctypes.c_void_p), ("logdet_a", ctypes.c_double)]


class OModel:
    """Host-side model description; keeps the A/H arrays alive."""

    def __init__(self, r, m=None, drift=F_COS, A=None, obs=H_CUBE, H=None, h_shift=0.0, q=1.0, rho2=1.0):
        self.r = int(r)
        self.m = int(m if m is not None else (H.shape[0] if H is not None else r))
        self.drift, self.obs = int(drift), int(obs)
        self.A = None if A is None else _f64(A).reshape(self.r, self.r)
        self.H = None if H is None else _f64(H).reshape(self.m, self.r)
        self.h_shift, self.q, self.rho2 = float(h_shift), float(q), float(rho2)
        self.c = Model(self.r, self.m, self.drift, _ptr(self.A), self.obs, _ptr(self.H),
                       self.h_shift, self.q, self.rho2)


def splitmix64_at(seed: int, counter: int) -> int:
    return int(_load().yyo_splitmix64_at(seed, counter))


def primitive_poly(idx: int) -> tuple[int, int]:
    p = ctypes.c_uint32(0)
    deg = _load().yyo_primitive_poly(idx, ctypes.byref(p))
    return deg, int(p.value)


def sobol_directions(r: int) -> np.ndarray:
    v = np.zeros((r, 32), dtype=np.uint32)
    _load().yyo_sobol_directions(r, _ptr(v))
    return v


def sobol_codes(r: int, n: int, first: int = 0, scramble: bool = True, seed: int = 0) -> np.ndarray:
    codes = np.zeros((n, r), dtype=np.uint32)
    _load().yyo_sobol_codes(r, n, first, int(bool(scramble)), seed & 0xFFFFFFFFFFFFFFFF, _ptr(codes))
    return codes


def codes_to_points(codes: np.ndarray, lo, hi) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    n, r = codes.shape
    lo, hi = _f64(lo), _f64(hi)
    x = np.zeros((n, r))
    _load().yyo_codes_to_points(r, n, _ptr(codes), _ptr(lo), _ptr(hi), _ptr(x))
    return x


def is_boundary(x: np.ndarray, lo, hi) -> np.ndarray:
    x = _f64(x)
    lo, hi = _f64(lo), _f64(hi)
    r = x.shape[1]
    lib = _load()
    return np.array([lib.yyo_is_boundary(r, _ptr(np.ascontiguousarray(x[i])), _ptr(lo), _ptr(hi))
                     for i in range(x.shape[0])], dtype=bool)


def kernel_coefficients(s) -> np.ndarray:
    s = _f64(s)
    c = np.zeros(len(s) + 1)
    rc = _load().yyo_kernel_coefficients(len(s), _ptr(s), _ptr(c))
    if rc != 0:
        raise ValueError(f"coefficient solve failed ({rc})")
    return c


def drift(model: OModel, x: np.ndarray) -> np.ndarray:
    x = _f64(x)
    out = np.zeros((x.shape[0], model.r))
    lib = _load()
    for i in range(x.shape[0]):
        xi = np.ascontiguousarray(x[i])
        fi = np.zeros(model.r)
        lib.yyo_drift(ctypes.byref(model.c), _ptr(xi), _ptr(fi))
        out[i] = fi
    return out


def obs(model: OModel, x: np.ndarray) -> np.ndarray:
    x = _f64(x)
    out = np.zeros((x.shape[0], model.m))
    lib = _load()
    for i in range(x.shape[0]):
        xi = np.ascontiguousarray(x[i])
        hi = np.zeros(model.m)
        lib.yyo_obs(ctypes.byref(model.c), _ptr(xi), _ptr(hi))
        out[i] = hi
    return out


def propagate(model: OModel, s, c, x, lo, hi, dt, logw_in):
    """Returns (logw_out, nclamped)."""
    s, c, x, lo, hi, lw = _f64(s), _f64(c), _f64(x), _f64(lo), _f64(hi), _f64(logw_in)
    n = x.shape[0]
    out = np.zeros(n)
    ncl = _load().yyo_propagate(ctypes.byref(model.c), len(s), _ptr(s), _ptr(c), n, _ptr(x),
                                _ptr(lo), _ptr(hi), float(dt), _ptr(lw), _ptr(out))
    return out, int(ncl)


def propagate_rows(model: OModel, s, c, x, lo, hi, dt, logw_in, rows):
    s, c, x, lo, hi, lw = _f64(s), _f64(c), _f64(x), _f64(lo), _f64(hi), _f64(logw_in)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n = x.shape[0]
    out = np.zeros(len(rows))
    ncl = _load().yyo_propagate_rows(ctypes.byref(model.c), len(s), _ptr(s), _ptr(c), n, _ptr(x),
                                     _ptr(lo), _ptr(hi), float(dt), _ptr(lw), len(rows), _ptr(rows),
                                     _ptr(out))
    return out, int(ncl)


def noise_pinv(U):
    """Sec. 7: a = U U^T, its eigen-decomposition a = Q diag(lam) Q^T, the pseudo-inverse
    a^+ = Q diag(1/lam_i for lam_i > 0, else 0) Q^T and log det_+ a = sum of log lam_i over the
    positive eigenvalues (those above PINV_RTOL times the largest).  Returns (a^+, log det_+ a, rank)."""
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    a = U @ U.T
    lam, Q = np.linalg.eigh(0.5 * (a + a.T))
    pos = lam > PINV_RTOL * max(float(lam.max()), 0.0)
    inv = np.zeros_like(lam)
    inv[pos] = 1.0 / lam[pos]
    return (Q * inv) @ Q.T, float(np.sum(np.log(lam[pos]))), int(pos.sum())


def divergence(model: OModel, x, mode: int = DIV_CLOSED, h: float = 1e-20) -> np.ndarray:
    x = _f64(np.atleast_2d(x))
    lib = _load()
    return np.array([lib.yyo_divergence(ctypes.byref(model.c), _ptr(np.ascontiguousarray(x[i])), int(mode),
                                        float(h)) for i in range(x.shape[0])])


def _kernel(form, div_mode, cs_step, apinv, logdet_a):
    ap = None if apinv is None else _f64(apinv)
    k = Kernel(int(form), int(div_mode), float(cs_step), _ptr(ap), float(logdet_a))
    return k, ap


def propagate_ex(model: OModel, s, c, x, lo, hi, dt, logw_in, form=FORM_PUSH, div_mode=DIV_CLOSED,
                 cs_step=1e-20, apinv=None, logdet_a=0.0):
    """The prediction with the pull form and/or general process noise (a^+, log det_+ a); returns
    (logw_out, nclamped)."""
    s, c, x, lo, hi, lw = _f64(s), _f64(c), _f64(x), _f64(lo), _f64(hi), _f64(logw_in)
    k, keep = _kernel(form, div_mode, cs_step, apinv, logdet_a)
    n = x.shape[0]
    out = np.zeros(n)
    ncl = _load().yyo_propagate_ex(ctypes.byref(model.c), ctypes.byref(k), len(s), _ptr(s), _ptr(c), n, _ptr(x),
                                   _ptr(lo), _ptr(hi), float(dt), _ptr(lw), _ptr(out))
    del keep
    return out, int(ncl)


def propagate_rows_ex(model: OModel, s, c, x, lo, hi, dt, logw_in, rows, form=FORM_PUSH, div_mode=DIV_CLOSED,
                      cs_step=1e-20, apinv=None, logdet_a=0.0):
    s, c, x, lo, hi, lw = _f64(s), _f64(c), _f64(x), _f64(lo), _f64(hi), _f64(logw_in)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    k, keep = _kernel(form, div_mode, cs_step, apinv, logdet_a)
    out = np.zeros(len(rows))
    ncl = _load().yyo_propagate_rows_ex(ctypes.byref(model.c), ctypes.byref(k), len(s), _ptr(s), _ptr(c),
                                        x.shape[0], _ptr(x), _ptr(lo), _ptr(hi), float(dt), _ptr(lw), len(rows),
                                        _ptr(rows), _ptr(out))
    del keep
    return out, int(ncl)


def loglik_update_ex(model: OModel, x, dy, dt, bpinv, logw) -> np.ndarray:
    x, dy, bp = _f64(x), _f64(dy), _f64(bpinv)
    lw = _f64(logw).copy()
    _load().yyo_loglik_update_ex(ctypes.byref(model.c), x.shape[0], _ptr(x), _ptr(dy), float(dt), _ptr(bp), _ptr(lw))
    return lw


def loglik_update(model: OModel, x, dy, dt, logw) -> np.ndarray:
    x, dy = _f64(x), _f64(dy)
    lw = _f64(logw).copy()
    _load().yyo_loglik_update(ctypes.byref(model.c), x.shape[0], _ptr(x), _ptr(dy), float(dt), _ptr(lw))
    return lw


def normalise_moments(x, logw, logZ_acc: float = 0.0, want_cov: bool = True):
    """Returns dict(logw, w, logZ_step, logZ_acc, mean, cov, ess, status)."""
    x = _f64(x)
    n, r = x.shape
    lw = _f64(logw).copy()
    w = np.zeros(n)
    mean = np.zeros(r)
    cov = np.zeros((r, r)) if want_cov else None
    lz = ctypes.c_double(0.0)
    acc = ctypes.c_double(logZ_acc)
    ess = ctypes.c_double(0.0)
    st = _load().yyo_normalise_moments(n, r, _ptr(x), _ptr(lw), _ptr(w), ctypes.byref(lz),
                                       ctypes.byref(acc), _ptr(mean), _ptr(cov), ctypes.byref(ess))
    return dict(logw=lw, w=w, logZ_step=lz.value, logZ_acc=acc.value, mean=mean, cov=cov,
                ess=ess.value, status=int(st))


def resample(w, seed: int, step: int) -> np.ndarray:
    w = _f64(w)
    idx = np.zeros(len(w), dtype=np.int64)
    rc = _load().yyo_resample(len(w), _ptr(w), seed & 0xFFFFFFFFFFFFFFFF, step, _ptr(idx))
    if rc != 0:
        raise ValueError("all resampling weights are zero")
    return idx


def restart_nodes(codes, mean, R):
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    n, r = codes.shape
    mean = _f64(mean)
    lo, hi = np.zeros(r), np.zeros(r)
    x = np.zeros((n, r))
    lw = np.zeros(n)
    _load().yyo_restart_nodes(n, r, _ptr(codes), _ptr(mean), float(R), _ptr(lo), _ptr(hi), _ptr(x), _ptr(lw))
    return lo, hi, x, lw
