"""Python binding of libyy (the C ABI in include/yy.h) -- argument marshalling only.

Each ``yy_*`` function here calls the C function of the same name: tensors are
passed as device pointers (torch supplies device memory and streams, nothing
else), scalars and small host arrays are converted to C types, and a non-OK
status raises ``YYError`` with the library's error text.  Every step of the
filter runs in the library's HIP kernels.  There is no fallback: if libyy.so
is missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libyy.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"libyy.so not found at {LIB_PATH}; build it with paper_2509_16896_amd/build.py")
_lib = ctypes.CDLL(LIB_PATH)

YY_OK, YY_ERR_ARG, YY_ERR_ALLOC, YY_ERR_HIP, YY_ERR_NUMERIC, YY_ERR_UNSUPPORTED = range(6)
YY_FLAG_ALL_ZERO, YY_FLAG_CLAMPED, YY_FLAG_RESAMPLE_ZERO, YY_FLAG_LOW_ESS = 1, 2, 4, 8
YY_F_ZERO, YY_F_COS, YY_F_LINEAR, YY_F_PAPER_SINMIX = 0, 1, 2, 3
YY_H_IDENTITY, YY_H_CUBE, YY_H_LINEAR = 0, 1, 2
(YY_PREC_AUTO, YY_PREC_FP32, YY_PREC_FP32_MFMA, YY_PREC_BF16X3, YY_PREC_BF16X1, YY_PREC_BF16X3G, YY_PREC_BF16X3S,
 YY_PREC_BF16X3P) = 0, 1, 2, 3, 4, 5, 6, 7
PREC_BY_NAME = {"auto": YY_PREC_AUTO, "fp32": YY_PREC_FP32, "fp32_mfma": YY_PREC_FP32_MFMA,
                "bf16x3": YY_PREC_BF16X3, "bf16x1": YY_PREC_BF16X1,
                "bf16x3g": YY_PREC_BF16X3G, "bf16x3s": YY_PREC_BF16X3S, "bf16x3p": YY_PREC_BF16X3P}
EXPORTED = ["yy_last_error", "yy_create", "yy_destroy", "yy_set_stream", "yy_get_status",
            "yy_kernel_coefficients", "yy_nodes_sobol", "yy_propagate", "yy_loglik_update",
            "yy_normalise_moments", "yy_normalise_moments_noalloc", "yy_loglik_normalise",
            "yy_noise_create", "yy_noise_destroy", "yy_noise_info",
            "yy_operator_build", "yy_operator_apply", "yy_operator_info", "yy_operator_destroy", "yy_restart", "yy_timing_enable", "yy_timing_read", "yy_screen_count",
            "yy_proposal_create", "yy_proposal_destroy", "yy_proposal_num_params", "yy_proposal_get_params",
            "yy_proposal_set_params", "yy_proposal_forward", "yy_proposal_train_step", "yy_sample_moments",
            "yy_tune", "yy_batch_create", "yy_batch_destroy", "yy_batch_reset", "yy_batch_step",
            "yy_batch_run_graph", "yy_batch_tune", "yy_batch_results", "yy_batch_step_count",
            "yy_batch_screen_count", "yy_batch_run_form", "yy_batch_set_run_form"]


class YYError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        text = _lib.yy_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {text}")


class yy_model(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("m", ctypes.c_int32), ("drift", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("obs", ctypes.c_int32), ("H", ctypes.c_void_p),
                ("h_shift", ctypes.c_double), ("q", ctypes.c_double), ("rho2", ctypes.c_double),
                ("noise", ctypes.c_void_p)]


class yy_scales(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("s", ctypes.POINTER(ctypes.c_double)),
                ("c", ctypes.POINTER(ctypes.c_double)), ("form", ctypes.c_int32), ("div", ctypes.c_int32)]


class yy_restart_params(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("ess_min", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("proposal", ctypes.c_void_p), ("cover_min", ctypes.c_double)]


class yy_batch_run(ctypes.Structure):
    _fields_ = [("model", yy_model), ("n", ctypes.c_int64), ("dt", ctypes.c_double), ("box_half", ctypes.c_double),
                ("R", ctypes.c_double), ("restart_every", ctypes.c_int32), ("K", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("dys", ctypes.c_void_p)]


_P, _i32, _i64, _u64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
_lib.yy_last_error.restype = ctypes.c_char_p
_lib.yy_last_error.argtypes = []
for _name, _args in {
    "yy_create": [ctypes.POINTER(_P), ctypes.c_int, _P],
    "yy_destroy": [_P],
    "yy_set_stream": [_P, _P],
    "yy_get_status": [_P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_i64)],
    "yy_kernel_coefficients": [_i32, ctypes.POINTER(_f64), ctypes.POINTER(_f64)],
    "yy_nodes_sobol": [_P, _i32, _i64, _i64, _i32, _u64, _P, _P, _P, _P],
    "yy_propagate": [_P, ctypes.POINTER(yy_model), ctypes.POINTER(yy_scales), _i32, _i64, _P, _u64,
                     _P, _P, _f64, _P, _P],
    "yy_loglik_update": [_P, ctypes.POINTER(yy_model), _i64, _P, _P, _f64, _P],
    "yy_normalise_moments": [_P, _i64, _i32, _P, _P, _P, _P, _P, _P, _P, _P],
    "yy_normalise_moments_noalloc": [_P, _i64, _i32, _P, _P, _P, _P, _P, _P, _P, _P],
    "yy_noise_create": [_P, _i32, _P, _i32, _P, ctypes.POINTER(_P)],
    "yy_operator_build": [_P, ctypes.POINTER(yy_model), ctypes.POINTER(yy_scales), _i64, _P, _u64, _P, _P, _f64,
                          ctypes.POINTER(_P)],
    "yy_operator_apply": [_P, _P, _P],
    "yy_operator_info": [_P, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i64)],
    "yy_operator_destroy": [_P],
    "yy_noise_destroy": [_P],
    "yy_noise_info": [_P, ctypes.POINTER(_i32), ctypes.POINTER(_f64), ctypes.POINTER(_i32), ctypes.POINTER(_f64)],
    "yy_loglik_normalise": [_P, ctypes.POINTER(yy_model), _i64, _P, _P, _f64, _P, _P, _P, _P, _P, _P],
    "yy_restart": [_P, _i64, _i32, _P, _P, _P, _P, _P, _i64, ctypes.POINTER(yy_restart_params), _P, _P,
                   _P, _P, _P, _P],
    "yy_proposal_create": [_P, _i32, _i32, _u64, _P, ctypes.POINTER(_P)],
    "yy_proposal_destroy": [_P],
    "yy_proposal_num_params": [_P, ctypes.POINTER(_i64)],
    "yy_proposal_get_params": [_P, _P],
    "yy_proposal_set_params": [_P, _P],
    "yy_proposal_forward": [_P, _i32, _P, _P],
    "yy_proposal_train_step": [_P, _i32, _P, _P, _P, _f64, _f64, _i32, _P, _P],
    "yy_sample_moments": [_P, _i64, _i32, _P, _P, _P, _P],
    "yy_tune": [_P, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(yy_scales), _i32, _i32,
                ctypes.POINTER(_i32)],
    "yy_batch_create": [_P, _i32, ctypes.POINTER(yy_batch_run), ctypes.POINTER(yy_scales), _i32, _i32,
                        ctypes.POINTER(_P)],
    "yy_batch_destroy": [_P],
    "yy_batch_reset": [_P],
    "yy_batch_step": [_P],
    "yy_batch_run_graph": [_P, _i32],
    "yy_batch_tune": [_P, _i32, _i32, ctypes.POINTER(_i32)],
    "yy_batch_results": [_P, _i32, _P, _P, _P],
    "yy_batch_step_count": [_P, ctypes.POINTER(_i32)],
    "yy_batch_screen_count": [_P, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "yy_batch_run_form": [_P, _i32, ctypes.POINTER(_i32)],
    "yy_batch_set_run_form": [_P, _i32, _i32],
    "yy_timing_enable": [_P, _i32],
    "yy_timing_read": [_P, ctypes.POINTER(_f64), ctypes.POINTER(_i64)],
    "yy_screen_count": [_P, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
}.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = ctypes.c_int


def _check(status: int, where: str):
    if status != YY_OK:
        raise YYError(status, where)


def _dptr(t, dtype=None, numel=None, name="array"):
    """Device pointer of a contiguous CUDA/HIP tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype and not (dtype == torch.uint32 and t.dtype == torch.int32):
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Model:
    """Host description of yy_model; keeps A/H device tensors alive."""

    def __init__(self, r, m=None, drift=YY_F_COS, A=None, obs=YY_H_CUBE, H=None, h_shift=0.0, q=1.0,
                 rho2=1.0, device="cuda", noise=None):
        self.A = None if A is None else torch.as_tensor(A, dtype=torch.float64, device=device).contiguous()
        self.H = None if H is None else torch.as_tensor(H, dtype=torch.float64, device=device).contiguous()
        m = int(m if m is not None else (self.H.shape[0] if self.H is not None else r))
        self.noise = noise     # a yy_noise handle (yy_noise_create), kept alive by the caller
        self.c = yy_model(int(r), m, int(drift), None if self.A is None else self.A.data_ptr(), int(obs),
                          None if self.H is None else self.H.data_ptr(), float(h_shift), float(q), float(rho2),
                          noise)

    @property
    def r(self):
        return self.c.r

    @property
    def m(self):
        return self.c.m


YY_FORM_PUSH, YY_FORM_PULL = 0, 1
YY_DIV_CLOSED, YY_DIV_COMPLEX_STEP = 0, 1
FORM_BY_NAME = {"push": YY_FORM_PUSH, "pull": YY_FORM_PULL}


class Scales:
    """The kernel operator: scale divisors, optional coefficients, the first-order kernel's form
    ("push" or "pull") and, for the pull form, how the divergence is evaluated."""

    def __init__(self, s, c=None, form="push", div=YY_DIV_CLOSED):
        self._s = (ctypes.c_double * len(s))(*[float(v) for v in s])
        self._c = None if c is None else (ctypes.c_double * (len(s) + 1))(*[float(v) for v in c])
        self.c = yy_scales(len(s), self._s, self._c, FORM_BY_NAME.get(form, form), int(div))


def yy_kernel_coefficients(s) -> list:
    S = len(s)
    sa = (ctypes.c_double * S)(*[float(v) for v in s])
    ca = (ctypes.c_double * (S + 1))()
    _check(_lib.yy_kernel_coefficients(S, sa, ca), "yy_kernel_coefficients")
    return list(ca)


def yy_create(device: int = 0, stream=None):
    ctx = ctypes.c_void_p()
    _check(_lib.yy_create(ctypes.byref(ctx), int(device), _stream_handle(stream)), "yy_create")
    return ctx


def yy_destroy(ctx):
    _check(_lib.yy_destroy(ctx), "yy_destroy")


def yy_set_stream(ctx, stream=None):
    _check(_lib.yy_set_stream(ctx, _stream_handle(stream)), "yy_set_stream")


def yy_get_status(ctx):
    flags = ctypes.c_uint32(0)
    ncl = ctypes.c_int64(0)
    _check(_lib.yy_get_status(ctx, ctypes.byref(flags), ctypes.byref(ncl)), "yy_get_status")
    return int(flags.value), int(ncl.value)


def yy_nodes_sobol(ctx, r, n, first_index, scramble, seed, box_lo, box_hi, codes=None, x=None):
    _check(_lib.yy_nodes_sobol(ctx, int(r), int(n), int(first_index), int(bool(scramble)),
                               int(seed) & 0xFFFFFFFFFFFFFFFF,
                               _dptr(box_lo, torch.float64, r, "box_lo"), _dptr(box_hi, torch.float64, r, "box_hi"),
                               _dptr(codes, torch.uint32, n * r, "codes"), _dptr(x, torch.float64, n * r, "x")),
           "yy_nodes_sobol")


def yy_propagate(ctx, model: Model, scales: Scales, prec, n, x, node_version, box_lo, box_hi, dt,
                 logw_in, logw_out):
    prec = PREC_BY_NAME[prec] if isinstance(prec, str) else int(prec)
    r = model.r
    _check(_lib.yy_propagate(ctx, ctypes.byref(model.c), ctypes.byref(scales.c), prec, int(n),
                             _dptr(x, torch.float64, n * r, "x"), int(node_version) & 0xFFFFFFFFFFFFFFFF,
                             _dptr(box_lo, torch.float64, r, "box_lo"), _dptr(box_hi, torch.float64, r, "box_hi"),
                             float(dt), _dptr(logw_in, torch.float64, n, "logw_in"),
                             _dptr(logw_out, torch.float64, n, "logw_out")), "yy_propagate")


def yy_loglik_update(ctx, model: Model, n, x, dy, dt, logw):
    _check(_lib.yy_loglik_update(ctx, ctypes.byref(model.c), int(n), _dptr(x, torch.float64, n * model.r, "x"),
                                 _dptr(dy, torch.float64, model.m, "dy"), float(dt),
                                 _dptr(logw, torch.float64, n, "logw")), "yy_loglik_update")


def yy_loglik_normalise(ctx, model: Model, n, x, dy, dt, logw, w, logZ_step, logZ_acc, mean, ess):
    _check(_lib.yy_loglik_normalise(ctx, ctypes.byref(model.c), int(n), _dptr(x, torch.float64, n * model.r, "x"),
                                    _dptr(dy, torch.float64, model.m, "dy"), float(dt),
                                    _dptr(logw, torch.float64, n, "logw"), _dptr(w, torch.float64, n, "w"),
                                    _dptr(logZ_step, torch.float64, 1, "logZ_step"),
                                    _dptr(logZ_acc, torch.float64, 1, "logZ_acc"),
                                    _dptr(mean, torch.float64, model.r, "mean"),
                                    _dptr(ess, torch.float64, 1, "ess")), "yy_loglik_normalise")


def yy_normalise_moments(ctx, n, r, x, logw, w, logZ_step, logZ_acc, mean, cov, ess):
    _check(_lib.yy_normalise_moments(ctx, int(n), int(r), _dptr(x, torch.float64, n * r, "x"),
                                     _dptr(logw, torch.float64, n, "logw"), _dptr(w, torch.float64, n, "w"),
                                     _dptr(logZ_step, torch.float64, 1, "logZ_step"),
                                     _dptr(logZ_acc, torch.float64, 1, "logZ_acc"),
                                     _dptr(mean, torch.float64, r, "mean"), _dptr(cov, torch.float64, r * r, "cov"),
                                     _dptr(ess, torch.float64, 1, "ess")), "yy_normalise_moments")


def yy_noise_create(ctx, r, U=None, m=None, V=None):
    """General noise coefficients a = U U^T (r x r) and/or b = V V^T (m x m), host arrays; returns a handle."""
    import numpy as np
    m = r if m is None else m
    Ua = None if U is None else np.ascontiguousarray(U, dtype=np.float64).reshape(r, r)
    Va = None if V is None else np.ascontiguousarray(V, dtype=np.float64).reshape(m, m)
    out = ctypes.c_void_p()
    _check(_lib.yy_noise_create(ctx, int(r), None if Ua is None else Ua.ctypes.data_as(ctypes.c_void_p), int(m),
                                None if Va is None else Va.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)),
           "yy_noise_create")
    return out


def yy_noise_destroy(noise):
    _check(_lib.yy_noise_destroy(noise), "yy_noise_destroy")


def yy_noise_info(noise):
    ra, rb = ctypes.c_int32(), ctypes.c_int32()
    la, lb = ctypes.c_double(), ctypes.c_double()
    _check(_lib.yy_noise_info(noise, ctypes.byref(ra), ctypes.byref(la), ctypes.byref(rb), ctypes.byref(lb)),
           "yy_noise_info")
    return ra.value, la.value, rb.value, lb.value


def yy_operator_build(ctx, model, scales, n, x, node_version, box_lo, box_hi, dt, op=None):
    """Builds (or, given op, rebuilds in place) the stored operator; returns the handle."""
    h = op if op is not None else ctypes.c_void_p()
    r = model.r
    _check(_lib.yy_operator_build(ctx, ctypes.byref(model.c), ctypes.byref(scales.c), int(n),
                                  _dptr(x, torch.float64, n * r, "x"), int(node_version) & 0xFFFFFFFFFFFFFFFF,
                                  _dptr(box_lo, torch.float64, r, "box_lo"), _dptr(box_hi, torch.float64, r, "box_hi"),
                                  float(dt), ctypes.byref(h)), "yy_operator_build")
    return h


def yy_operator_apply(op, logw_in, logw_out):
    n = ctypes.c_int64()
    _check(_lib.yy_operator_info(op, ctypes.byref(n), None, None), "yy_operator_info")
    _check(_lib.yy_operator_apply(op, _dptr(logw_in, torch.float64, n.value, "logw_in"),
                                  _dptr(logw_out, torch.float64, n.value, "logw_out")), "yy_operator_apply")


def yy_operator_info(op):
    n, S, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.yy_operator_info(op, ctypes.byref(n), ctypes.byref(S), ctypes.byref(b)), "yy_operator_info")
    return n.value, S.value, b.value


def yy_operator_destroy(op):
    _check(_lib.yy_operator_destroy(op), "yy_operator_destroy")


def yy_normalise_moments_noalloc(ctx, n, r, x, logw, w, logZ_step, logZ_acc, mean, cov, ess):
    _check(_lib.yy_normalise_moments_noalloc(
        ctx, int(n), int(r), _dptr(x, torch.float64, n * r, "x"), _dptr(logw, torch.float64, n, "logw"),
        _dptr(w, torch.float64, n, "w"), _dptr(logZ_step, torch.float64, 1, "logZ_step"),
        _dptr(logZ_acc, torch.float64, 1, "logZ_acc"), _dptr(mean, torch.float64, r, "mean"),
        _dptr(cov, torch.float64, r * r, "cov"), _dptr(ess, torch.float64, 1, "ess")),
        "yy_normalise_moments_noalloc")


def yy_restart(ctx, n, r, codes, x_cur, w, mean, ess, step, R, ess_min, seed, idx, box_lo, box_hi, x_new,
               logw_new, proposal=None, cover_min=0.95, used=None):
    params = yy_restart_params(float(R), float(ess_min), int(seed) & 0xFFFFFFFFFFFFFFFF, proposal,
                               float(cover_min))
    _check(_lib.yy_restart(ctx, int(n), int(r), _dptr(codes, torch.uint32, n * r, "codes"),
                           _dptr(x_cur, torch.float64, n * r, "x_cur"),
                           _dptr(w, torch.float64, n, "w"), _dptr(mean, torch.float64, r, "mean"),
                           _dptr(ess, torch.float64, 1, "ess"), int(step), ctypes.byref(params),
                           _dptr(idx, torch.int64, n, "idx"), _dptr(box_lo, torch.float64, r, "box_lo"),
                           _dptr(box_hi, torch.float64, r, "box_hi"), _dptr(x_new, torch.float64, n * r, "x_new"),
                           _dptr(logw_new, torch.float64, n, "logw_new"), _dptr(used, torch.int32, 1, "used")),
           "yy_restart")


def proposal_num_params(r: int, hidden: int) -> int:
    """P = H r + H + H^2 + H + 2 r H + 2 r (the layout of include/yy.h)."""
    return hidden * r + hidden + hidden * hidden + hidden + 2 * r * hidden + 2 * r


def yy_proposal_create(ctx, r, hidden=256, seed=0, params=None):
    out = ctypes.c_void_p()
    if params is not None and params.numel() != proposal_num_params(r, hidden):
        raise ValueError(f"params has {params.numel()} elements, the network needs {proposal_num_params(r, hidden)}")
    _check(_lib.yy_proposal_create(ctx, int(r), int(hidden), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                   _dptr(params, torch.float32, None, "params"), ctypes.byref(out)),
           "yy_proposal_create")
    return out


def yy_proposal_destroy(p):
    _check(_lib.yy_proposal_destroy(p), "yy_proposal_destroy")


def yy_proposal_num_params(p) -> int:
    P = ctypes.c_int64(0)
    _check(_lib.yy_proposal_num_params(p, ctypes.byref(P)), "yy_proposal_num_params")
    return int(P.value)


def yy_proposal_get_params(p, params):
    _check(_lib.yy_proposal_get_params(p, _dptr(params, torch.float32, yy_proposal_num_params(p), "params")),
           "yy_proposal_get_params")


def yy_proposal_set_params(p, params):
    _check(_lib.yy_proposal_set_params(p, _dptr(params, torch.float32, yy_proposal_num_params(p), "params")),
           "yy_proposal_set_params")


def yy_proposal_forward(p, B, xhat, out, r):
    _check(_lib.yy_proposal_forward(p, int(B), _dptr(xhat, torch.float64, B * r, "xhat"),
                                    _dptr(out, torch.float32, B * 2 * r, "out")), "yy_proposal_forward")


def yy_proposal_train_step(p, B, xhat, mu, var, R, lr, update, loss=None, grad=None, r=None):
    r = xhat.numel() // B if r is None else r
    _check(_lib.yy_proposal_train_step(p, int(B), _dptr(xhat, torch.float64, B * r, "xhat"),
                                       _dptr(mu, torch.float64, B * r, "mu"), _dptr(var, torch.float64, B * r, "var"),
                                       float(R), float(lr), int(bool(update)),
                                       _dptr(loss, torch.float64, 1, "loss"), _dptr(grad, torch.float32, None, "grad")),
           "yy_proposal_train_step")


def yy_sample_moments(ctx, n, r, x, idx, mean, var):
    _check(_lib.yy_sample_moments(ctx, int(n), int(r), _dptr(x, torch.float64, n * r, "x"),
                                  _dptr(idx, torch.int64, n, "idx"), _dptr(mean, torch.float64, r, "mean"),
                                  _dptr(var, torch.float64, r, "var")), "yy_sample_moments")


def yy_timing_enable(ctx, on: bool = True):
    _check(_lib.yy_timing_enable(ctx, int(bool(on))), "yy_timing_enable")


def yy_timing_read(ctx):
    """Returns (total pairwise-kernel milliseconds, number of timed launches) and resets them."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(_lib.yy_timing_read(ctx, ctypes.byref(ms), ctypes.byref(cnt)), "yy_timing_read")
    return float(ms.value), int(cnt.value)


def yy_screen_count(ctx):
    """(flagged tiles, tiles) of the last BF16X3S or BF16X3P propagation on ctx."""
    fl = ctypes.c_int64(0)
    t = ctypes.c_int64(0)
    _check(_lib.yy_screen_count(ctx, ctypes.byref(fl), ctypes.byref(t)), "yy_screen_count")
    return int(fl.value), int(t.value)


def yy_tune(ctx, shapes, scales: Scales, prec, reps=3):
    """Tunes the matrix-core kernel's source splits for each (r, n); returns the chosen counts."""
    prec = PREC_BY_NAME[prec] if isinstance(prec, str) else int(prec)
    cnt = len(shapes)
    ra = (_i32 * cnt)(*[int(r) for r, _ in shapes])
    na = (_i64 * cnt)(*[int(n) for _, n in shapes])
    out = (_i32 * cnt)()
    _check(_lib.yy_tune(ctx, cnt, ra, na, ctypes.byref(scales.c), prec, int(reps), out), "yy_tune")
    return list(out)


def yy_batch_create(ctx, runs, scales: Scales, prec, max_split=0):
    """runs: list of (Model, n, dt, box_half, R, restart_every, K, seed, dys device tensor [K*m])."""
    prec = PREC_BY_NAME[prec] if isinstance(prec, str) else int(prec)
    arr = (yy_batch_run * len(runs))()
    for t, (model, n, dt, box_half, R, every, K, seed, dys) in enumerate(runs):
        arr[t] = yy_batch_run(model.c, int(n), float(dt), float(box_half), float(R), int(every), int(K),
                              int(seed) & 0xFFFFFFFFFFFFFFFF, _dptr(dys, torch.float64, K * model.m, "dys"))
    out = ctypes.c_void_p()
    _check(_lib.yy_batch_create(ctx, len(runs), arr, ctypes.byref(scales.c), prec, int(max_split),
                                ctypes.byref(out)), "yy_batch_create")
    return out


def yy_batch_destroy(b):
    _check(_lib.yy_batch_destroy(b), "yy_batch_destroy")


def yy_batch_reset(b):
    _check(_lib.yy_batch_reset(b), "yy_batch_reset")


def yy_batch_step(b):
    _check(_lib.yy_batch_step(b), "yy_batch_step")


def yy_batch_run_graph(b, k_end):
    _check(_lib.yy_batch_run_graph(b, int(k_end)), "yy_batch_run_graph")


def yy_batch_tune(b, reps=3, forms=0) -> int:
    """forms: bit 0 the vector-ALU form, bit 1 (BF16X3P batches) the split form on every tile."""
    best = _i32(0)
    _check(_lib.yy_batch_tune(b, int(reps), int(forms), ctypes.byref(best)), "yy_batch_tune")
    return int(best.value)


def yy_batch_results(b, run, mean_hist=None, logZ_hist=None, ess_hist=None):
    _check(_lib.yy_batch_results(b, int(run), _dptr(mean_hist, torch.float64, None, "mean_hist"),
                                 _dptr(logZ_hist, torch.float64, None, "logZ_hist"),
                                 _dptr(ess_hist, torch.float64, None, "ess_hist")), "yy_batch_results")


def yy_batch_screen_count(b, run):
    """(flagged tiles, tiles) of the last propagation of run `run` of a batch in a screened form."""
    f, t = _i64(0), _i64(0)
    _check(_lib.yy_batch_screen_count(b, int(run), ctypes.byref(f), ctypes.byref(t)), "yy_batch_screen_count")
    return int(f.value), int(t.value)


def yy_batch_run_form(b, run) -> str:
    """Run `run`'s pairwise form: the batch's matrix-core form, "fp32" (vector ALUs) or, in a
    BF16X3P batch, "bf16x3g" (the split form on every tile, no screen)."""
    p = _i32(0)
    _check(_lib.yy_batch_run_form(b, int(run), ctypes.byref(p)), "yy_batch_run_form")
    return {v: k for k, v in PREC_BY_NAME.items() if k != "auto"}[int(p.value)]


def yy_batch_set_run_form(b, run, prec: str):
    _check(_lib.yy_batch_set_run_form(b, int(run), PREC_BY_NAME[prec]), "yy_batch_set_run_form")


def yy_batch_step_count(b) -> int:
    k = _i32(0)
    _check(_lib.yy_batch_step_count(b, ctypes.byref(k)), "yy_batch_step_count")
    return int(k.value)
