"""Helpers shared by the GPU tests: device tensors, unique node versions and the
log-density comparison used for parity."""
import itertools

import numpy as np
import torch
from scipy.special import logsumexp

_versions = itertools.count(1000)


def next_version() -> int:
    return next(_versions)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def compare_logw(got, ref, tol, weight_floor=1e-12):
    """Parity of log-densities on the nodes that carry weight.

    Both vectors are normalised (shift-invariant comparison); on nodes whose
    oracle weight is at least `weight_floor` the error must satisfy
    |d| <= tol * max(1, |normalised log-density|).  Returns the worst ratio
    err / allowed and the number of compared nodes."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fr = np.isfinite(ref)
    assert fr.any(), "oracle produced no finite log-density"
    rn = ref - logsumexp(ref[fr])
    sel = fr & (rn >= np.log(weight_floor))
    assert np.all(np.isfinite(got[sel])), "GPU produced -inf where the oracle has weight"
    gn = got - logsumexp(got[np.isfinite(got)])
    allowed = tol * np.maximum(1.0, np.abs(rn[sel]))
    worst = float(np.max(np.abs(gn[sel] - rn[sel]) / allowed))
    return worst, int(sel.sum())
