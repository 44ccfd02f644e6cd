"""Helpers shared by the GPU parity tests: error measures and the
conditioning floor of the reference.

Errors are norm-wise: ||x - y|| / ||y|| for arrays (Frobenius for matrices),
|x - y| / max(|y|, 1) for scalars.  The floor is the disagreement of the
FP64 reference with itself when the N data points are presented in another
order (a mathematically identical problem); a GPU result is held to
max(bar, 10 x floor).
"""
import dataclasses

import numpy as np


def rel(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.ndim == 0 or x.size == 1:
        return float(abs(x.ravel()[0] - y.ravel()[0]) / max(abs(y.ravel()[0]), 1.0))
    n = np.linalg.norm(y)
    return float(np.linalg.norm(x - y) / (n if n > 0 else 1.0))


def permuted(spec, q, seed=123):
    """(spec', q', index map) with the data points in another order."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(spec.N)
    s2 = dataclasses.replace(spec, X=spec.X[p], y=spec.y[p])
    full = np.concatenate([p, spec.N + np.arange(spec.P)])
    q2 = q[full]
    return s2, q2, full


def unpermute_vec(v2, full):
    v = np.empty_like(v2)
    v[full] = v2
    return v


def unpermute_mat(M2, full):
    M = np.empty_like(M2)
    M[np.ix_(full, full)] = M2
    return M


def record(name, **vals):
    """Print one line of measured errors (kept in the pytest log)."""
    items = " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in vals.items())
    print(f"[parity] {name} {items}", flush=True)
