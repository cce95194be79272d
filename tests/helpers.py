"""Shared test helpers (no method arithmetic)."""
import numpy as np


def relerr(y, o):
    """Normwise relative error max|y - o| / max|o| over a whole output array.

    Elementwise relative error is undefined at structural zeros (e.g. cross-axis entries of S), so
    every tolerance in the suite is stated in this normwise form.
    """
    y = np.asarray(y, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    scale = np.max(np.abs(o))
    if scale == 0.0:
        return float(np.max(np.abs(y)))
    return float(np.max(np.abs(y - o)) / scale)


def random_psd(rng, n, rank=None, scale=1.0):
    k = n if rank is None else rank
    X = rng.standard_normal((n, k))
    return scale * (X @ X.T) / max(k, 1)


def random_tuple(rng, nx, scale=1.0):
    A = np.eye(nx) + 0.3 * rng.standard_normal((nx, nx))
    b = rng.standard_normal(nx)
    C = random_psd(rng, nx, scale=scale)
    eta = rng.standard_normal(nx)
    J = random_psd(rng, nx, scale=scale)
    return A, b, C, eta, J
