"""Error norms and ensemble statistics (paper Sec. 4.3 spatial and ensemble
averages; Sec. 6.2 error as the mean absolute pointwise error).

Test infrastructure only (see oracle/__init__.py).  All sums use math.fsum so
the result is the correctly rounded sum, independent of order.
"""
from __future__ import annotations

import math

import numpy as np


def mean_abs(u: np.ndarray, ref: np.ndarray) -> float:
    """<E> = (1/N) sum |u - u_ref| over all nodal values."""
    d = np.abs(np.asarray(u) - np.asarray(ref)).ravel()
    return math.fsum(d.tolist()) / d.size


def max_abs(u: np.ndarray, ref: np.ndarray) -> float:
    return float(np.max(np.abs(np.asarray(u) - np.asarray(ref))))


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 over all entries."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    num = math.fsum(((a - b) ** 2).tolist())
    den = math.fsum((b ** 2).tolist())
    return math.sqrt(num / den) if den > 0 else math.sqrt(num)


def ensemble_mean_var(values) -> tuple:
    """Ensemble average (overbar) and population variance over realizations."""
    v = [float(x) for x in values]
    n = len(v)
    mean = math.fsum(v) / n
    var = math.fsum([(x - mean) ** 2 for x in v]) / n
    return mean, var
