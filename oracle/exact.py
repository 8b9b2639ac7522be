"""Exact solutions used to measure error (paper Sec. 6.1).

Test infrastructure only (see oracle/__init__.py).

* Linear advection: u_a(x, t) = sum A sin(kappa (x - a t) + phi) (+ offset).
* Inviscid Burgers before the first shock: u(x, t) = u0(xi) with
  x = xi + u0(xi) t, solved for xi by Newton's method (method of
  characteristics; the paper's Burgers runs are viscous and use a fine
  reference solution instead, so this is our reading for the inviscid case).
"""
from __future__ import annotations

import numpy as np


def _u0(ic, x):
    u = np.full_like(np.asarray(x, dtype=np.float64), ic.offset)
    for k, a, ph in zip(ic.kappa, ic.amp, ic.phase):
        u = u + a * np.sin(k * x + ph)
    return u


def _du0(ic, x):
    d = np.zeros_like(np.asarray(x, dtype=np.float64))
    for k, a, ph in zip(ic.kappa, ic.amp, ic.phase):
        d = d + a * k * np.cos(k * x + ph)
    return d


def advection(w, x: np.ndarray, t: float) -> np.ndarray:
    return _u0(w.ic, x - w.speed * t)


def burgers(w, x: np.ndarray, t: float, iters: int = 60) -> np.ndarray:
    """Pre-shock solution; requires 1 + u0'(xi) t > 0 everywhere."""
    xi = np.array(x, dtype=np.float64, copy=True) - _u0(w.ic, x) * t
    for _ in range(iters):
        g = xi + _u0(w.ic, xi) * t - x
        dg = 1.0 + _du0(w.ic, xi) * t
        if np.any(dg <= 0):
            raise ValueError("characteristics crossed: shock has formed")
        step = g / dg
        xi = xi - step
        if np.max(np.abs(step)) < 1e-15 * (1 + np.max(np.abs(x))):
            break
    return _u0(w.ic, xi)


def solution(w, x: np.ndarray, t: float) -> np.ndarray:
    return advection(w, x, t) if w.equation == "advection" else burgers(w, x, t)
