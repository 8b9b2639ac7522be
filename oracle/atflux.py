"""Asynchrony-tolerant flux coefficients (paper Sec. 5, Eq. for the general AT
flux, the moment constraints, the fourth-order example and Table 1).

Test infrastructure only (see oracle/__init__.py).

The AT flux at a PE boundary is a linear combination of standard fluxes from
the q time levels n-k, ..., n-k-q+1 (L1 = k, L2 = k+q-1).  The coefficients
c^l make the Taylor expansion about level n reproduce the level-n flux up to
order q: sum_l c^l (-l dt)^z / z! = 1 for z = 0 and 0 for 0 < z < q.  The dt^z/z!
factors are common to each row, so the system is solved with exact rational
arithmetic on the integer Vandermonde rows (-l)^z.

q = (N_p + 1)/r with r = 1 for advection (Sec. 5).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List


def _solve_exact(a: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    """Gauss-Jordan elimination over the rationals."""
    n = len(b)
    m = [row[:] + [b[i]] for i, row in enumerate(a)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        inv = 1 / m[col][col]
        m[col] = [v * inv for v in m[col]]
        for r in range(n):
            if r != col and m[r][col] != 0:
                f = m[r][col]
                m[r] = [vr - f * vc for vr, vc in zip(m[r], m[col])]
    return [m[i][n] for i in range(n)]


def at_coefficients_exact(q: int, k: int) -> List[Fraction]:
    """c^{k+j}, j = 0..q-1, for delay k and q levels (moment constraints)."""
    if q < 1 or k < 0:
        raise ValueError("q >= 1 and k >= 0 required")
    levels = [k + j for j in range(q)]
    a = [[Fraction(-l) ** z for l in levels] for z in range(q)]
    b = [Fraction(1)] + [Fraction(0)] * (q - 1)
    return _solve_exact(a, b)


def at_coefficients(q: int, k: int) -> List[float]:
    """Same coefficients as floats (they are integers, so exact in FP64)."""
    return [float(c) for c in at_coefficients_exact(q, k)]
