"""Pins for the AT-flux coefficients (paper Sec. 5, Table 1 and the
fourth-order example)."""
import json
import os
from fractions import Fraction

import pytest

from oracle import atflux

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "at_table1.json")))


def _poly(entry, k):
    return Fraction(sum(c * k ** i for i, c in enumerate(entry["num"])), entry["den"])


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("k", [0, 1, 2, 3, 5])
def test_table1(order, k):
    printed = [_poly(e, k) for e in GOLD[f"order_{order}"]]
    assert atflux.at_coefficients_exact(order, k) == printed


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_consistency_and_reduction(q, k):
    c = atflux.at_coefficients_exact(q, k)
    assert sum(c) == 1
    if k == 0:   # reduces to the standard flux (Sec. 5)
        assert c == [1] + [0] * (q - 1)
    # Lagrange extrapolation to t_n from t_{n-k-j} reproduces polynomials of
    # degree < q exactly: sum_j c_j g(-(k+j)) = g(0)
    for deg in range(q):
        g = lambda t: (t + 3) ** deg
        assert sum(cj * g(-(k + j)) for j, cj in enumerate(c)) == g(0)


def test_integer_valued():
    for q in range(1, 6):
        for k in range(8):
            for c in atflux.at_coefficients_exact(q, k):
                assert c.denominator == 1
