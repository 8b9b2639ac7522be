"""Pins of oracle/stats.py: the spatial average <E> and the ensemble average
(overbar) of Sec. 4.3, with the error measured at every nodal point as in
Sec. 6.2, checked against values computed by hand on small integer arrays.

Each case is chosen so that a plausible mistake gives a different number:
dividing by the number of elements instead of the number of nodal values,
the sample (n - 1) instead of the population (n) variance, a naive
left-to-right sum instead of the correctly rounded one, a signed instead of
an absolute difference, a swapped reference in the relative norm."""
import math

import numpy as np
import pytest

from oracle import stats


def test_mean_abs_divides_by_nodal_values_not_elements():
    # 2 elements x 3 nodes; |u - ref| = 1, 2, 3, 4, 5, 6 -> sum 21 over 6 values.
    u = np.array([[1.0, -2.0, 3.0], [4.0, 5.0, -6.0]])
    ref = np.zeros_like(u)
    assert stats.mean_abs(u, ref) == 21.0 / 6.0
    assert stats.mean_abs(u, ref) != 21.0 / 2.0  # per-element divisor


def test_mean_abs_takes_absolute_differences():
    u = np.array([[2.0, 0.0], [5.0, 1.0]])
    ref = np.array([[3.0, 2.0], [1.0, 1.0]])  # differences -1, -2, 4, 0
    assert stats.mean_abs(u, ref) == 7.0 / 4.0   # the signed mean would be 1/4


def test_mean_abs_is_correctly_rounded():
    # 1e16 + 1 + 1: a left-to-right double sum gives 1e16 (each +1 rounds away),
    # the exact sum 1e16 + 2 is representable.
    u = np.array([1e16, 1.0, 1.0])
    assert stats.mean_abs(u, np.zeros(3)) == (1e16 + 2.0) / 3.0
    assert (1e16 + 1.0) + 1.0 == 1e16


def test_max_abs():
    u = np.array([[1.0, -7.0], [3.0, 2.0]])
    ref = np.array([[0.0, 0.0], [-3.0, 2.0]])
    assert stats.max_abs(u, ref) == 7.0


def test_rel_l2_hand_values():
    # ||a - b|| = ||(3, 4)|| = 5, ||b|| = ||(0, 5)|| = 5
    assert stats.rel_l2(np.array([3.0, 9.0]), np.array([0.0, 5.0])) == 1.0
    # the reference is the second argument: ||(3, 4)|| / ||(3, 9)|| = 5 / sqrt(90)
    assert stats.rel_l2(np.array([0.0, 5.0]), np.array([3.0, 9.0])) == pytest.approx(5.0 / math.sqrt(90.0), 1e-15)
    assert stats.rel_l2(np.ones(4), np.ones(4)) == 0.0


def test_ensemble_mean_and_population_variance():
    mean, var = stats.ensemble_mean_var([1, 2, 3, 4])
    assert mean == 2.5
    assert var == 1.25            # population: 5 / 4
    assert var != 5.0 / 3.0       # sample: 5 / 3


def test_ensemble_single_and_constant_members():
    assert stats.ensemble_mean_var([7.0]) == (7.0, 0.0)
    # the correctly rounded sum of ten 0.1 is 1.0, so the mean is 0.1 exactly
    assert stats.ensemble_mean_var([0.1] * 10) == (0.1, 0.0)


def test_ensemble_variance_is_second_central_moment():
    # two-point distribution {0, 2}: mean 1, every deviation 1 -> variance 1
    assert stats.ensemble_mean_var([0.0, 2.0, 0.0, 2.0]) == (1.0, 1.0)
    # shift invariance of the variance (exact in these integers)
    assert stats.ensemble_mean_var([10.0, 12.0, 10.0, 12.0]) == (11.0, 1.0)
