"""Pins for the simulated-delay model (paper Sec. 6.1 delay emulation)."""
import json
import os

import numpy as np
import pytest

from oracle import delays, stepper

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")))


def test_splitmix64_published_vectors():
    outs = [delays.splitmix64(k * delays.GAMMA - delays.GAMMA) for k in (1, 2, 3)]
    assert outs == [int(h, 16) for h in GOLD["seed0_outputs"]]


def test_vectorised_hash_matches_scalar():
    edges = delays.thresholds(["0.5", "0.25", "0.15", "0.1"])
    b = np.arange(300)
    for seed, step, key in [(0, 0, 0), (7, 123456789, 3), ((5 << 32) | 17, 999, 1)]:
        v = stepper.draw_vec(seed, step, key, b, edges)
        s = [delays.draw(seed, step, key, int(i), edges) for i in b]
        assert v.tolist() == s


def test_bins_half_open_paper_example():
    # p = {0.3, 0.4, 0.3} -> bins [0, 0.3), [0.3, 0.7), [0.7, 1]
    t = delays.thresholds(["0.3", "0.4", "0.3"])
    assert t[0] == int(0.3 * 2 ** 53) or abs(t[0] - 0.3 * 2 ** 53) < 1
    def bin_of(u):
        return sum(1 for x in t if u >= x)
    assert bin_of(0) == 0
    assert bin_of(t[0] - 1) == 0 and bin_of(t[0]) == 1
    assert bin_of(t[1] - 1) == 1 and bin_of(t[1]) == 2
    assert bin_of(2 ** 53 - 1) == 2


def test_thresholds_exact_rationals():
    assert delays.thresholds(["1/3", "1/3", "1/3"]) == [2 ** 53 // 3, (2 * 2 ** 53) // 3]
    assert delays.thresholds(["0.5", "0.25", "0.15", "0.1"])[:2] == [2 ** 52, 3 * 2 ** 51]
    with pytest.raises(ValueError):
        delays.thresholds(["0.5", "0.4"])


@pytest.mark.parametrize("probs", [["0.3", "0.4", "0.3"], ["0.5", "0.25", "0.15", "0.1"], ["0", "0", "1"]])
def test_frequencies(probs):
    edges = delays.thresholds(probs)
    n = 200000
    ks = stepper.draw_vec(11, 5, 2, np.arange(n), edges)
    for k, p in enumerate(probs):
        p = float(eval(p)) if "/" in p else float(p)
        freq = np.mean(ks == k)
        sd = np.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(freq - p) <= 5 * sd + 1e-12


def test_clamp_keeps_levels_nonnegative():
    for q in range(1, 6):
        for n in range(10):
            for k in range(5):
                kc = delays.clamp(k, n, q)
                assert 0 <= kc <= k and n - kc - (q - 1) >= 0 or kc == 0
