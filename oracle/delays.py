"""Simulated communication delays at PE boundaries (paper Sec. 3 and Sec. 6.1).

Test infrastructure only (see oracle/__init__.py).

The paper draws one uniform number in [0, 1] per PE boundary per time step
and maps it into L bins of widths p_0..p_{L-1}: bin k gives delay k
([0, p_0), [p_0, p_0 + p_1), ..., last bin closed).  Readings:
* The uniform number comes from a counter-based generator so that any
  implementation can reproduce the schedule: the SplitMix64 output function
  (Steele, Lea & Flood, OOPSLA 2014; public-domain C by S. Vigna) is chained
  over (seed, step, stage key, boundary):
      h = mix(mix(mix(mix(seed) ^ step) ^ stage_key) ^ boundary)
  and U = h >> 11 is a 53-bit integer uniform on [0, 2^53).
* Bin edges T_k = floor(2^53 * (p_0 + ... + p_{k-1})), k = 1..L-1, computed
  exactly from the decimal probabilities; delay = #{k : U >= T_k}.
* stage_key is the RK stage index when delays are drawn per stage, else 0.
* Before enough history exists the delay is clamped:
  k = min(k_drawn, max(0, n - q + 1)) so that every level n-k-j (j < q) is >= 0.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Sequence

import numpy as np

# Communication-avoiding schedule (Sec. 7, the two-dimensional runs): in
# every cycle of five steps the first two communicate with synchronisation and
# the remaining three do not, during which the PE-boundary data are 0, 1 and 2
# levels old (L = 3).  Deterministic and equal at every PE boundary.
CAA_CYCLE = (0, 0, 0, 1, 2)


def caa_delay(step: int) -> int:
    return CAA_CYCLE[step % len(CAA_CYCLE)]


MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    """One SplitMix64 output for state x: z = x + gamma, then the variant-13
    finaliser (xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31)."""
    z = (x + GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def delay_hash(seed: int, step: int, stage_key: int, boundary: int) -> int:
    h = splitmix64(seed & MASK64)
    h = splitmix64(h ^ (step & MASK64))
    h = splitmix64(h ^ (stage_key & MASK64))
    h = splitmix64(h ^ (boundary & MASK64))
    return h


def thresholds(probs: Sequence) -> list:
    """Integer bin edges T_1..T_{L-1} on [0, 2^53) from exact probabilities."""
    ps = [Fraction(p) for p in probs]
    if any(p < 0 for p in ps) or sum(ps) != 1:
        raise ValueError("probabilities must be non-negative and sum to 1")
    out, acc = [], Fraction(0)
    for p in ps[:-1]:
        acc += p
        out.append(int((acc * (1 << 53)).__floor__()))
    return out


def draw(seed: int, step: int, stage_key: int, boundary: int, edges: Sequence[int]) -> int:
    u = delay_hash(seed, step, stage_key, boundary) >> 11
    return sum(1 for t in edges if u >= t)


def clamp(k_drawn: int, step: int, q: int) -> int:
    return min(k_drawn, max(0, step - q + 1))


def schedule(seed: int, probs: Sequence, n_steps: int, n_stages: int, n_bound: int,
             per_stage: bool, q: int, step0: int = 0, caa: bool = False) -> np.ndarray:
    """Clamped delays k[n - step0, s, b] for steps step0..step0+n_steps-1
    (caa: the communication-avoiding cycle instead of random draws)."""
    edges = thresholds(probs)
    out = np.zeros((n_steps, n_stages, n_bound), dtype=np.int32)
    for i in range(n_steps):
        n = step0 + i
        for s in range(n_stages):
            key = s if per_stage else 0
            for b in range(n_bound):
                k = caa_delay(n) if caa else draw(seed, n, key, b, edges)
                out[i, s, b] = clamp(k, n, q)
    return out
