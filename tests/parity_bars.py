"""Parity bars shared by the GPU tests (imported by them; not collected).

Two norms are checked:
  * relative L2 over the whole state (the target's 1e-12 bar);
  * max |GPU - oracle| over the nodal values of the elements on either side
    of each PE face, divided by max |oracle|.  An error confined to PE-face
    elements is diluted in the whole-state L2 by about sqrt(N_E / P) (16 at
    2^20 elements and 4096 PEs); this norm sees it undiluted.

Where a case is ill-conditioned (AT weights of high q at the largest delays,
unstable modes) the bar in each norm is 30 times the oracle's own change
under a rounding-level (1e-16 relative) perturbation of the initial state,
if that is larger than 1e-12: no FP64 evaluation order can agree more
closely than the problem's conditioning allows, while a wrong term, sign or
level moves the result by orders of magnitude more."""
from __future__ import annotations

import numpy as np

from oracle import stats, stepper

TOL = 1e-12
RESPONSE_FACTOR = 30.0


def pe_face_elements(w) -> np.ndarray:
    """Elements left and right of every PE face (empty when no face is
    asynchronous: synchronous DG or a single PE)."""
    n_pe = w.n_elem // w.pe_size
    if w.scheme == "dg" or n_pe <= 1:
        return np.zeros(0, dtype=np.int64)
    f = np.arange(n_pe, dtype=np.int64) * w.pe_size
    return np.unique(np.concatenate([f, (f - 1) % w.n_elem]))


def pe_max_rel(got, ref, w) -> float:
    """max |got - ref| over the PE-face elements / max |ref| (0 without PE faces)."""
    els = pe_face_elements(w)
    if els.size == 0:
        return 0.0
    got, ref = np.asarray(got), np.asarray(ref)
    scale = float(np.max(np.abs(ref)))
    d = float(np.max(np.abs(got[els] - ref[els])))
    return d / scale if scale > 0 else d


def oracle_response(w, u0, n, ref):
    """(relative L2, PE-face max) change of the oracle's n-step result under a
    1e-16 relative perturbation of u0; infinite where the oracle blows up."""
    rng = np.random.default_rng(12345)
    u1 = u0 * (1.0 + 1e-16 * rng.standard_normal(u0.shape))
    r1 = stepper.Stepper(w).run(u1, n)
    if not (np.isfinite(ref).all() and np.isfinite(r1).all()):
        return float("inf"), float("inf")
    return stats.rel_l2(r1, ref), pe_max_rel(r1, ref, w)


def derived_bars(w, u0, n, ref):
    """(L2 bar, PE-face max bar) from the oracle's own rounding response."""
    l2, pe = oracle_response(w, u0, n, ref)
    return max(TOL, RESPONSE_FACTOR * l2), max(TOL, RESPONSE_FACTOR * pe)
