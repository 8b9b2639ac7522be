"""Discrete adjoint of the oracle stepper with the delay schedule held fixed.

Test infrastructure only (see oracle/__init__.py).

The method paper defines no adjoint; this module computes the plain
definition: the gradient of J(u_T) through the exact discrete forward map of
stepper.Stepper (same fluxes, delays, AT combinations), by reverse-mode
differentiation.  It is pinned in tests by dense Jacobians assembled from
the forward oracle (linear advection), central finite differences and the
dot-product identity.

Readings (not in the paper):
* dt is held fixed when the speed a changes.
* RK schemes are differentiated in Butcher form
  (Y_i = U + dt sum_{j<i} a_ij K_j, U' = U + dt sum_i b_i K_i), which is the
  same map as the stepper's algebraic forms.
* Local Lax-Friedrichs: lambda = max(|u-|, |u+|) is differentiated on the
  branch taken (ties pick u-), d|u|/du = sign(u) with sign(0) = +1.
"""
from __future__ import annotations

import numpy as np

from . import stepper as stp

def butcher_from_2n(A, B):
    """Butcher form of a 2N-storage scheme, exact: with U_0 = U and K_s the
    operator at U_{s-1}, U_s = U + dt sum_{j<=s} beta_{s,j} K_j where
    beta_{s,j} = B_s alpha_{s,j} + beta_{s-1,j} and alpha_{s,j} (the weights
    of dU_s) = A_s alpha_{s-1,j} for j < s, 1 for j = s.  Stage s+1 reads
    U_s, so a_{s+1,j} = beta_{s,j} and b_j = beta_{S,j}."""
    from fractions import Fraction
    A = [Fraction(x) for x in A]
    B = [Fraction(x) for x in B]
    S = len(A)
    alpha = [Fraction(0)] * S
    beta = [Fraction(0)] * S
    rows = [[]]
    for s in range(S):
        alpha = [A[s] * alpha[j] if j < s else (Fraction(1) if j == s else Fraction(0)) for j in range(S)]
        beta = [beta[j] + B[s] * alpha[j] for j in range(S)]
        if s + 1 < S:
            rows.append(beta[:s + 1])
    return rows, beta


def _float_table(rows, b):
    return [[float(x) for x in r] for r in rows], [float(x) for x in b]


BUTCHER = {
    "lsrk3": _float_table(*butcher_from_2n(stp.LSRK3_A, stp.LSRK3_B)),
    "lsrk4": _float_table(*butcher_from_2n(stp.LSRK4_A, stp.LSRK4_B)),
    "heun": ([[], [1.0]], [0.5, 0.5]),
    "ssprk3": ([[], [1.0], [0.25, 0.25]], [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]),
    "rk4": ([[], [0.5], [0.0, 0.5], [0.0, 0.0, 1.0]], [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]),
}


def _fhat_partials(st: stp.Stepper, um, up):
    """(d fhat / d u-, d fhat / d u+) elementwise."""
    w = st.w
    if w.flux == "upwind":
        return (np.full_like(um, st.a if st.a >= 0 else 0.0), np.full_like(up, 0.0 if st.a >= 0 else st.a))
    if w.flux == "central":
        return np.full_like(um, 0.5 * st.a), np.full_like(up, 0.5 * st.a)
    # LLF for f = u^2/2: 1/2 (f(u-) + f(u+)) - 1/2 lam (u+ - u-), lam = max(|u-|, |u+|)
    pick_m = np.abs(um) >= np.abs(up)
    lam = np.where(pick_m, np.abs(um), np.abs(up))
    sgn_m = np.where(um >= 0, 1.0, -1.0)
    sgn_p = np.where(up >= 0, 1.0, -1.0)
    dlam_dm = np.where(pick_m, sgn_m, 0.0)
    dlam_dp = np.where(pick_m, 0.0, sgn_p)
    jump = up - um
    dm = 0.5 * um - 0.5 * dlam_dm * jump + 0.5 * lam
    dp = 0.5 * up - 0.5 * dlam_dp * jump - 0.5 * lam
    return dm, dp


def _dflux_fn(st: stp.Stepper, y):
    return np.full_like(y, st.a) if st.w.equation == "advection" else y


class Tape:
    """Forward run recording every stage input and every delay."""

    def __init__(self, w, u0, n_steps):
        self.st = stp.Stepper(w, record_delays=True)
        self.n_steps = n_steps
        self.stage_inputs = []      # [n][s] -> Y
        self.stage_values = []      # [n][s] -> K = L(Y)
        st = self.st
        u = np.array(u0, dtype=np.float64, copy=True)
        a_tab, b_tab = BUTCHER[w.rk]
        dt = st.dt
        for n in range(n_steps):
            ys, ks = [], []
            for i in range(st.n_stages):
                y = u.copy()
                for j in range(i):
                    if a_tab[i][j] != 0.0:
                        y = y + dt * a_tab[i][j] * ks[j]
                ys.append(y)
                ks.append(st.operator(y, n, i))
            self.stage_inputs.append(ys)
            self.stage_values.append(ks)
            un = u.copy()
            for i in range(st.n_stages):
                un = un + dt * b_tab[i] * ks[i]
            u = un
        self.u_final = u


def gradient(w, u0, n_steps, cot_fn, with_scale=False):
    """Returns (u_T, dJ/du0, dJ/da) where cot_fn(u_T) = dJ/du_T; with_scale
    also returns the sum of |terms| of dJ/da, the scale of its rounding
    error (dJ/da is a cancelling sum over every DOF, stage and step)."""
    tape = Tape(w, u0, n_steps)
    st = tape.st
    a_tab, b_tab = BUTCHER[w.rk]
    S = st.n_stages
    dt = st.dt
    ne, npp = st.n_elem, st.np_
    lam = np.array(cot_fn(tape.u_final), dtype=np.float64)
    adj_ring = {}                    # (level, stage) -> sensitivity of the raw PE flux per boundary
    dj_da = 0.0
    dj_da_scale = 0.0
    minv = np.linalg.inv(st.mass)
    faces = st.faces
    left_of = (faces - 1) % ne
    for n in range(n_steps - 1, -1, -1):
        ys = tape.stage_inputs[n]
        kvals = tape.stage_values[n]
        mu = [None] * S
        lam_u = lam.copy()
        for i in range(S - 1, -1, -1):
            lk = dt * b_tab[i] * lam
            for j in range(i + 1, S):
                if a_tab[j][i] != 0.0:
                    lk = lk + dt * a_tab[j][i] * mu[j]
            y = ys[i]
            # dJ/da through the explicit speed dependence of this stage (linear advection)
            if w.equation == "advection":
                dj_da += float(np.sum(lk * kvals[i])) / st.a
                dj_da_scale += float(np.sum(np.abs(lk * kvals[i]))) / abs(st.a)
            # transpose of K = (2/dx) M^-1 (S f(y) + phi(-1) F_l - phi(1) F_r)
            wv = (2.0 / st.dx) * (lk @ minv.T)                # M^-T lk per element
            m_i = (wv @ st.stiff) * _dflux_fn(st, y)           # S^T w, times f'(y)
            lam_fl = wv @ st.phi_m1                             # sensitivity of the left-face flux used by e
            lam_fr = -(wv @ st.phi_p1)                          # ... of the right-face flux used by e
            um = np.roll(y[:, -1], 1)
            up = y[:, 0]
            dm, dp = _fhat_partials(st, um, up)
            lam_face = lam_fl + np.roll(lam_fr, 1)              # face e: used by e (left) and e-1 (right)
            lam_raw = lam_face.copy()
            if st.scheme != "dg" and st.n_pe > 1:
                k = st.delay_log[(n, i)]
                lam_at = lam_face[faces]
                lam_raw[faces] = np.where(k == 0, lam_at, 0.0) + adj_ring.pop((n, i), np.zeros(st.n_pe))
                for b in range(st.n_pe):
                    kb = int(k[b])
                    if kb == 0:
                        continue
                    c = st.coef[kb]
                    for jj in range(st.q):
                        key = (n - kb - jj, i)
                        acc = adj_ring.setdefault(key, np.zeros(st.n_pe))
                        acc[b] += c[jj] * lam_at[b]
            # raw flux at face f depends on y^{f-1}_p (u-) and y^f_0 (u+)
            m_i[:, 0] += lam_raw * dp
            m_i[:, -1] += np.roll(lam_raw * dm, -1)
            mu[i] = m_i
            lam_u = lam_u + m_i
        lam = lam_u
    if with_scale:
        return tape.u_final, lam, dj_da, dj_da_scale
    return tape.u_final, lam, dj_da


def misfit_cotangent(u_ref):
    """J = 1/2 ||u_T - u_ref||^2 over all DG coefficients."""
    return lambda ut: ut - u_ref


def dense_step_map(w, n_steps):
    """Dense matrix of u0 -> u_T for linear advection (fixed schedule),
    column by column through the forward oracle."""
    ne, npp = w.n_elem, w.degree + 1
    size = ne * npp
    g = np.zeros((size, size))
    for c in range(size):
        e = np.zeros(size)
        e[c] = 1.0
        g[:, c] = stp.Stepper(w).run(e.reshape(ne, npp), n_steps).ravel()
    return g
