"""DG, ADG, ADG-AT and naive-ADG time stepping (paper Secs. 2-5).

Test infrastructure only (see oracle/__init__.py).

Semi-discrete element update, reference element [-1, 1] (Sec. 2, element-wise
weak form mapped with xi = (2x - x_e - x_{e+1}) / dx):
    M du^e/dt = (2/dx) ( S f(u^e) + phi(-1) F_e - phi(1) F_{e+1} )
F_e is the numerical flux at face x_e between elements e-1 and e, computed
from the traces u-_e = u^{e-1}_p and u+_e = u^e_0.  For f = a u and the flux
a (B+ u- + B- u+) this is exactly the paper's K-matrix form (tested).

Fluxes: upwind / central a(B+ u- + B- u+) (Sec. 2), local Lax-Friedrichs
1/2 (f(u-) + f(u+)) - lambda/2 (u+ - u-), lambda = max|f'(u+-)| (Sec. 6.1).
Inviscid Burgers uses f = u^2/2 collocated at the nodes (reading: the paper
runs viscous Burgers with LDG; the inviscid volume flux is interpolated).

Processing elements (Sec. 2, parallel implementation): PE b owns elements
[b E_pe, (b+1) E_pe); its left face f_b = b E_pe is a PE boundary.  With one
PE there are no PE boundaries.

Asynchronous PE-boundary flux (Secs. 3, 4.1, 5).  Readings:
* A delayed level of an RK stage is that stage's traces saved at step n - k
  (one history per stage).
* Conservative ADG: one delay per boundary; both neighbours use the flux of
  the common level n - k (Sec. 4.1), so the flux is single-valued.
* ADG-AT: F = sum_{j<q} c_j(k) fhat(traces at level n-k-j) (Sec. 5).
  q = 1 is plain ADG; scheme "dg" forces k = 0.
* Naive ADG (Sec. 3 update, shown non-conservative in Sec. 4.1): element f_b
  uses fhat(delayed u-, current u+), element f_b - 1 uses
  fhat(current u-, delayed u+), with independent delays (boundary keys 2b and
  2b + 1).  Oracle-only negative control.

Time integrators: Heun RK2 as printed in Sec. 4.2 (k_i include dt); classical
RK4 and the Shu-Osher SSP-RK3 (textbook forms).  The paper integrates with
low-storage 2N schemes from the works it cites in Sec. 6.1 without printing
which ones; two published members of that family are built in their 2N
form: Williamson's three-stage third-order scheme and Carpenter & Kennedy's
five-stage fourth-order scheme.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import basis, atflux, delays

N_STAGES = {"heun": 2, "ssprk3": 3, "rk4": 4, "lsrk3": 3, "lsrk4": 5}

# Williamson's third-order 2N-storage scheme (J. Comput. Phys. 35, 1980), of
# the low-storage family the paper integrates with (Sec. 6.1):
#   dU_s = A_s dU_{s-1} + dt L(U_{s-1}),  U_s = U_{s-1} + B_s dU_s,  s = 1..3.
LSRK3_A = ("0", "-5/9", "-153/128")
LSRK3_B = ("1/3", "15/16", "8/15")

# Carpenter & Kennedy's five-stage fourth-order 2N-storage scheme (NASA
# TM-109112, 1994; the 2N family that Kennedy, Carpenter & Lewis 2000, cited
# in Sec. 6.1, build on), in the same 2N form, s = 1..5.  LSRK4_C are the
# published stage abscissae, used only to check the Butcher form.
LSRK4_A = ("0", "-567301805773/1357537059087", "-2404267990393/2016746695238",
           "-3550918686646/2091501179385", "-1275806237668/842570457699")
LSRK4_B = ("1432997174477/9575080441755", "5161836677717/13612068292357", "1720146321549/2090206949498",
           "3134564353537/4481467310338", "2277821191437/14882151754819")
LSRK4_C = ("0", "1432997174477/9575080441755", "2526269341429/6820363962896", "2006345519317/3224310063776",
           "2802321613138/2924317926251")

LOW_STORAGE = {"lsrk3": (LSRK3_A, LSRK3_B), "lsrk4": (LSRK4_A, LSRK4_B)}

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix_vec(x: np.ndarray) -> np.ndarray:
    """Vectorised SplitMix64 output function on uint64 arrays (wrapping)."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(delays.GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def draw_vec(seed: int, step: int, stage_key: int, boundary: np.ndarray, edges) -> np.ndarray:
    """delays.draw for a vector of boundary keys (same definition, numpy uint64)."""
    h = _mix_vec(np.array([seed], dtype=np.uint64))
    h = _mix_vec(h ^ np.uint64(step))
    h = _mix_vec(h ^ np.uint64(stage_key))
    h = _mix_vec(h ^ boundary.astype(np.uint64))
    u = h >> np.uint64(11)
    k = np.zeros(boundary.shape, dtype=np.int64)
    for t in edges:
        k += (u >= np.uint64(t)).astype(np.int64)
    return k


class Stepper:
    """Explicit stepper for one problem.  `w` carries the problem parameters
    (a `workloads.Workload`); `U` arrays are shaped (n_elem, degree + 1)."""

    def __init__(self, w, record_delays: bool = False):
        self.w = w
        self.p = w.degree
        self.np_ = w.degree + 1
        self.n_elem = w.n_elem
        self.dx = w.length / w.n_elem
        self.dt = w.dt
        self.a = w.speed
        self.mass = basis.mass_matrix(self.p)
        self.stiff = basis.stiffness_matrix(self.p)
        nodes = basis.gll_nodes(self.p)
        self.phi_m1 = np.array([basis.lagrange(nodes, j, np.array(-1.0)) for j in range(self.np_)])
        self.phi_p1 = np.array([basis.lagrange(nodes, j, np.array(1.0)) for j in range(self.np_)])
        self.weights = self.mass @ np.ones(self.np_)
        self.n_stages = N_STAGES[w.rk]
        if w.n_elem % w.pe_size:
            raise ValueError("pe_size must divide n_elem")
        self.n_pe = w.n_elem // w.pe_size
        self.scheme = w.scheme
        if self.scheme == "adg_at":
            self.q = w.at_levels if w.at_levels else self.p + 1
        else:
            self.q = 1
        self.edges = delays.thresholds(w.probs)
        self.n_delays = len(w.probs)
        self.coef = {k: np.array(atflux.at_coefficients(self.q, k)) for k in range(self.n_delays)}
        self.faces = np.arange(self.n_pe, dtype=np.int64) * w.pe_size
        self.hist = {}          # (level, stage) -> (u-, u+) at the PE faces
        self.hist_u = {}        # local DG: (level, stage) -> u-hat at the PE faces
        self.hist_g = {}        # local DG: (level, stage) -> total flux G at the PE faces
        self.record = record_delays
        self.delay_log = {}     # (step, stage) -> clamped delays per boundary
        self.forced = None      # optional fixed delays: callable (n, s) -> int array

    # ---- physics ----------------------------------------------------------
    def flux_fn(self, u):
        if self.w.equation == "advection":
            return self.a * u
        return 0.5 * u * u  # Burgers, inviscid or viscous

    def fhat(self, um, up):
        w = self.w
        if w.flux == "upwind":
            bp, bm = (1.0, 0.0) if self.a >= 0 else (0.0, 1.0)
            return self.a * (bp * um + bm * up)
        if w.flux == "central":
            return self.a * (0.5 * um + 0.5 * up)
        if w.flux == "llf":
            lam = np.maximum(np.abs(um), np.abs(up))
            return 0.5 * (self.flux_fn(um) + self.flux_fn(up)) - 0.5 * lam * (up - um)
        raise ValueError(w.flux)

    def residual(self, y, f_left, f_right):
        """(2/dx) M^-1 ( S f(y) + phi(-1) F_left - phi(1) F_right ) per element."""
        r = self.flux_fn(y) @ self.stiff.T
        r = r + np.outer(f_left, self.phi_m1) - np.outer(f_right, self.phi_p1)
        return (2.0 / self.dx) * np.linalg.solve(self.mass, r.T).T

    # ---- delays -----------------------------------------------------------
    def delays_at(self, n: int, s: int, keys: np.ndarray) -> np.ndarray:
        if self.forced is not None:
            k = np.asarray(self.forced(n, s), dtype=np.int64)
        elif getattr(self.w, "caa", False):
            k = np.full(len(keys), delays.caa_delay(n), dtype=np.int64)
        else:
            key = s if self.w.per_stage else 0
            k = draw_vec(self.w.seed, n, key, keys, self.edges)
        return np.minimum(k, max(0, n - self.q + 1))

    # ---- viscous Burgers, local DG (Sec. 6.1) ------------------------------
    def _at_face_values(self, store: dict, raw: np.ndarray, n: int, s: int) -> np.ndarray:
        """Face values at the PE faces after the delay rule: the raw level-n
        values are stored per (level, stage); a delayed face takes the AT
        combination sum_j c_j(k) of the stored levels n-k-j (Sec. 5)."""
        store[(n, s)] = raw.copy()
        store.pop((n - (self.n_delays + self.q), s), None)
        k = self.delays_at(n, s, np.arange(self.n_pe))
        out = raw.copy()
        for b in range(self.n_pe):
            kb = int(k[b])
            if kb > 0:
                c = self.coef[kb]
                out[b] = sum(c[j] * store[(n - kb - j, s)][b] for j in range(self.q))
        return out, k

    def operator_ldg(self, y: np.ndarray, n: int, s: int) -> np.ndarray:
        """u_t + (u^2/2 - nu q)_x = 0 with q = u_x, local DG with alternating
        fluxes (u-hat = u from the left, q-hat = q from the right) and the LLF
        flux for u^2/2.  Per element, with D = M^-1 S and the lifts l_l, l_r:
          q = (2/dx) ( -D u + l_r u-hat_right - l_l u-hat_left ),
          du/dt = (2/dx) ( D g + l_l G_left - l_r G_right ),  g = u^2/2 - nu q,
          G = fhat_LLF(u-, u+) - nu q+.
        At PE faces both face values (u-hat and G) use the delayed AT
        combination, with one delay per face per (step[, stage])."""
        nu = self.w.viscosity
        uhat = np.roll(y[:, -1], 1)          # face e: the right trace of element e-1
        asyn = self.scheme != "dg" and self.n_pe > 1
        fb = self.faces
        if asyn:
            uhat[fb], k = self._at_face_values(self.hist_u, uhat[fb], n, s)
            if self.record:
                self.delay_log[(n, s)] = k.copy()
        rq = -(y @ self.stiff.T) + np.outer(np.roll(uhat, -1), self.phi_p1) - np.outer(uhat, self.phi_m1)
        q = (2.0 / self.dx) * np.linalg.solve(self.mass, rq.T).T
        um = np.roll(y[:, -1], 1)
        G = self.fhat(um, y[:, 0]) - nu * q[:, 0]
        if asyn:
            G[fb], _ = self._at_face_values(self.hist_g, G[fb], n, s)
        g = 0.5 * y * y - nu * q
        r = g @ self.stiff.T + np.outer(G, self.phi_m1) - np.outer(np.roll(G, -1), self.phi_p1)
        return (2.0 / self.dx) * np.linalg.solve(self.mass, r.T).T

    # ---- one operator evaluation -------------------------------------------
    def operator(self, y: np.ndarray, n: int, s: int) -> np.ndarray:
        if self.w.equation == "viscous_burgers":
            return self.operator_ldg(y, n, s)
        um = np.roll(y[:, -1], 1)
        up = y[:, 0].copy()
        f = self.fhat(um, up)
        f_left = f.copy()
        f_right = np.roll(f, -1)
        if self.scheme != "dg" and self.n_pe > 1:
            fb = self.faces
            left_of = (fb - 1) % self.n_elem
            self.hist[(n, s)] = (um[fb].copy(), up[fb].copy())
            self.hist.pop((n - (self.n_delays + self.q), s), None)
            if self.scheme == "naive":
                km = self.delays_at(n, s, 2 * np.arange(self.n_pe))
                kp = self.delays_at(n, s, 2 * np.arange(self.n_pe) + 1)
                old_m = np.array([self.hist[(n - km[b], s)][0][b] for b in range(self.n_pe)])
                old_p = np.array([self.hist[(n - kp[b], s)][1][b] for b in range(self.n_pe)])
                f_left[fb] = self.fhat(old_m, up[fb])
                f_right[left_of] = self.fhat(um[fb], old_p)
                if self.record:
                    self.delay_log[(n, s)] = (km, kp)
            else:
                k = self.delays_at(n, s, np.arange(self.n_pe))
                if self.record:
                    self.delay_log[(n, s)] = k.copy()
                fat = np.zeros(self.n_pe)
                for kval in np.unique(k):
                    sel = k == kval
                    c = self.coef[int(kval)]
                    acc = np.zeros(int(sel.sum()))
                    for j in range(self.q):
                        hm, hp = self.hist[(n - int(kval) - j, s)] if n - int(kval) - j >= 0 else \
                            (np.zeros(self.n_pe), np.zeros(self.n_pe))
                        acc = acc + c[j] * self.fhat(hm[sel], hp[sel])
                    fat[sel] = acc
                f_left[fb] = fat
                f_right[left_of] = fat
        return self.residual(y, f_left, f_right)

    # ---- one time step ----------------------------------------------------
    def step(self, u: np.ndarray, n: int) -> np.ndarray:
        dt = self.dt
        L = self.operator
        rk = self.w.rk
        if rk == "heun":
            k1 = dt * L(u, n, 0)
            k2 = dt * L(u + k1, n, 1)
            return u + 0.5 * (k1 + k2)
        if rk == "ssprk3":
            u1 = u + dt * L(u, n, 0)
            u2 = 0.75 * u + 0.25 * (u1 + dt * L(u1, n, 1))
            return u / 3.0 + (2.0 / 3.0) * (u2 + dt * L(u2, n, 2))
        if rk in LOW_STORAGE:
            du = np.zeros_like(u)
            y = u
            for s_, (a, b) in enumerate(zip(*LOW_STORAGE[rk])):
                du = float(Fraction(a)) * du + dt * L(y, n, s_)
                y = y + float(Fraction(b)) * du
            return y
        if rk == "rk4":
            k1 = L(u, n, 0)
            k2 = L(u + 0.5 * dt * k1, n, 1)
            k3 = L(u + 0.5 * dt * k2, n, 2)
            k4 = L(u + dt * k3, n, 3)
            return u + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        raise ValueError(rk)

    def run(self, u0: np.ndarray, n_steps: int, step0: int = 0, callback=None) -> np.ndarray:
        u = np.array(u0, dtype=np.float64, copy=True)
        for n in range(step0, step0 + n_steps):
            u = self.step(u, n)
            if callback is not None:
                callback(n + 1, u)
        return u

    def integral(self, u: np.ndarray) -> float:
        """I = int u_h dx = (dx/2) sum_e w^T u^e, summed exactly (fsum)."""
        import math
        return (self.dx / 2.0) * math.fsum((u @ self.weights).tolist())


def initial_condition(w, x: np.ndarray) -> np.ndarray:
    """Nodal interpolation of the multi-sine initial data at physical nodes."""
    ic = w.ic
    u = np.full_like(x, ic.offset, dtype=np.float64)
    for k, a, ph in zip(ic.kappa, ic.amp, ic.phase):
        u = u + a * np.sin(k * x + ph)
    return u


def initial_state(w) -> np.ndarray:
    x = basis.element_nodes(w.x_left, w.length, w.n_elem, w.degree)
    return initial_condition(w, x)


def solve(w, n_steps: int | None = None, u0: np.ndarray | None = None, **kw) -> np.ndarray:
    st = Stepper(w, **kw)
    if u0 is None:
        u0 = initial_state(w)
    return st.run(u0, w.n_steps if n_steps is None else n_steps)
