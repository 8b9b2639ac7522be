"""Pins for the oracle stepper (paper Secs. 2-6).

Each test checks the oracle against something it does not compute itself:
the paper's K-matrix equations, exact solutions, invariants (conservation),
the printed convergence orders, and special cases that must collapse to
plain DG."""
import math
from dataclasses import replace

import numpy as np
import pytest

from paper_2404_03399_amd import workloads as W
from oracle import basis, exact, stats, stepper


def _wl(**kw):
    base = dict(name="t", degree=2, n_elem=32, pe_size=8, probs=("0.3", "0.4", "0.3"), seed=3,
                dt=0.01, n_steps=10, ic=W.PAPER_MULTISINE)
    base.update(kw)
    return W.Workload(**base)


def _kmatrix_operator(u, p, a, dx, bp, bm, old=None, faces=()):
    """Paper's matrix form, assembled element by element:
    M du^e/dt = (2a/dx) (K^- u^{e-1} + (K_l + S + K_r) u^e + K^+ u^{e+1}),
    and, at a PE face x_e with common delayed level (Sec. 4.1),
    e-1: K^- u^{e-2} + (K_l + S) u^{e-1} + K_r u_old^{e-1} + K^+ u_old^e
    e  : K^- u_old^{e-1} + K_l u_old^e + (S + K_r) u^e + K^+ u^{e+1}."""
    m = basis.mass_matrix(p)
    s = basis.stiffness_matrix(p)
    km, kp, kl, kr = basis.flux_matrices(p, bp, bm)
    ne = u.shape[0]
    out = np.zeros_like(u)
    faces = set(faces)
    for e in range(ne):
        em, ep = (e - 1) % ne, (e + 1) % ne
        left_pe = e in faces
        right_pe = ep in faces
        r = s @ u[e]
        if left_pe:
            r = r + km @ old[em] + kl @ old[e]
        else:
            r = r + km @ u[em] + kl @ u[e]
        if right_pe:
            r = r + kr @ old[e] + kp @ old[ep]
        else:
            r = r + kr @ u[e] + kp @ u[ep]
        out[e] = (2.0 * a / dx) * np.linalg.solve(m, r)
    return out


@pytest.mark.parametrize("flux,bp,bm", [("upwind", 1.0, 0.0), ("central", 0.5, 0.5)])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_sync_operator_equals_paper_matrix_form(flux, bp, bm, p):
    w = _wl(scheme="dg", flux=flux, degree=p, speed=1.7)
    st = stepper.Stepper(w)
    u = np.random.default_rng(p).standard_normal((w.n_elem, p + 1))
    ref = _kmatrix_operator(u, p, 1.7, st.dx, bp, bm)
    np.testing.assert_allclose(st.operator(u, 0, 0), ref, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("flux,bp,bm", [("upwind", 1.0, 0.0), ("central", 0.5, 0.5)])
def test_conservative_adg_equals_paper_equation(flux, bp, bm):
    """Sec. 4.1 conservative update at PE faces with a delayed common level."""
    p = 2
    w = _wl(scheme="adg", flux=flux, degree=p, probs=("0", "1"))
    st = stepper.Stepper(w)
    st.forced = lambda n, s: np.full(w.n_pe, 0 if n == 4 else 1)
    rng = np.random.default_rng(0)
    u_old = rng.standard_normal((w.n_elem, p + 1))
    u_new = rng.standard_normal((w.n_elem, p + 1))
    st.operator(u_old, 4, 1)                 # level 4, stage 1 is stored as history
    got = st.operator(u_new, 5, 1)           # every boundary delayed by k = 1
    faces = [b * w.pe_size for b in range(w.n_pe)]
    ref = _kmatrix_operator(u_new, p, 1.0, st.dx, bp, bm, old=u_old, faces=faces)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-10)


def _run_error(w):
    st = stepper.Stepper(w)
    u0 = stepper.initial_state(w)
    i0 = st.integral(u0)
    u = st.run(u0, w.n_steps)
    x = basis.element_nodes(w.x_left, w.length, w.n_elem, w.degree)
    ue = exact.solution(w, x, w.dt * w.n_steps)
    return stats.mean_abs(u, ue), stats.max_abs(u, ue), abs(st.integral(u) - i0)


CASES = [(1, "heun", 0.1), (2, "ssprk3", 0.02), (3, "rk4", 0.01)]


def _series(p, rk, sig, scheme, sizes, probs=("0.3", "0.4", "0.3"), seed=1, t_final=0.5):
    out = []
    for ne in sizes:
        dt, n = W.time_step(W.TWO_PI, ne, sig, 1.0, t_final)
        w = _wl(scheme=scheme, rk=rk, degree=p, n_elem=ne, pe_size=ne // 8, probs=probs,
                seed=seed, per_stage=False, dt=dt, n_steps=n)
        out.append(_run_error(w))
    return np.array(out)


@pytest.mark.parametrize("p,rk,sig", CASES)
def test_sync_dg_order_and_conservation(p, rk, sig):
    e = _series(p, rk, sig, "dg", [32, 64, 128])
    slopes = np.log2(e[:-1, 0] / e[1:, 0])
    assert np.all(slopes > p + 1 - 0.15), slopes      # paper Fig. 7: slopes -2, -3, -4
    assert e[:, 2].max() < 1e-12


@pytest.mark.parametrize("p,rk,sig", CASES)
def test_adg_loses_order_at_recovers_it(p, rk, sig):
    sizes = [64, 128, 256] if p < 3 else [64, 128]
    dg = _series(p, rk, sig, "dg", sizes)
    adg = _series(p, rk, sig, "adg", sizes)
    at = _series(p, rk, sig, "adg_at", sizes)
    # conservative schemes conserve the integral to round-off (Sec. 4.1)
    assert adg[:, 2].max() < 1e-12 and at[:, 2].max() < 1e-12
    # standard fluxes with delays: at most first order in the max norm and far
    # larger errors than synchronous DG (Sec. 4.3, Fig. 7)
    linf_adg = np.log2(adg[:-1, 1] / adg[1:, 1])
    assert linf_adg.mean() < 1.6, linf_adg
    assert np.all(adg[:, 1] > 2 * dg[:, 1]) and np.all(adg[:, 0] > 1.2 * dg[:, 0])
    if p > 1:
        assert adg[-1, 0] > 10 * dg[-1, 0]
    # AT fluxes restore order p+1 and DG-level errors (Sec. 5, Fig. 8)
    slopes_at = np.log2(at[:-1, 0] / at[1:, 0])
    assert np.all(slopes_at > p + 1 - 0.2), slopes_at
    assert np.all(at[:, 0] < 1.5 * dg[:, 0])


def _series_caa(p, rk, sig, scheme, sizes, t_final=0.5):
    out = []
    for ne in sizes:
        dt, n = W.time_step(W.TWO_PI, ne, sig, 1.0, t_final)
        w = _wl(scheme=scheme, rk=rk, degree=p, n_elem=ne, pe_size=ne // 8, probs=W.DELAYS_UNIFORM3,
                caa=True, per_stage=False, dt=dt, n_steps=n)
        out.append(_run_error(w))
    return np.array(out)


def test_williamson_lsrk3_order_conditions():
    """The 2N-storage coefficients (A, B) give, in Butcher form, c = (0, 1/3,
    3/4), a21 = 1/3, a31 = -3/16, a32 = 15/16, b = (1/6, 3/10, 8/15), which
    meets the four third-order conditions exactly and misses fourth order."""
    from fractions import Fraction as Fr
    from oracle import adjoint
    rows, b = adjoint.butcher_from_2n(stepper.LSRK3_A, stepper.LSRK3_B)
    assert rows == [[], [Fr(1, 3)], [Fr(-3, 16), Fr(15, 16)]] and b == [Fr(1, 6), Fr(3, 10), Fr(8, 15)]
    c = [sum(r, Fr(0)) for r in rows]
    assert sum(b) == 1
    assert sum(bi * ci for bi, ci in zip(b, c)) == Fr(1, 2)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == Fr(1, 3)
    assert b[2] * rows[2][1] * c[1] == Fr(1, 6)
    assert sum(bi * ci ** 3 for bi, ci in zip(b, c)) != Fr(1, 4)


def test_williamson_lsrk3_converges_at_third_order():
    e = _series(2, "lsrk3", 0.02, "dg", [32, 64, 128])
    slopes = np.log2(e[:-1, 0] / e[1:, 0])
    assert np.all(slopes > 2.85), slopes
    assert e[:, 2].max() < 1e-12
    at = _series(2, "lsrk3", 0.02, "adg_at", [32, 64, 128])
    slopes = np.log2(at[:-1, 0] / at[1:, 0])
    assert np.all(slopes > 2.8), slopes
    # the same map as its Butcher form (one step of the adjoint's table)
    w = _wl(scheme="dg", rk="lsrk3", degree=2, n_elem=16, pe_size=4, dt=0.01, n_steps=1)
    st = stepper.Stepper(w)
    u = stepper.initial_state(w)
    from oracle import adjoint
    rows, b = adjoint.BUTCHER["lsrk3"]
    ks = []
    for i in range(3):
        y = u + w.dt * sum((rows[i][j] * ks[j] for j in range(i)), np.zeros_like(u))
        ks.append(st.operator(y, 0, i))
    ref = u + w.dt * sum(bi * k for bi, k in zip(b, ks))
    np.testing.assert_allclose(st.step(u, 0), ref, rtol=0, atol=1e-14)


def _order_conditions(rows, b):
    """The eight order conditions of a four-stage-order Runge-Kutta method,
    each as (value, exact target), in exact rationals."""
    from fractions import Fraction as Fr
    S = len(b)
    a = [list(r) + [Fr(0)] * (S - len(r)) for r in rows]
    c = [sum(r, Fr(0)) for r in a]

    def A(v):
        return [sum(a[i][j] * v[j] for j in range(S)) for i in range(S)]

    def dot(u, v):
        return sum(x * y for x, y in zip(u, v))

    c2 = [x * x for x in c]
    return {"b": (sum(b), Fr(1)), "bc": (dot(b, c), Fr(1, 2)), "bc2": (dot(b, c2), Fr(1, 3)),
            "bAc": (dot(b, A(c)), Fr(1, 6)), "bc3": (dot(b, [x ** 3 for x in c]), Fr(1, 4)),
            "bcAc": (dot(b, [x * y for x, y in zip(c, A(c))]), Fr(1, 8)),
            "bAc2": (dot(b, A(c2)), Fr(1, 12)), "bAAc": (dot(b, A(A(c))), Fr(1, 24)),
            "bc4 (fifth order)": (dot(b, [x ** 4 for x in c]), Fr(1, 5))}, c


def test_carpenter_kennedy_lsrk4_order_conditions():
    """The published 2N coefficients (A, B), turned into Butcher form exactly,
    meet all eight fourth-order conditions to the accuracy of their 13-digit
    rationals (1e-24) and miss the fifth-order condition b.c^4 = 1/5 by
    about 1e-4; their stage abscissae equal the published c.  A mistyped
    digit in any coefficient breaks a condition at 1e-13 or more."""
    from fractions import Fraction as Fr
    from oracle import adjoint
    rows, b = adjoint.butcher_from_2n(stepper.LSRK4_A, stepper.LSRK4_B)
    assert len(b) == 5 and stepper.N_STAGES["lsrk4"] == 5
    conds, c = _order_conditions(rows, b)
    fifth = conds.pop("bc4 (fifth order)")
    for name, (v, t) in conds.items():
        assert abs(v - t) < Fr(1, 10 ** 24), (name, float(v - t))
    assert abs(fifth[0] - fifth[1]) > Fr(1, 10 ** 5)
    for ci, pub in zip(c, stepper.LSRK4_C):
        assert abs(ci - Fr(pub)) < Fr(1, 10 ** 24)
    # a one-digit change of one coefficient is caught
    bad_a = list(stepper.LSRK4_A)
    bad_a[2] = "-2404267990394/2016746695238"
    rows2, b2 = adjoint.butcher_from_2n(bad_a, stepper.LSRK4_B)
    conds2, _ = _order_conditions(rows2, b2)
    conds2.pop("bc4 (fifth order)")
    assert max(abs(v - t) for v, t in conds2.values()) > Fr(1, 10 ** 13)


def test_lsrk4_stability_polynomial():
    """One step of a linear problem multiplies by R(Z) = sum_{j<=4} Z^j/j! +
    g5 Z^5 with g5 = b^T A^4 1 (the only fifth-degree elementary weight of a
    five-stage explicit method); g5 != 1/120 (the scheme is not fifth order)."""
    from fractions import Fraction as Fr
    from oracle import adjoint, fourier
    rows, b = adjoint.butcher_from_2n(stepper.LSRK4_A, stepper.LSRK4_B)
    g5 = b[4] * rows[4][3] * rows[3][2] * rows[2][1] * rows[1][0]
    assert abs(g5 - Fr(1, 120)) > Fr(1, 10 ** 5)
    for p, th in ((2, 0.7), (3, -1.9)):
        z = fourier.stage_matrix(p, "upwind", 0.05, th)
        g = np.eye(p + 1, dtype=complex)
        term = np.eye(p + 1, dtype=complex)
        for j in range(1, 5):
            term = term @ z / j
            g = g + term
        g = g + float(g5) * np.linalg.matrix_power(z, 5)
        np.testing.assert_allclose(fourier.amplification(p, "lsrk4", "upwind", 0.05, th), g, atol=1e-14)


def test_lsrk4_converges_at_fourth_order():
    """DG(3) and ADG(3)-AT4 with the five-stage fourth-order 2N scheme
    converge at order 4 (Sec. 6.1 matches the integrator's order to the
    spatial order); the 2N map equals its Butcher form."""
    e = _series(3, "lsrk4", 0.01, "dg", [32, 64, 128])
    slopes = np.log2(e[:-1, 0] / e[1:, 0])
    assert np.all(slopes > 3.85), slopes
    assert e[:, 2].max() < 1e-12
    at = _series(3, "lsrk4", 0.01, "adg_at", [32, 64, 128])
    slopes = np.log2(at[:-1, 0] / at[1:, 0])
    assert np.all(slopes > 3.8), slopes
    assert np.all(at[:, 0] < 1.5 * e[:, 0]), (at[:, 0], e[:, 0])
    w = _wl(scheme="adg_at", rk="lsrk4", degree=3, n_elem=16, pe_size=4, dt=0.01, n_steps=1)
    st = stepper.Stepper(w)
    u = stepper.initial_state(w)
    from oracle import adjoint
    rows, b = adjoint.BUTCHER["lsrk4"]
    ks = []
    for i in range(5):
        y = u + w.dt * sum((rows[i][j] * ks[j] for j in range(i)), np.zeros_like(u))
        ks.append(st.operator(y, 0, i))
    ref = u + w.dt * sum(bi * k for bi, k in zip(b, ks))
    np.testing.assert_allclose(stepper.Stepper(w).step(u, 0), ref, rtol=0, atol=1e-14)


def test_communication_avoiding_cycle():
    """Sec. 7's communication-avoiding runs (L = 3, delays 0, 1, 2 in the three
    steps of every five without communication): ADG(1)-AT2-RK2 keeps second
    order and DG-level errors, conservation holds, and the cycle's delays are
    really applied (plain ADG with the same cycle is far less accurate)."""
    sizes = [64, 128, 256]
    dg = _series(1, "heun", 0.1, "dg", sizes)
    at = _series_caa(1, "heun", 0.1, "adg_at", sizes)
    plain = _series_caa(1, "heun", 0.1, "adg", sizes)
    slopes = np.log2(at[:-1, 0] / at[1:, 0])
    assert np.all(slopes > 1.85), slopes
    assert np.all(at[:, 0] < 1.5 * dg[:, 0])
    assert at[:, 2].max() < 1e-12 and plain[:, 2].max() < 1e-12
    assert np.all(plain[:, 1] > 2 * dg[:, 1])
    st = stepper.Stepper(_wl(scheme="adg_at", rk="heun", degree=1, n_elem=32, pe_size=4,
                             probs=W.DELAYS_UNIFORM3, caa=True, dt=1e-3, n_steps=12), record_delays=True)
    st.run(stepper.initial_state(st.w), 12)
    ks = [int(st.delay_log[(n, 0)][0]) for n in range(12)]
    assert ks == [0, 0, 0, 1, 2, 0, 0, 0, 1, 2, 0, 0]  # the cycle (0, 0, 0, 1, 2) by step mod 5


def test_naive_adg_breaks_conservation():
    """Sec. 4.1: independent delays on the two sides make the flux two-valued."""
    e = _series(1, "heun", 0.1, "naive", [64])
    assert e[0, 2] > 1e-6
    sizes = [64, 128, 256]
    naive = _series(1, "heun", 0.1, "naive", sizes)
    slopes = np.log2(naive[:-1, 0] / naive[1:, 0])
    assert np.all(slopes < 1.3), slopes                  # first order (Fig. 7)


@pytest.mark.parametrize("rk", ["heun", "ssprk3", "rk4"])
def test_special_cases_reduce_to_dg(rk):
    base = _wl(rk=rk, degree=2, n_elem=48, pe_size=12, dt=0.002, n_steps=25, seed=9)
    u0 = stepper.initial_state(base)
    dg = stepper.Stepper(replace(base, scheme="dg")).run(u0, 25)
    # one delay level only (L = 1): every delay is zero
    for sch in ("adg", "adg_at"):
        got = stepper.Stepper(replace(base, scheme=sch, probs=("1",))).run(u0, 25)
        assert np.array_equal(got, dg)
        # zero-probability delays
        got = stepper.Stepper(replace(base, scheme=sch, probs=("1", "0", "0"))).run(u0, 25)
        assert np.array_equal(got, dg)
        # a single PE has no PE boundaries
        got = stepper.Stepper(replace(base, scheme=sch, pe_size=48)).run(u0, 25)
        assert np.array_equal(got, dg)
    # AT with one level is plain ADG
    a = stepper.Stepper(replace(base, scheme="adg")).run(u0, 25)
    b = stepper.Stepper(replace(base, scheme="adg_at", at_levels=1)).run(u0, 25)
    assert np.array_equal(a, b)


def test_delays_really_applied_and_clamped():
    w = _wl(scheme="adg_at", degree=2, probs=("0", "0", "1"))   # always k = 2 (mean delay 2.0)
    st = stepper.Stepper(w, record_delays=True)
    st.run(stepper.initial_state(w), 8)
    ks = [st.delay_log[(n, 0)][0] for n in range(8)]
    # q = 3: k = min(2, max(0, n - 2))
    assert ks == [0, 0, 0, 1, 2, 2, 2, 2]


def test_burgers_pre_shock_exact_solution():
    errs = []
    for ne in (32, 64, 128):
        dx = W.TWO_PI / ne
        w = W.c3_burgers(n_elem=ne, n_steps=0, sigma=0.05, scheme="dg")
        dt, n = W.time_step(W.TWO_PI, ne, 0.05, 1.5, 0.4)
        w = replace(w, dt=dt, n_steps=n, pe_size=ne // 4)
        errs.append(_run_error(w))
    e = np.array(errs)
    assert e[:, 2].max() < 1e-12                                   # conservation
    slopes = np.log2(e[:-1, 0] / e[1:, 0])
    assert np.all(slopes > 2.3), slopes                            # high order before the shock
    # asynchronous AT run stays at the DG error level (smaller Courant number:
    # the AT extrapolation narrows the stability region, Sec. 4.2.2)
    ne = 128
    dt, n = W.time_step(W.TWO_PI, ne, 0.01, 1.5, 0.4)
    w = replace(W.c3_burgers(n_elem=ne, n_steps=n, sigma=0.01), dt=dt, pe_size=16)
    at = _run_error(w)
    dg = _run_error(replace(w, scheme="dg"))
    adg = _run_error(replace(w, scheme="adg"))
    assert at[2] < 1e-12 and adg[2] < 1e-12
    assert at[0] < 1.1 * dg[0] and adg[0] > 1.5 * dg[0]


# ---- viscous Burgers, local DG (Sec. 6.1, Fig. 11) -------------------------
def _ldg(**kw):
    base = dict(name="ldg", equation="viscous_burgers", flux="llf", rk="heun", degree=2, n_elem=32, pe_size=8,
                probs=("0.3", "0.4", "0.3"), scheme="dg", viscosity=0.1, dt=1e-3, n_steps=10,
                ic=W.PAPER_MULTISINE)
    base.update(kw)
    return W.Workload(**base)


def test_ldg_without_viscosity_is_the_dg_burgers_operator():
    y = np.random.default_rng(2).standard_normal((32, 3))
    for scheme in ("dg", "adg_at"):
        a = stepper.Stepper(_ldg(viscosity=0.0, scheme=scheme, at_levels=2 if scheme == "adg_at" else 0))
        b = stepper.Stepper(_ldg(equation="burgers", viscosity=0.0, scheme=scheme,
                                 at_levels=2 if scheme == "adg_at" else 0))
        for n in range(5):  # builds up delayed history on both
            np.testing.assert_allclose(a.operator(y + 0.01 * n, n, 0), b.operator(y + 0.01 * n, n, 0),
                                       rtol=0, atol=1e-12)


def _heat_error(p, ne, scheme, eps=1e-6, nu=0.1, t_final=0.05):
    """Small-amplitude data: the nonlinear term is O(eps^2), so the solution
    is the heat equation's, each mode decaying as exp(-nu kappa^2 t)."""
    ic = W.MultiSine((2, 3), (2.0 * eps, 1.0 * eps), (0.3, 1.1))
    dx = W.TWO_PI / ne
    # dt = 0.002 dx^2 / nu: the AT extrapolation of the stiff diffusive face
    # values needs a smaller step than the synchronous scheme
    dt, n = W.time_step(W.TWO_PI, ne, 0.002 * dx / nu, 1.0, t_final)
    w = _ldg(degree=p, n_elem=ne, pe_size=ne // 4, scheme=scheme, at_levels=2 if scheme == "adg_at" else 0,
             rk="rk4", viscosity=nu, dt=dt, n_steps=n, ic=ic)
    st = stepper.Stepper(w)
    u0 = stepper.initial_state(w)
    i0 = st.integral(u0)
    u = st.run(u0, n)
    x = basis.element_nodes(w.x_left, w.length, ne, p)
    ue = sum(a * np.exp(-nu * k * k * t_final) * np.sin(k * x + ph) for k, a, ph in zip(ic.kappa, ic.amp, ic.phase))
    return stats.mean_abs(u, ue) / eps, abs(st.integral(u) - i0) / eps, u


@pytest.mark.parametrize("p", [1, 2])
def test_ldg_diffusion_converges_at_order_p_plus_1(p):
    errs = [_heat_error(p, ne, "dg")[0] for ne in (16, 32, 64)]
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > p - 0.7) and slopes[-1] > p + 1 - 0.15, slopes  # alternating fluxes: optimal order
    at = [_heat_error(p, ne, "adg_at") for ne in (16, 32, 64)]
    slopes = np.log2(np.array([e[0] for e in at[:-1]]) / np.array([e[0] for e in at[1:]]))
    assert np.all(slopes > p - 0.7) and slopes[-1] > p + 1 - 0.15, slopes  # AT2 at both face values
    assert max(e[1] for e in at) < 1e-10            # one value per face: conservative
