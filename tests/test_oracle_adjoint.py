"""Pins for the oracle's discrete adjoint: dense Jacobians from the forward
oracle, central finite differences and the dot-product identity."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2404_03399_amd import workloads as W
from oracle import adjoint, stepper


def _small(scheme="adg_at", rk="rk4", p=2, ne=12, pe=3, flux="upwind", per_stage=True, seed=5, speed=1.0):
    dt = 0.02 * W.TWO_PI / ne
    return W.Workload(name="adj", scheme=scheme, rk=rk, degree=p, n_elem=ne, pe_size=pe, flux=flux,
                      probs=("0.3", "0.3", "0.4"), seed=seed, per_stage=per_stage, dt=dt, speed=speed,
                      ic=W.PAPER_MULTISINE)


@pytest.mark.parametrize("scheme", ["dg", "adg", "adg_at"])
@pytest.mark.parametrize("rk", ["heun", "ssprk3", "rk4", "lsrk3", "lsrk4"])
def test_gradient_equals_dense_jacobian_transpose(scheme, rk):
    w = _small(scheme=scheme, rk=rk)
    n = 9
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(1).standard_normal(u0.shape)
    g = adjoint.dense_step_map(w, n)
    ut_dense = (g @ u0.ravel()).reshape(u0.shape)
    ut, grad, _ = adjoint.gradient(w, u0, n, adjoint.misfit_cotangent(ref))
    np.testing.assert_allclose(ut, ut_dense, rtol=0, atol=1e-13)
    expect = g.T @ (ut_dense - ref).ravel()
    np.testing.assert_allclose(grad.ravel(), expect, rtol=0, atol=1e-12 * np.max(np.abs(expect)))


@pytest.mark.parametrize("flux", ["upwind", "central"])
def test_dot_product_identity(flux):
    w = _small(flux=flux, p=3, ne=16, pe=4)
    n = 7
    rng = np.random.default_rng(3)
    v = rng.standard_normal((w.n_elem, w.degree + 1))
    c = rng.standard_normal(v.shape)
    # <G v, c> == <v, G^T c> with G^T c from the adjoint (cotangent c, linear map)
    gv = stepper.Stepper(w).run(v, n)
    _, gtc, _ = adjoint.gradient(w, v, n, lambda ut: c)
    lhs, rhs = float(np.sum(gv * c)), float(np.sum(v * gtc))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def _J(w, u0, n, ref):
    ut = stepper.Stepper(w).run(u0, n)
    return 0.5 * float(np.sum((ut - ref) ** 2))


def test_speed_gradient_central_difference():
    w = _small(p=2)
    n = 10
    u0 = stepper.initial_state(w)
    ref = np.zeros_like(u0)
    _, _, dja = adjoint.gradient(w, u0, n, adjoint.misfit_cotangent(ref))
    h = 1e-5
    fd = (_J(replace(w, speed=w.speed + h), u0, n, ref) - _J(replace(w, speed=w.speed - h), u0, n, ref)) / (2 * h)
    assert abs(dja - fd) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("per_stage", [True, False])
def test_burgers_gradient_central_difference(per_stage):
    ne = 16
    w = W.c3_burgers(n_elem=ne, n_steps=0, sigma=0.02)
    w = replace(w, pe_size=4, per_stage=per_stage)
    n = 12
    u0 = stepper.initial_state(w)
    ref = 0.3 * np.ones_like(u0)
    _, grad, _ = adjoint.gradient(w, u0, n, adjoint.misfit_cotangent(ref))
    rng = np.random.default_rng(7)
    d = rng.standard_normal(u0.shape)
    h = 1e-6
    fd = (_J(w, u0 + h * d, n, ref) - _J(w, u0 - h * d, n, ref)) / (2 * h)
    assert abs(float(np.sum(grad * d)) - fd) <= 1e-6 * max(1.0, abs(fd))


def test_initial_state_gradient_exact_for_quadratic_misfit():
    # J is quadratic in u0 for linear advection: the central difference is
    # exact up to rounding for any step
    w = _small(p=1, ne=10, pe=5, rk="heun")
    n = 6
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(2).standard_normal(u0.shape)
    _, grad, _ = adjoint.gradient(w, u0, n, adjoint.misfit_cotangent(ref))
    d = np.random.default_rng(8).standard_normal(u0.shape)
    h = 0.5
    fd = (_J(w, u0 + h * d, n, ref) - _J(w, u0 - h * d, n, ref)) / (2 * h)
    assert abs(float(np.sum(grad * d)) - fd) <= 1e-11 * max(1.0, abs(fd))
