"""Pins for the oracle's reference-element operators (paper Sec. 2).

Each check is fixed by calculus or by the paper's definitions, not by the
oracle's own formulas."""
import math

import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_nodes_closed_form(p):
    known = {
        1: [-1.0, 1.0],
        2: [-1.0, 0.0, 1.0],
        3: [-1.0, -1.0 / math.sqrt(5.0), 1.0 / math.sqrt(5.0), 1.0],
        4: [-1.0, -math.sqrt(3.0 / 7.0), 0.0, math.sqrt(3.0 / 7.0), 1.0],
    }
    np.testing.assert_allclose(basis.gll_nodes(p), known[p], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_is_cardinal(p):
    nodes = basis.gll_nodes(p)
    for j in range(p + 1):
        np.testing.assert_allclose(basis.lagrange(nodes, j, nodes), np.eye(p + 1)[j], atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mass_matrix(p):
    m = basis.mass_matrix(p)
    np.testing.assert_allclose(m, m.T, atol=1e-15)
    assert np.all(np.linalg.eigvalsh(m) > 0)
    # integral of 1 over [-1, 1] is 2; of xi^2 is 2/3
    one = np.ones(p + 1)
    assert abs(one @ m @ one - 2.0) < 1e-14
    x = basis.gll_nodes(p)
    assert abs(x @ m @ x - 2.0 / 3.0) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_summation_by_parts(p):
    # S + S^T = e_p e_p^T - e_0 e_0^T (integration by parts of phi_i phi_j)
    s = basis.stiffness_matrix(p)
    target = np.zeros((p + 1, p + 1))
    target[p, p] = 1.0
    target[0, 0] = -1.0
    np.testing.assert_allclose(s + s.T, target, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_weak_derivative_identity(p):
    # For any polynomial u of degree <= p:
    #   M^-1 S u = lift_r u(1) - lift_l u(-1) - u'   (integration by parts)
    d, ll, lr, w = basis.element_operators(p)
    x = basis.gll_nodes(p)
    for k in range(p + 1):
        u = x ** k
        du = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        np.testing.assert_allclose(d @ u, lr * 1.0 - ll * ((-1.0) ** k) - du, atol=1e-12)
    np.testing.assert_allclose(d @ np.ones(p + 1), lr - ll, atol=1e-13)
    # quadrature weights integrate polynomials of degree <= p exactly
    for k in range(p + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("bp,bm", [(1.0, 0.0), (0.5, 0.5)])
def test_flux_matrices_definitions(p, bp, bm):
    km, kp, kl, kr = basis.flux_matrices(p, bp, bm)
    # nodal basis with end-point nodes: phi_j(-1) = delta_j0, phi_j(1) = delta_jp
    e0 = np.eye(p + 1)[0]
    ep = np.eye(p + 1)[p]
    np.testing.assert_allclose(km, bp * np.outer(e0, ep), atol=1e-14)
    np.testing.assert_allclose(kp, -bm * np.outer(ep, e0), atol=1e-14)
    np.testing.assert_allclose(kl, bm * np.outer(e0, e0), atol=1e-14)
    np.testing.assert_allclose(kr, -bp * np.outer(ep, ep), atol=1e-14)
