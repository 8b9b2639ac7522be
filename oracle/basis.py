"""Reference-element operators (paper Sec. 2, Eqs. for the element-wise weak
form and the reference matrices M, S, K-, K+, K_l, K_r).

Test infrastructure only (see oracle/__init__.py).

Readings:
* Node set: the paper uses Lagrange polynomials whose first and last nodes are
  the element end points (Sec. 2, Fig. 1) but does not name the interior
  nodes; we take Gauss-Lobatto-Legendre (GLL) nodes.
* The mass matrix is the exact integral (not lumped), as written.
All integrals are evaluated exactly with Gauss-Legendre quadrature on p+2
points (integrands are polynomials of degree <= 2p).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(p: int) -> np.ndarray:
    """xi_0 = -1 < ... < xi_p = 1: end points plus the roots of P_p'."""
    if p < 1:
        raise ValueError("degree must be >= 1")
    inner = npleg.Legendre.basis(p).deriv().roots() if p > 1 else np.array([])
    return np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))


def lagrange(nodes: np.ndarray, j: int, x: np.ndarray) -> np.ndarray:
    """phi_j(x) = prod_{m != j} (x - xi_m) / (xi_j - xi_m)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    for m, xm in enumerate(nodes):
        if m != j:
            out = out * (x - xm) / (nodes[j] - xm)
    return out


def lagrange_deriv(nodes: np.ndarray, j: int, x: np.ndarray) -> np.ndarray:
    """phi_j'(x) by the product rule over the factors of phi_j."""
    x = np.asarray(x, dtype=np.float64)
    total = np.zeros_like(x)
    others = [m for m in range(len(nodes)) if m != j]
    for skip in others:
        term = np.ones_like(x) / (nodes[j] - nodes[skip])
        for m in others:
            if m != skip:
                term = term * (x - nodes[m]) / (nodes[j] - nodes[m])
        total = total + term
    return total


def _quad(p: int):
    return npleg.leggauss(p + 2)


def mass_matrix(p: int) -> np.ndarray:
    """[M]_ij = int_{-1}^{1} phi_j phi_i dxi."""
    nodes = gll_nodes(p)
    xq, wq = _quad(p)
    phi = np.array([lagrange(nodes, j, xq) for j in range(p + 1)])
    return np.einsum("iq,jq,q->ij", phi, phi, wq)


def stiffness_matrix(p: int) -> np.ndarray:
    """[S]_ij = int_{-1}^{1} phi_j dphi_i/dxi dxi."""
    nodes = gll_nodes(p)
    xq, wq = _quad(p)
    phi = np.array([lagrange(nodes, j, xq) for j in range(p + 1)])
    dphi = np.array([lagrange_deriv(nodes, i, xq) for i in range(p + 1)])
    return np.einsum("iq,jq,q->ij", dphi, phi, wq)


def flux_matrices(p: int, b_plus: float, b_minus: float):
    """K^-, K^+, K_l, K_r of the reference weak form:
    [K^-]_ij = B+ phi_j(1) phi_i(-1),  [K^+]_ij = -B- phi_j(-1) phi_i(1),
    [K_l]_ij = B- phi_j(-1) phi_i(-1), [K_r]_ij = -B+ phi_j(1) phi_i(1)."""
    nodes = gll_nodes(p)
    at_m1 = np.array([lagrange(nodes, j, np.array(-1.0)) for j in range(p + 1)])
    at_p1 = np.array([lagrange(nodes, j, np.array(1.0)) for j in range(p + 1)])
    k_minus = b_plus * np.outer(at_m1, at_p1)      # row i: phi_i(-1), col j: phi_j(1)
    k_plus = -b_minus * np.outer(at_p1, at_m1)
    k_l = b_minus * np.outer(at_m1, at_m1)
    k_r = -b_plus * np.outer(at_p1, at_p1)
    return k_minus, k_plus, k_l, k_r


def element_operators(p: int):
    """Operators of the collapsed element update used by the stepper:
    D = M^-1 S, lift_l = M^-1 phi(-1), lift_r = M^-1 phi(1), quadrature
    weights w = M 1 (so that int u_h dxi = w^T u)."""
    m = mass_matrix(p)
    s = stiffness_matrix(p)
    nodes = gll_nodes(p)
    at_m1 = np.array([lagrange(nodes, j, np.array(-1.0)) for j in range(p + 1)])
    at_p1 = np.array([lagrange(nodes, j, np.array(1.0)) for j in range(p + 1)])
    d = np.linalg.solve(m, s)
    lift_l = np.linalg.solve(m, at_m1)
    lift_r = np.linalg.solve(m, at_p1)
    w = m @ np.ones(p + 1)
    return d, lift_l, lift_r, w


def element_nodes(x_left: float, length: float, n_elem: int, p: int) -> np.ndarray:
    """Physical node positions X[e, j] = x_e + (xi_j + 1) dx / 2, from the map
    xi(x) = (2x - x_e - x_{e+1}) / dx."""
    dx = length / n_elem
    xe = x_left + dx * np.arange(n_elem)
    return xe[:, None] + (gll_nodes(p)[None, :] + 1.0) * (dx / 2.0)
