"""Fourier-mode analysis (paper Sec. 4.2).

Test infrastructure only (see oracle/__init__.py).

* Synchronous: for a mode u^e = mu exp(i kappa x_e), one operator evaluation
  multiplies mu by Z = 2 sigma M^-1 (e^{-i theta} K^- + K_l + S + K_r
  + e^{i theta} K^+), theta = kappa dx (Sec. 4.2.1, first stage of the RK2
  derivation).  The amplification matrix G^s is obtained by pushing Z
  through the integrator's stage formulas.  Non-dimensional K = theta/(N_p+1),
  Omega = i ln(lambda) / (sigma (N_p + 1)).
* Asynchronous ADG(1)-RK2 with one-level delay: the block-companion matrix
  built from the coefficient matrices of Sec. 4.2.2, transcribed as printed
  (parity unpinned beyond the paper's qualitative statement at sigma = 0.333).
"""
from __future__ import annotations

import numpy as np

from . import basis


def _ops(p: int, flux: str):
    bp, bm = (1.0, 0.0) if flux == "upwind" else (0.5, 0.5)
    m = basis.mass_matrix(p)
    s = basis.stiffness_matrix(p)
    km, kp, kl, kr = basis.flux_matrices(p, bp, bm)
    return m, s, km, kp, kl, kr


def stage_matrix(p: int, flux: str, sigma: float, theta: float) -> np.ndarray:
    """Z(theta) = dt * L-hat for a = 1: 2 sigma M^-1 (e^{-i th} K^- + K_l + S + K_r + e^{i th} K^+)."""
    m, s, km, kp, kl, kr = _ops(p, flux)
    inner = np.exp(-1j * theta) * km + kl + s + kr + np.exp(1j * theta) * kp
    return 2.0 * sigma * np.linalg.solve(m, inner)


def amplification(p: int, rk: str, flux: str, sigma: float, theta: float) -> np.ndarray:
    """G^s: the integrator's stage formulas applied with the operator Z."""
    z = stage_matrix(p, flux, sigma, theta)
    eye = np.eye(p + 1)
    if rk == "heun":
        k1 = z
        k2 = z @ (eye + k1)
        return eye + 0.5 * (k1 + k2)
    if rk == "ssprk3":
        u1 = eye + z
        u2 = 0.75 * eye + 0.25 * (u1 + z @ u1)
        return eye / 3.0 + (2.0 / 3.0) * (u2 + z @ u2)
    if rk in ("lsrk3", "lsrk4"):
        from fractions import Fraction
        from .stepper import LOW_STORAGE
        du = np.zeros_like(eye, dtype=complex)
        g = eye.astype(complex)
        for a, b in zip(*LOW_STORAGE[rk]):
            du = float(Fraction(a)) * du + z @ g
            g = g + float(Fraction(b)) * du
        return g
    if rk == "rk4":
        k1 = z
        k2 = z @ (eye + 0.5 * k1)
        k3 = z @ (eye + 0.5 * k2)
        k4 = z @ (eye + k3)
        return eye + (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
    raise ValueError(rk)


def spectral_radius_max(p, rk, flux, sigma, n_theta=721):
    thetas = np.linspace(-np.pi, np.pi, n_theta)
    return max(np.max(np.abs(np.linalg.eigvals(amplification(p, rk, flux, sigma, t)))) for t in thetas)


def sigma_star(p, rk, flux="upwind", lo=1e-3, hi=2.0, tol=1e-5, n_theta=721):
    """Largest sigma with max_theta |lambda| <= 1 (bisection)."""
    def stable(s):
        return spectral_radius_max(p, rk, flux, s, n_theta) <= 1.0 + 1e-10
    if not stable(lo):
        return 0.0
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo


def dispersion(p, rk, flux, sigma, theta):
    """(K, Omega) for every eigenmode at theta = kappa dx."""
    lam = np.linalg.eigvals(amplification(p, rk, flux, sigma, theta))
    kk = theta / (p + 1)
    return kk, 1j * np.log(lam) / (sigma * (p + 1))


def paper_async_companion(sigma: float, theta: float, p: int = 1) -> np.ndarray:
    """Block-companion G^as of ADG(p)-RK2 with upwind flux and delay 1 at the
    left boundary, from the coefficient matrices of Sec. 4.2.2."""
    m, s, km, kp, kl, kr = _ops(p, "upwind")
    eye = np.eye(p + 1)
    inv = lambda a: 2.0 * sigma * np.linalg.solve(m, a)
    e1, em1 = np.exp(1j * theta), np.exp(-1j * theta)
    full = kl + s + kr
    k10_e = inv((s + kr) + e1 * kp)
    k11_e = inv(em1 * km + kl)
    k11_em1 = inv(np.exp(-2j * theta) * km + em1 * full + kp)
    k10_ep1 = inv(km + e1 * full + np.exp(2j * theta) * kp)
    k20_e = inv(kl @ k10_e + (s + kr) @ (eye + k10_e) + kp @ (e1 * eye + k10_ep1))
    k21_e = inv(km @ (em1 * eye + k11_em1) + kl @ (eye + k11_e) + (s + kr) @ k11_e)
    g_n = eye + 0.5 * (k10_e + k20_e)
    g_nm1 = 0.5 * (k11_e + k21_e)
    top = np.hstack([g_n, g_nm1])
    bot = np.hstack([eye, np.zeros_like(eye)])
    return np.vstack([top, bot])


def global_step_matrix(stepper_obj, n: int = 0) -> np.ndarray:
    """Dense matrix of one step of a (linear) stepper, column by column."""
    ne, npp = stepper_obj.n_elem, stepper_obj.np_
    size = ne * npp
    g = np.zeros((size, size))
    for c in range(size):
        e = np.zeros(size)
        e[c] = 1.0
        g[:, c] = stepper_obj.step(e.reshape(ne, npp), n).ravel()
    return g
