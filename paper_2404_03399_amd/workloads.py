"""Seeded synthetic workloads: problem parameters and random draws only.

This module is shared by the test oracle and by the device path.  It holds
no discretisation arithmetic: no nodes, no operators, no fluxes, no time
stepping, no delay binning.  It only says *which* problem to solve (mesh
size, degree, delay probabilities, seeds, initial-condition modes, time step)
so that both sides are fed identical inputs.

The paper benchmarks on no public dataset; every workload here is synthetic
and follows the shapes of the paper's experiments (Section 6: periodic domain
of length 2*pi, multi-sine initial data, P processing elements, maximum delay
L with probabilities p_k) scaled to the sizes named below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class MultiSine:
    """u0(x) = sum_i A_i sin(kappa_i x + phi_i) (Section 6.1, initial condition),
    plus a constant offset (used by the Burgers workload, u0 = 0.5 + sin x)."""
    kappa: Tuple[int, ...]
    amp: Tuple[float, ...]
    phase: Tuple[float, ...]
    offset: float = 0.0


@dataclass(frozen=True)
class Workload:
    """One problem instance.  Field names follow the paper's notation:
    n_elem = N_E, degree = N_p, pe_size = N_E / P, probs = {p_k} (L = len),
    speed = a, dt = Delta t."""
    name: str
    equation: str = "advection"      # "advection" | "burgers" | "viscous_burgers"
    scheme: str = "adg_at"           # "dg" | "adg" | "adg_at"
    flux: str = "upwind"             # "upwind" | "central" | "llf"
    rk: str = "rk4"                  # "heun" | "ssprk3" | "rk4"
    degree: int = 2
    n_elem: int = 64
    pe_size: int = 16
    probs: Tuple[str, ...] = ("1",)  # decimal strings, exact
    seed: int = 0
    per_stage: bool = True           # delay key includes the RK stage
    caa: bool = False                # delays follow the communication-avoiding cycle (L = 3)
    at_levels: int = 0               # q; 0 -> degree + 1
    x_left: float = 0.0
    length: float = TWO_PI
    speed: float = 1.0
    viscosity: float = 0.0           # nu of the viscous Burgers equation
    dt: float = 0.0
    n_steps: int = 0
    ic: MultiSine = field(default_factory=lambda: MultiSine((1,), (1.0,), (0.0,)))

    @property
    def n_delays(self) -> int:
        return len(self.probs)

    @property
    def n_pe(self) -> int:
        return self.n_elem // self.pe_size


def time_step(length: float, n_elem: int, sigma: float, a_max: float, t_final: float) -> Tuple[float, int]:
    """Fixed step reaching t_final exactly: dt = T / ceil(T a_max / (sigma dx)).
    Uniform dt is assumed by the AT construction (Section 5)."""
    dx = length / n_elem
    n = int(math.ceil(t_final * a_max / (sigma * dx) - 1e-12))
    return t_final / n, n


def multisine_draw(seed: int, n_modes: int, kmin: int, kmax: int) -> MultiSine:
    """kappa_i ~ U{kmin..kmax} (with replacement), A_i ~ N(0,1), phi_i ~ U[0, 2pi),
    drawn in that order from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    kappa = rng.integers(kmin, kmax + 1, size=n_modes)
    amp = rng.standard_normal(n_modes)
    phase = rng.uniform(0.0, TWO_PI, size=n_modes)
    return MultiSine(tuple(int(k) for k in kappa), tuple(float(a) for a in amp),
                     tuple(float(p) for p in phase))


# Multi-scale initial data of the paper's experiments: kappa = {2,3,5},
# A = {3,2,1}; the phases are not printed, these are fixed choices.
PAPER_MULTISINE = MultiSine((2, 3, 5), (3.0, 2.0, 1.0), (0.3, 1.1, 2.0))
SINE = MultiSine((1,), (1.0,), (0.0,))

DELAYS_C2 = ("0.5", "0.25", "0.15", "0.1")
DELAYS_UNIFORM3 = ("1/3", "1/3", "1/3")


def c1_advection_small(scheme: str = "adg_at", sigma: float = 0.1) -> Workload:
    """Linear advection, 64 elements, p=2, 4 PEs of 16, delays uniform in {0,1,2},
    RK4, u0 = sin x, T = 1."""
    dt, n = time_step(TWO_PI, 64, sigma, 1.0, 1.0)
    return Workload(name=f"c1_{scheme}_s{sigma}", scheme=scheme, degree=2, n_elem=64, pe_size=16,
                    probs=DELAYS_UNIFORM3, seed=0, dt=dt, n_steps=n, ic=SINE)


def c2_advection_large(scheme: str = "adg_at", n_elem: int = 1 << 20, n_steps: int = 1000,
                       sigma: float = 0.005) -> Workload:
    """Linear advection, 2^20 elements, p=3, PEs of 256, delays {0..3} with
    probabilities (0.5, 0.25, 0.15, 0.1), eight sine modes with kappa ~ U{1..32}
    and N(0,1) amplitudes, RK4."""
    dx = TWO_PI / n_elem
    return Workload(name=f"c2_{scheme}_{n_elem}", scheme=scheme, degree=3, n_elem=n_elem,
                    pe_size=256, probs=DELAYS_C2, seed=0, dt=sigma * dx, n_steps=n_steps,
                    ic=multisine_draw(0, 8, 1, 32))


def c3_burgers(n_elem: int = 1 << 22, n_steps: int = 1000, sigma: float = 0.01,
               scheme: str = "adg_at") -> Workload:
    """Inviscid Burgers, p=2, local Lax-Friedrichs, u0 = 0.5 + sin x, SSP-RK3,
    PEs of 256, delays {0..3} as in c2.  dt = sigma dx / max|u0|."""
    dx = TWO_PI / n_elem
    return Workload(name=f"c3_burgers_{n_elem}", equation="burgers", flux="llf", rk="ssprk3",
                    scheme=scheme, degree=2, n_elem=n_elem, pe_size=256, probs=DELAYS_C2,
                    seed=0, dt=sigma * dx / 1.5, n_steps=n_steps,
                    ic=MultiSine((1,), (1.0,), (0.0,), offset=0.5))


# Stable Courant numbers per degree for RK4 with per-stage delays in {0..3}.
SIGMA_BY_DEGREE = {1: 0.05, 2: 0.01, 3: 0.005, 4: 0.001}


def c4_ensemble(n_meshes: int = 12, n_real: int = 256, n_steps: int = 500,
                log2_min: float = 10.0, log2_max: float = 16.0, mesh_seed: int = 4) -> List[Workload]:
    """Batched ensemble: n_meshes linear-advection meshes with N_E = 64*round(2^U/64),
    U ~ U[log2_min, log2_max], p ~ U{1..4}, PE size 64, delays {0..3} with c2's
    probabilities, ADG-AT with q = p+1, RK4, n_steps steps; n_real delay
    realizations per mesh (seed = mesh * 2^32 + r)."""
    rng = np.random.default_rng(mesh_seed)
    us = rng.uniform(log2_min, log2_max, size=n_meshes)
    ps = rng.integers(1, 5, size=n_meshes)
    out = []
    for m in range(n_meshes):
        ne = max(64, 64 * int(round(2.0 ** us[m] / 64.0)))
        p = int(ps[m])
        dt = SIGMA_BY_DEGREE[p] * TWO_PI / ne
        for r in range(n_real):
            out.append(Workload(name=f"c4_m{m}_r{r}", degree=p, n_elem=ne, pe_size=64,
                                probs=DELAYS_C2, seed=(m << 32) | r, dt=dt, n_steps=n_steps,
                                ic=PAPER_MULTISINE))
    return out


def c5_adjoint_advection(n_elem: int = 1 << 20, n_steps: int = 2000, sigma: float = 0.005) -> Workload:
    """Adjoint workload: linear advection, p=3, RK4, ADG-AT, c2's delays."""
    w = c2_advection_large("adg_at", n_elem=n_elem, n_steps=n_steps, sigma=sigma)
    return replace(w, name=f"c5_adv_{n_elem}")


def c5_adjoint_burgers(n_elem: int = 1 << 18, n_steps: int = 1000, sigma: float = 0.01) -> Workload:
    w = c3_burgers(n_elem=n_elem, n_steps=n_steps, sigma=sigma)
    return replace(w, name=f"c5_burgers_{n_elem}")


# ---- statistical scaling experiments (Section 6.2, Figs. 9 and 10) ----------
# Initial data of the Section 6 advection experiments: kappa = {2, 3},
# A = {2, 1} (phases not printed: 0).
SCALING_IC = MultiSine((2, 3), (2.0, 1.0), (0.0, 0.0))
DELAYS_FIG9 = ("0.3", "0.4", "0.3")
# The two AT schemes of Figs. 9-10: ADG(1)-AT2-RK2 at sigma = 0.1 and
# ADG(3)-AT4-RK4 at sigma = 0.01.
SCALING_SCHEMES = {"at2": {"degree": 1, "rk": "heun", "sigma": 0.1},
                   "at4": {"degree": 3, "rk": "rk4", "sigma": 0.01}}


def uniform_probs(n_delays: int) -> Tuple[str, ...]:
    """p_k = 1/L for k = 0..L-1, as exact rationals."""
    return tuple(f"1/{n_delays}" for _ in range(n_delays))


def scaling_workload(scheme_key: str, n_elem: int, n_pe: int, probs, seed: int, t_final: float = 1.0,
                     scheme: str = "adg_at", name: str = "", sigma: float = 0.0) -> Workload:
    """One problem of the scaling experiments: linear advection a = 1 on
    [0, 2 pi), P = n_pe PEs, delays drawn once per step (Section 6.1);
    sigma overrides the scheme's Courant number."""
    cfg = SCALING_SCHEMES[scheme_key]
    dt, n = time_step(TWO_PI, n_elem, sigma or cfg["sigma"], 1.0, t_final)
    return Workload(name=name or f"{scheme_key}_{scheme}_N{n_elem}_P{n_pe}_s{seed}", scheme=scheme,
                    rk=cfg["rk"], degree=cfg["degree"], n_elem=n_elem, pe_size=n_elem // n_pe,
                    probs=tuple(probs), seed=seed, per_stage=False, dt=dt, n_steps=n, ic=SCALING_IC)


def error_vs_pe_workloads(scheme_key: str, n_elem: int, pe_counts, n_real: int, probs=DELAYS_FIG9,
                          t_final: float = 1.0, seed_base: int = 9, sigma: float = 0.0):
    """Fig. 9 at one mesh: n_real delay realizations for each P (group g =
    index of P).  Seeds are distinct across meshes, P and realizations."""
    out, group = [], []
    for g, npe in enumerate(pe_counts):
        for r in range(n_real):
            seed = (seed_base << 48) | (n_elem << 24) | (npe << 16) | r
            out.append(scaling_workload(scheme_key, n_elem, npe, probs, seed, t_final, sigma=sigma))
            group.append(g)
    return out, group


def error_vs_delay_workloads(scheme_key: str, n_elem: int, n_pe: int, delay_counts, n_real: int,
                             t_final: float = 1.0, seed_base: int = 10, sigma: float = 0.0):
    """Fig. 10: n_real realizations for each maximum delay L with uniform p_k
    (group g = index of L)."""
    out, group = [], []
    for g, nd in enumerate(delay_counts):
        for r in range(n_real):
            seed = (seed_base << 48) | (nd << 24) | r
            out.append(scaling_workload(scheme_key, n_elem, n_pe, uniform_probs(nd), seed, t_final, sigma=sigma))
            group.append(g)
    return out, group


# Viscous Burgers runs (Fig. 11): kappa = {2,3,5}, A = {3,2,1}, nu = 0.1,
# sigma = 0.0005, P = 4, L = 3 with p = (0.3, 0.4, 0.3), LDG(2) with RK2 and
# AT2 at the PE faces.  dt = sigma dx / a_max with a_max = sum |A| = 6.
VISCOUS_IC = MultiSine((2, 3, 5), (3.0, 2.0, 1.0), (0.3, 1.1, 2.0))


def viscous_burgers_workload(n_elem: int, scheme: str = "adg_at", degree: int = 2, nu: float = 0.1,
                             sigma: float = 0.0005, n_pe: int = 4, t_final: float = 0.1, seed: int = 0,
                             rk: str = "heun") -> Workload:
    """dt = sigma dx / a_max, capped by the explicit diffusive limit
    0.002 dx^2 / nu on fine meshes (it binds only above ~1500 elements)."""
    a_max = float(sum(abs(a) for a in VISCOUS_IC.amp))
    dx = TWO_PI / n_elem
    sig_eff = min(sigma, 0.002 * dx * a_max / nu) if nu > 0 else sigma
    dt, n = time_step(TWO_PI, n_elem, sig_eff, a_max, t_final)
    return Workload(name=f"vburgers_{scheme}_{n_elem}", equation="viscous_burgers", flux="llf", rk=rk,
                    scheme=scheme, degree=degree, n_elem=n_elem, pe_size=n_elem // n_pe, probs=DELAYS_FIG9,
                    seed=seed, per_stage=False, at_levels=2 if scheme == "adg_at" else 0, viscosity=nu,
                    dt=dt, n_steps=n, ic=VISCOUS_IC)


def random_coefficients(seed: int, shape) -> np.ndarray:
    """Generic N(0,1) FP64 array (cotangents, perturbation directions)."""
    return np.random.default_rng(seed).standard_normal(shape)
