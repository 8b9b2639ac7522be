"""Statistical scaling experiments of Section 6.2 on the batched engine.

The ensemble-averaged overall error <E-bar> (Sec. 4.3: spatial mean of
|u_h - u_exact| over all nodal values, averaged over delay realizations) of
the two AT schemes of Figs. 9-10, ADG(1)-AT2-RK2 at sigma = 0.1 and
ADG(3)-AT4-RK4 at sigma = 0.01, for linear advection with the Section 6
initial data:

* `error_vs_pe`: <E-bar> against the mesh for P = 2..32 PEs (Fig. 9): the AT
  schemes keep their order (slopes -2 and -4 in N_E) and, where asynchrony
  dominates, the error grows linearly with P (the Sec. 5 scaling
  <E_f> ~ (P / N_E) dt^a sum_m gamma_m E[k^m]).
* `error_vs_delay`: <E-bar> against the maximum delay L with p_k = 1/L
  (Fig. 10), fitted against the delay moment of the AT remainder,
  E[k (k+1) ... (k+q-1)] (E[k^2] + E[k] for q = 2; E[k^4] + 6E[k^3] +
  11E[k^2] + 6E[k] for q = 4).
* `async_vs_pe`, `async_vs_delay`: the same two experiments through the
  asynchrony term alone, <|u_AT - u_DG|> against the synchronous run of the
  same mesh.  For AT4 at sigma = 0.01 the asynchrony error is 10^-4 of the
  discretization error, so the excess of <E> over DG is lost to
  cancellation, while the term itself (1e-11 to 1e-10 at N_E = 64) is far
  above rounding.
* `error_caa`: the deterministic communication-avoiding cycle of Sec. 7
  against synchronous DG over the mesh.
* `viscous_burgers_convergence`: LDG(2)-RK2 and ALDG(2)-AT2-RK2 for the
  viscous Burgers equation (Fig. 11) against a finer synchronous run.

Every realization of one mesh runs in one batched context (one launch per
step for all of them); the statistics come from adg_ensemble_stats.  The
paper uses 5 realizations per point; the defaults here use 32.

    python -m paper_2404_03399_amd.experiments          # both figures, JSON
"""
from __future__ import annotations

import json
import math
import sys
import time
from dataclasses import replace
from fractions import Fraction
from typing import Dict, List, Sequence

from . import workloads as W

PE_COUNTS = (2, 4, 8, 16, 32)
STABLE_ERROR = 0.1  # <E> of a run still inside the stability region (|u0| <= 3)


# ---- analysis (host arithmetic on the measured errors) -----------------------
def delay_moment(probs: Sequence, q: int) -> Fraction:
    """E[k (k+1) ... (k+q-1)] for delays k = 0..L-1 with probabilities probs:
    the delay dependence of the leading AT remainder (Sec. 5), exact."""
    acc = Fraction(0)
    for k, p in enumerate(probs):
        term = Fraction(1)
        for i in range(q):
            term *= k + i
        acc += Fraction(p) * term
    return acc


def mean_delay(probs: Sequence) -> Fraction:
    return sum((Fraction(p) * k for k, p in enumerate(probs)), Fraction(0))


def loglog_slope(xs: Sequence[float], ys: Sequence[float]) -> float:
    """Least-squares slope of log y against log x."""
    lx = [math.log(x) for x in xs]
    ly = [math.log(y) for y in ys]
    mx, my = sum(lx) / len(lx), sum(ly) / len(ly)
    sxx = sum((a - mx) ** 2 for a in lx)
    sxy = sum((a - mx) * (b - my) for a, b in zip(lx, ly))
    return sxy / sxx


def loglog_slope_se(xs: Sequence[float], ys: Sequence[float], ses: Sequence[float]):
    """Weighted least-squares slope of log y against log x, each point
    weighted by the inverse variance of log y (standard error se of the mean
    y, delta method: var(log y) = (se / y)^2), and the slope's standard
    error."""
    lx = [math.log(x) for x in xs]
    ly = [math.log(y) for y in ys]
    w = [(y / se) ** 2 for y, se in zip(ys, ses)]
    sw = sum(w)
    mx = sum(wi * a for wi, a in zip(w, lx)) / sw
    my = sum(wi * b for wi, b in zip(w, ly)) / sw
    sxx = sum(wi * (a - mx) ** 2 for wi, a in zip(w, lx))
    sxy = sum(wi * (a - mx) * (b - my) for wi, a, b in zip(w, lx, ly))
    return sxy / sxx, math.sqrt(1.0 / sxx)


def linear_fit(xs: Sequence[float], ys: Sequence[float]) -> Dict[str, float]:
    """y = c0 + c1 x by least squares, with R^2."""
    n = len(xs)
    mx, my = sum(xs) / n, sum(ys) / n
    sxx = sum((x - mx) ** 2 for x in xs)
    sxy = sum((x - mx) * (y - my) for x, y in zip(xs, ys))
    c1 = sxy / sxx
    c0 = my - c1 * mx
    ss_res = sum((y - c0 - c1 * x) ** 2 for x, y in zip(xs, ys))
    ss_tot = sum((y - my) ** 2 for y in ys)
    return {"c0": c0, "c1": c1, "r2": 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0}


# ---- runs -----------------------------------------------------------------
def run_groups(workloads, group_of, n_groups: int, t_final: float):
    """Advance every problem to t_final in one batched context and return,
    per group, (mean <E>, variance of <E>, mean max-error, its variance)
    against the exact solution u0(x - a t_final)."""
    from .solver import Solver

    n_steps = {w.n_steps for w in workloads}
    if len(n_steps) != 1:
        raise ValueError("problems of one context must take the same number of steps")
    s = Solver(workloads)
    try:
        u = s.initial_state()
        s.run(u, n_steps.pop(), graph=True)
        ref = s.exact_advection_state(t_final)
        return s.ensemble_stats(u, ref, group_of, n_groups)
    finally:
        s.close()


def synchronous_twin(w):
    """The synchronous DG run of w's mesh, integrator and step (one PE)."""
    return replace(w, scheme="dg", at_levels=0, probs=("1",), pe_size=w.n_elem, caa=False,
                   name=f"{w.name}_dg")


def run_groups_async(workloads, group_of, n_groups: int):
    """Advance every problem in one batched context and return, per group,
    the statistics of the asynchrony term <|u - u_DG|>: each asynchronous
    run against the synchronous DG run of its own mesh (same integrator,
    step and initial data).  Both share the spatial and temporal
    discretization error, so the difference isolates the error that the
    delayed PE-face fluxes add (the E_f part of the Sec. 4.3 error split),
    which a difference of two errors against the exact solution can hide by
    cancellation."""
    from .solver import Solver

    n_steps = {w.n_steps for w in workloads}
    if len(n_steps) != 1:
        raise ValueError("problems of one context must take the same number of steps")
    n = n_steps.pop()
    s = Solver(workloads)
    try:
        u = s.initial_state()
        s.run(u, n, graph=True)
        ref = s.empty_state()
        twins = {}
        for i, w in enumerate(workloads):
            key = (w.n_elem, w.degree, w.rk, w.dt)
            if key not in twins:
                sd = Solver(synchronous_twin(w))
                try:
                    ud = sd.initial_state()
                    sd.run(ud, n, graph=True)
                    twins[key] = sd.view(ud, 0).clone()
                finally:
                    sd.close()
            s.view(ref, i).copy_(twins[key])
        return s.ensemble_stats(u, ref, group_of, n_groups)
    finally:
        s.close()


def async_vs_pe(scheme_key: str = "at4", n_elem: int = 64, pe_counts=PE_COUNTS, n_real: int = 32,
                probs=W.DELAYS_FIG9, t_final: float = 1.0) -> dict:
    """Fig. 9 through the asynchrony term alone: <|u_AT - u_DG|> against P at
    one mesh; the Sec. 5 scaling <E_f> ~ (P / N_E) dt^a sum gamma_m E[k^m]
    predicts slope 1 in P."""
    ws, grp = W.error_vs_pe_workloads(scheme_key, n_elem, pe_counts, n_real, probs, t_final)
    st = run_groups_async(ws, grp, len(pe_counts))
    mean = [x[0] for x in st]
    std = [math.sqrt(max(x[1], 0.0)) for x in st]
    out = {"scheme": scheme_key, **W.SCALING_SCHEMES[scheme_key], "n_elem": n_elem, "probs": list(probs),
           "t_final": t_final, "n_real": n_real, "pe_counts": list(pe_counts), "async_mean": mean,
           "async_std": std, "slope_vs_pe": None, "slope_se": None}
    if min(mean) > 0:
        # the term varies strongly between delay realizations: the slope
        # carries the standard errors of the means (std / sqrt(n_real))
        slope, se = loglog_slope_se(pe_counts, mean, [sd / math.sqrt(n_real) for sd in std])
        out.update({"slope_vs_pe": slope, "slope_se": se})
    return out


def async_vs_delay(scheme_key: str = "at4", n_elem: int = 128, n_pe: int = 16, delay_counts=(1, 2, 3, 4),
                   n_real: int = 32, sigma: float = 0.005, t_final: float = 1.0) -> dict:
    """Fig. 10 through the asynchrony term alone: <|u_AT - u_DG|> against the
    maximum delay L (uniform p_k), beside the delay moment of the AT remainder
    E[k (k+1) ... (k+q-1)] (zero for L = 1, where the run equals DG), and
    the ratio of the two (constant where the leading remainder dominates)."""
    q = W.SCALING_SCHEMES[scheme_key]["degree"] + 1
    ws, grp = W.error_vs_delay_workloads(scheme_key, n_elem, n_pe, delay_counts, n_real, t_final, sigma=sigma)
    st = run_groups_async(ws, grp, len(delay_counts))
    mean = [x[0] for x in st]
    moments = [float(delay_moment(W.uniform_probs(L), q)) for L in delay_counts]
    stable = [math.isfinite(m) and m < STABLE_ERROR for m in mean]
    return {"scheme": scheme_key, "degree": W.SCALING_SCHEMES[scheme_key]["degree"],
            "rk": W.SCALING_SCHEMES[scheme_key]["rk"], "sigma": sigma, "n_elem": n_elem, "n_pe": n_pe,
            "t_final": t_final, "n_real": n_real, "q": q, "delay_counts": list(delay_counts),
            "async_mean": mean, "async_std": [math.sqrt(max(x[1], 0.0)) if math.isfinite(x[1]) else None
                                              for x in st],
            "delay_moment": moments, "stable": stable,
            "ratio_to_moment": [m / d if d > 0 and ok else None for m, d, ok in zip(mean, moments, stable)]}


def sync_error(scheme_key: str, n_elem: int, t_final: float) -> float:
    """<E> of the synchronous DG scheme on the same mesh (no delays)."""
    w = W.scaling_workload(scheme_key, n_elem, 1, ("1",), 0, t_final, scheme="dg")
    return run_groups([w], [0], 1, t_final)[0][0]


def error_vs_pe(scheme_key: str = "at2", n_elems=(64, 128, 256, 512, 1024), pe_counts=PE_COUNTS,
                n_real: int = 32, probs=W.DELAYS_FIG9, t_final: float = 1.0) -> dict:
    """Fig. 9: <E-bar> for every (N_E, P) plus the synchronous DG error."""
    table = []
    for ne in n_elems:
        ws, grp = W.error_vs_pe_workloads(scheme_key, ne, pe_counts, n_real, probs, t_final)
        stats = run_groups(ws, grp, len(pe_counts), t_final)
        table.append({"n_elem": ne, "dg": sync_error(scheme_key, ne, t_final),
                      "mean": [st[0] for st in stats], "std": [math.sqrt(max(st[1], 0.0)) for st in stats]})
    out = {"scheme": scheme_key, **W.SCALING_SCHEMES[scheme_key], "probs": list(probs), "t_final": t_final,
           "n_real": n_real, "pe_counts": list(pe_counts), "table": table}
    if len(n_elems) > 1:
        out["order_in_n_elem"] = [loglog_slope(n_elems, [row["mean"][g] for row in table])
                                  for g in range(len(pe_counts))]
        out["order_in_n_elem_dg"] = loglog_slope(n_elems, [row["dg"] for row in table])
    last = table[-1]
    excess = [m - last["dg"] for m in last["mean"]]
    out["inset"] = {"n_elem": last["n_elem"], "mean": last["mean"], "excess_over_dg": excess,
                    "slope_excess_vs_pe": loglog_slope(pe_counts, excess) if min(excess) > 0 else None,
                    "slope_mean_vs_pe": loglog_slope(pe_counts, last["mean"])}
    return out


def error_vs_delay(scheme_key: str = "at2", n_elem: int = 512, n_pe: int = 16, delay_counts=(1, 2, 3, 4, 5),
                   n_real: int = 32, t_final: float = 1.0) -> dict:
    """Fig. 10: <E-bar> against L (uniform p_k) and its fit against the delay
    moment of the AT remainder."""
    q = W.SCALING_SCHEMES[scheme_key]["degree"] + 1
    ws, grp = W.error_vs_delay_workloads(scheme_key, n_elem, n_pe, delay_counts, n_real, t_final)
    stats = run_groups(ws, grp, len(delay_counts), t_final)
    means = [st[0] for st in stats]
    moments = [float(delay_moment(W.uniform_probs(L), q)) for L in delay_counts]
    # a run that left the scheme's stability region (Sec. 4.2.2: the region
    # shrinks as L grows) has errors of the size of the solution or NaN
    stable = [math.isfinite(m) and m < STABLE_ERROR for m in means]
    idx = [i for i, ok in enumerate(stable) if ok]
    fit = linear_fit([moments[i] for i in idx], [means[i] for i in idx]) if len(idx) > 2 else None
    return {"scheme": scheme_key, **W.SCALING_SCHEMES[scheme_key], "n_elem": n_elem, "n_pe": n_pe,
            "t_final": t_final, "n_real": n_real, "q": q, "delay_counts": list(delay_counts),
            "mean": means, "std": [math.sqrt(max(st[1], 0.0)) if math.isfinite(st[1]) else None for st in stats],
            "delay_moment": moments, "stable": stable, "fit": fit}


def error_caa(scheme_key: str = "at2", n_elems=(64, 128, 256, 512, 1024), n_pe: int = 8,
              t_final: float = 1.0) -> dict:
    """The communication-avoiding cycle of Sec. 7 (delays 0, 0, 0, 1, 2 by
    step mod 5; deterministic, so one run per mesh) against synchronous DG:
    the AT scheme keeps its order and DG-level errors."""
    at, dg = [], []
    for ne in n_elems:
        w = W.scaling_workload(scheme_key, ne, n_pe, W.DELAYS_UNIFORM3, 0, t_final)
        w = W.replace(w, caa=True, name=f"caa_{scheme_key}_{ne}")
        at.append(run_groups([w], [0], 1, t_final)[0][0])
        dg.append(sync_error(scheme_key, ne, t_final))
    return {"scheme": scheme_key, **W.SCALING_SCHEMES[scheme_key], "n_pe": n_pe, "n_elems": list(n_elems),
            "caa": at, "dg": dg, "order_caa": loglog_slope(n_elems, at), "order_dg": loglog_slope(n_elems, dg),
            "ratio_to_dg": [a / d for a, d in zip(at, dg)]}


def _eval_on(nodes_ref: "np.ndarray", u_ref, n_ref: int, x, length: float = W.TWO_PI):
    """Evaluate the reference DG solution (n_ref elements, Lagrange basis on
    the nodes nodes_ref in [-1, 1]) at the points x (barycentric form)."""
    import numpy as np
    dxr = length / n_ref
    e = np.minimum((x // dxr).astype(np.int64), n_ref - 1)
    xi = 2.0 * (x - e * dxr) / dxr - 1.0
    m = len(nodes_ref)
    w = np.array([1.0 / np.prod([nodes_ref[j] - nodes_ref[k] for k in range(m) if k != j]) for j in range(m)])
    diff = xi[..., None] - nodes_ref
    exact = np.isclose(diff, 0.0, atol=1e-15)
    diff = np.where(exact, 1.0, diff)
    terms = w / diff
    vals = u_ref[e]                      # (..., m) nodal values of the containing element
    out = (terms * vals).sum(-1) / terms.sum(-1)
    hit = exact.any(-1)
    if hit.any():
        out[hit] = (vals * exact)[hit].sum(-1)
    return out


def viscous_burgers_convergence(n_elems=(32, 64, 128), ref_factor: int = 8, t_final: float = 0.1,
                                degree: int = 2) -> dict:
    """Fig. 11(b): <E> of LDG(2)-RK2 and ALDG(2)-AT2-RK2 against a synchronous
    LDG run on a mesh ref_factor times finer than the finest (same scheme and
    Courant number), evaluated at the coarse nodes."""
    import numpy as np
    from . import adg
    from .solver import Solver

    def run(w):
        s = Solver(w)
        try:
            u = s.initial_state()
            s.run(u, w.n_steps, graph=True)
            return s.unpack(u)[0]
        finally:
            s.close()

    n_ref = ref_factor * max(n_elems)
    wr = W.viscous_burgers_workload(n_ref, "dg", degree, t_final=t_final)
    u_ref = run(wr)
    xi = np.array(adg.adg_nodes(degree))
    out = {"n_elems": list(n_elems), "n_ref": n_ref, "t_final": t_final, "degree": degree,
           "nu": wr.viscosity, "sigma": 0.0005}
    for scheme in ("dg", "adg_at"):
        errs = []
        for ne in n_elems:
            w = W.viscous_burgers_workload(ne, scheme, degree, t_final=t_final)
            if abs(w.dt * w.n_steps - wr.dt * wr.n_steps) > 1e-12:
                raise ValueError("reference and run end at different times")
            u = run(w)
            dx = W.TWO_PI / ne
            x = np.arange(ne)[:, None] * dx + (xi[None, :] + 1.0) * dx / 2.0
            errs.append(float(np.mean(np.abs(u - _eval_on(xi, u_ref, n_ref, x)))))
        out[scheme] = errs
        out["order_" + scheme] = loglog_slope(n_elems, errs)
    return out


def burgers_convergence(n_elems=(256, 512, 1024, 2048, 4096), t_final: float = 0.5, n_pe: int = 16,
                        sigma: float = 0.01) -> dict:
    """Inviscid Burgers of the full-size Burgers configuration (p = 2, LLF,
    SSP-RK3, u0 = 0.5 + sin x, delays {0..3}, AT3) run to t_final before the
    shock on small meshes with n_pe PEs: mean |u - u_exact| at the nodes for
    synchronous DG and ADG-AT, and their orders in N_E."""
    from .solver import Solver

    out = {"n_elems": list(n_elems), "t_final": t_final, "n_pe": n_pe, "sigma": sigma}
    for scheme in ("dg", "adg_at"):
        errs = []
        for ne in n_elems:
            dt, n = W.time_step(W.TWO_PI, ne, sigma, 1.5, t_final)
            w = replace(W.c3_burgers(n_elem=ne, n_steps=n, sigma=sigma, scheme=scheme), dt=dt, pe_size=ne // n_pe)
            s = Solver(w)
            try:
                u = s.initial_state()
                s.run(u, n, graph=True)
                errs.append(float(s.error_stats(u, s.exact_burgers_state(t_final))[0][0]))
            finally:
                s.close()
        out[scheme] = errs
        out["order_" + scheme] = loglog_slope(n_elems, errs)
    return out


def main(argv=None) -> int:
    t0 = time.perf_counter()
    out = {"error_vs_pe": [error_vs_pe("at2", n_elems=(64, 128, 256, 512, 1024)),
                           error_vs_pe("at4", n_elems=(64, 128, 256, 512))],
           "error_vs_delay": [error_vs_delay("at2", n_elem=512), error_vs_delay("at4", n_elem=128)],
           "async_vs_pe": [async_vs_pe("at4", n_elem=64), async_vs_pe("at2", n_elem=1024)],
           "async_vs_delay": [async_vs_delay("at4", n_elem=128), async_vs_delay("at2", n_elem=512,
                                                                                delay_counts=(1, 2, 3, 4, 5),
                                                                                sigma=0.1)],
           "communication_avoiding": [error_caa("at2"), error_caa("at4", n_elems=(64, 128, 256, 512))],
           "viscous_burgers": viscous_burgers_convergence(),
           "burgers": burgers_convergence()}
    out["wall_s"] = time.perf_counter() - t0
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
