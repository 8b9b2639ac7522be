#!/usr/bin/env python3
"""Throughput of the ADG-AT forward step on one MI355X.

Workload: 1D linear advection on [0, 2 pi], 2^20 elements, degree 3, 4096
PEs of 256 elements, delays {0..3} with probabilities (0.5, 0.25, 0.15, 0.1)
drawn per (step, stage, boundary), ADG-AT with q = 4, classical RK4, FP64,
eight-mode multi-sine initial data (synthetic).  One bench step = one RK
time step of the whole hot path (all four stages, interior and PE faces,
delay draws, ring traffic); the fused step kernel is replayed from a
hipGraph.  Metric: DOF-stage updates per second (N_E (p+1) S steps / s).

Prints ONE JSON line.  --gpus above 1 is rejected: the benchmark runs on
a single GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
BYTES_PER_DOF_STEP_FUSED = 16  # read u^n once, write u^{n+1} once (FP64)
BYTES_PER_DOF_STAGE_STAGEK = {"rk4": 34.0, "ssprk3": 64.0 / 3, "heun": 28.0}
FP64_VECTOR_PEAK_TFS = 78.6    # MI355X FP64 vector (no MFMA: the element operators are 4x4)


def fused_flops_per_elem_step(np_: int) -> int:
    """FP64 flops of one RK4 step of one element in the fused upwind kernel
    (halo recompute excluded): per stage the upwind flux a u^- (1), the lift
    and folded volume operator Kl F + Kdu y (np muls, np^2 FMAs); the RK4
    updates 13 np (FMA = 2 flops)."""
    return 4 * (2 * np_ * np_ + np_ + 1) + 13 * np_


FUSED_SOURCES = ("adg_fused.hip", "adg_device.hpp", "adg_common.hpp", "adg_launch.hpp")


def kernel_source_hash() -> str:
    """Hash of the sources the fused step kernel is compiled from."""
    h = hashlib.sha256()
    for name in FUSED_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2404_03399_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def ring_bytes_per_step(w) -> float:
    """PE-face ring traffic per step: each stage writes one flux per boundary
    and reads up to q past levels."""
    if w.scheme == "dg" or w.n_pe <= 1:
        return 0.0
    q = (w.at_levels or w.degree + 1) if w.scheme == "adg_at" else 1
    stages = {"rk4": 4, "ssprk3": 3, "heun": 2, "lsrk3": 3, "lsrk4": 5}[w.rk]
    return w.n_pe * stages * 8.0 * (1 + q)


def read_traffic(lane_elems: int, steps_per_launch: int, n_elem: int = 1 << 20, profile: str = ""):
    """HBM bytes per launch (or per advance of an ensemble) from a committed
    rocprofv3 PMC summary (by default the one of the single-problem mesh
    size), if it was taken on the current kernel source and holds a line for
    this launch shape."""
    tag = {1 << 20: "2p20", 1 << 24: "2p24"}.get(n_elem)
    name = profile or (f"pmc_fused_step_advection_{tag}.md" if tag else "")
    path = os.path.join(ROOT, "profiles", name)
    if not name or not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    # one line per measured launch shape
    for t in re.finditer(r"traffic_bytes_per_launch R=(\d+) K=(\d+):\s*([0-9.eE+]+)", text):
        if (int(t.group(1)), int(t.group(2))) == (lane_elems, steps_per_launch):
            return float(t.group(3))
    return None


def time_solver(torch, solver, u, steps, warmup, graph=True, reps=5):
    """GPU seconds of `steps` steps: the median over `reps` timed runs, each
    bracketed by HIP events on the stream the kernels are launched on.  The
    step graph is captured and the warm-up steps are run before the first
    event, so the timed region holds graph replays (and, for a step count
    that is not a multiple of the graph's 16, a few direct launches) only.
    Returns (median seconds, every rep's seconds, wall seconds of the reps)."""
    if graph:
        solver.capture_graph(u)
    solver.run(u, warmup, graph=graph)
    torch.cuda.synchronize()
    stream = solver.stream if solver.stream is not None else torch.cuda.current_stream()
    times = []
    t0 = time.perf_counter()
    for _ in range(reps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        solver.run(u, steps, graph=graph)
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) / 1e3)
    wall = time.perf_counter() - t0
    return statistics.median(times), times, wall


def fused_roofline(w, launch_s: float, R: int, K: int, traffic=None, note: str = ""):
    """Roofline block of the fused step kernel for workload w (one problem):
    algorithmic bytes per launch (u^n read once, u^{n+K} written once, K
    steps of PE-face ring traffic) and FP64 flops per launch (halo recompute
    excluded) over the measured launch duration, against the HBM and the FP64
    vector peaks; the binding roof is the larger fraction."""
    dofs = w.n_elem * (w.degree + 1)
    alg_bytes = BYTES_PER_DOF_STEP_FUSED * dofs + K * ring_bytes_per_step(w)
    achieved = alg_bytes / launch_s / 1e9
    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    flops = fused_flops_per_elem_step(w.degree + 1) * w.n_elem * K
    alu = {"bound": "alu", "achieved": flops / launch_s / 1e12, "peak": FP64_VECTOR_PEAK_TFS,
           "unit": "TFLOP/s", "frac": flops / launch_s / 1e12 / FP64_VECTOR_PEAK_TFS, "traffic": traffic}
    roof, other = (dict(alu), hbm) if alu["frac"] > hbm["frac"] else (dict(hbm), alu)
    roof["other_roof"] = {k: other[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roof.update({"kernel": f"k_fused_step<p={w.degree}, {w.rk}, {w.flux}, R={R} element(s) per lane, "
                           f"K={K} step(s) per launch>",
                 "alg_bytes_per_launch": alg_bytes, "alg_flops_per_launch": flops, "launch_us": launch_s * 1e6,
                 "steps_per_launch": K, "lane_elems": R, "note": note})
    return roof


def run_metrics(torch, s, w, u, n_done: int, sample_steps: int = 64):
    """Per-run metrics of the timed forward run: drift of the discrete
    integral of u over the run (conservation), and the histogram of the
    clamped delays the kernels draw, over the first sample_steps steps, beside
    the probabilities asked for."""
    import numpy as np
    u0 = s.initial_state()
    i0 = s.error_stats(u0, u0)[0][2]
    i1 = s.error_stats(u, u)[0][2]
    k = np.asarray(s.delay_schedule(0, 1000, sample_steps))  # past the start-up clamp
    counts = np.bincount(k.ravel(), minlength=w.n_delays)
    return {"steps": n_done, "integral_start": i0, "integral_end": i1, "integral_drift": abs(i1 - i0),
            "delay_histogram": {"sample_steps": sample_steps, "draws": int(k.size),
                                "fraction": (counts / k.size).tolist(), "asked": [float(p) for p in w.probs]}}


def _oracle_window(w, steps: int) -> float:
    """Seconds the FP64 oracle takes for a window of steps of w, one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import stepper
    u0 = stepper.initial_state(w)
    with threadpool_limits(1):
        st = stepper.Stepper(w)
        t0 = time.perf_counter()
        st.run(u0, steps)
        return time.perf_counter() - t0


def cpu_baseline(w, steps: int, procs: int = 0, proc_steps: int = 20):
    """The FP64 oracle on a bounded window of the same workload, one thread;
    then one process per host core (at most 16), each running a window of
    its own delay realization, for the aggregate rate of the host."""
    import multiprocessing as mp
    from dataclasses import replace
    dt = _oracle_window(w, steps)
    dof_stage = w.n_elem * (w.degree + 1) * 4 * steps
    out = {"value": dof_stage / dt, "unit": "DOF-stage/s", "cores": 1, "kind": "oracle",
           "sample": f"{steps} RK4 steps of the same 2^20-element ADG-AT problem ({dt:.1f} s, numpy FP64, 1 thread)"}
    procs = procs or min(16, os.cpu_count() or 1)
    if procs > 1:
        ws = [replace(w, seed=w.seed + 1 + i) for i in range(procs)]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(procs) as pool:  # fresh interpreters, no GPU state
            times = pool.starmap(_oracle_window, [(x, proc_steps) for x in ws])
        wall = time.perf_counter() - t0
        agg = procs * w.n_elem * (w.degree + 1) * 4 * proc_steps / max(times)
        out["all_cores"] = {"value": agg, "unit": "DOF-stage/s", "cores": procs, "kind": "oracle",
                            "sample": f"{procs} processes x {proc_steps} steps, one delay realization each "
                                      f"(slowest {max(times):.1f} s, {wall:.1f} s wall with start-up)"}
    return out


def _timed_adjoint(torch, s, n_steps, cot_of):
    u = s.initial_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(u, n_steps, graph=True, record=True)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    cot = cot_of(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, ga = s.adjoint(cot)
    torch.cuda.synchronize()
    return g, ga[0], t_fwd, time.perf_counter() - t0


def bench_adjoint(torch, W, Solver, n_steps: int, n_elem: int, stage: bool, large: bool = True):
    """Recorded forward + discrete adjoint of the misfit J = 1/2 ||u(T) - u_ref||^2
    against the exact solution for a speed 1% larger, u_ref = u0(x - 1.01 a T)
    (linear advection, ADG-AT, p=3, RK4, checkpoint every 64 steps): fused
    reverse-step kernel, and for comparison the per-stage reverse kernels on
    the same cotangent.  dJ/da is compared with its continuous-in-space-and-time
    value sum_nodes (u0(x - aT) - u_ref) (-T) u0'(x - aT)."""
    w = W.c5_adjoint_advection(n_elem=n_elem, n_steps=n_steps)
    T = n_steps * w.dt
    s = Solver(w, n_steps_record=n_steps, ckpt_every=64)
    u_ref = s.exact_advection_state(1.01 * T)
    cot_holder = {}

    def cot_of(u):
        cot_holder["cot"] = u - u_ref
        return cot_holder["cot"]

    g, ga, t_fwd, t_adj = _timed_adjoint(torch, s, n_steps, cot_of)
    xs = s.nodes(0) - w.speed * T
    du0 = torch.zeros_like(xs)
    for k, amp, ph in zip(w.ic.kappa, w.ic.amp, w.ic.phase):
        du0 = du0 + amp * k * torch.cos(k * xs + ph)
    ga_cont = float(((s.view(s.exact_advection_state(T)) - s.view(u_ref)) * (-T) * du0).sum())
    dofs = w.n_elem * (w.degree + 1)
    out = {"workload": f"ADG-AT(q=4) RK4 N_E={n_elem} p=3, {n_steps} steps, checkpoint every 64, "
                       f"J = 1/2 ||u(T) - u0(x - 1.01 a T)||^2",
           "reverse_dof_stage_per_s": dofs * 4 * n_steps / t_adj, "adjoint_s": t_adj,
           "recorded_forward_s": t_fwd, "dJ_da": ga, "dJ_da_continuous": ga_cont,
           "dJ_da_rel_diff": abs(ga - ga_cont) / abs(ga_cont),
           "grad_finite": bool(torch.isfinite(g).all().item())}
    # dJ/du0 only: linear advection needs no forward recomputation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g0, _ = s.adjoint(cot_holder["cot"], want_speed=False)
    torch.cuda.synchronize()
    t_u0 = time.perf_counter() - t0
    out["u0_only"] = {"reverse_dof_stage_per_s": dofs * 4 * n_steps / t_u0, "adjoint_s": t_u0,
                      "bitwise_equal_to_full": bool(torch.equal(s.view(g0), s.view(g)))}
    s.close()
    # every state resident (C = 1): the recorded forward writes each state
    # into its slot and the adjoint recomputes nothing
    s = Solver(w, n_steps_record=n_steps, ckpt_every=1)
    g1, ga1, t_fwd1, t_adj1 = _timed_adjoint(torch, s, n_steps, lambda u: cot_holder["cot"])
    out["all_states"] = {"reverse_dof_stage_per_s": dofs * 4 * n_steps / t_adj1, "adjoint_s": t_adj1,
                         "recorded_forward_s": t_fwd1, "resident_state_bytes": 8 * dofs * n_steps,
                         "bitwise_equal_to_c64": bool(torch.equal(s.view(g1), s.view(g))) and ga1 == ga}
    s.close()
    if stage:
        s = Solver(w, kernel="stage", n_steps_record=n_steps, ckpt_every=64)
        g2, ga2, _, t2 = _timed_adjoint(torch, s, n_steps, lambda u: cot_holder["cot"])
        out["stage_kernels"] = {"reverse_dof_stage_per_s": dofs * 4 * n_steps / t2, "adjoint_s": t2,
                                "grad_rel_l2_vs_fused": float(torch.linalg.vector_norm(g2 - g)
                                                              / torch.linalg.vector_norm(g)),
                                "dJ_da": ga2}
        s.close()
    out["burgers"] = bench_adjoint_burgers(torch, W, Solver, stage)
    out["roofline"] = adjoint_roofline(torch, W, Solver, n_elem)
    if large:
        out["roofline_large"] = adjoint_roofline(torch, W, Solver, 1 << 24)
    return out


def adjoint_roofline(torch, W, Solver, n_elem: int, n1: int = 64, n2: int = 128):
    """HBM fractions of the two reverse kernels on the headline problem at
    n_elem elements (linear advection ADG-AT, p = 3, RK4).  Two recordings of
    n1 and n2 steps; each adjoint call is timed with HIP events on the
    solver's stream (median of three), and the difference of the two calls
    per reverse launch drops the per-call copies and fills.  dJ/du0 only:
    k_adj_fused2, two reverse steps per launch, reads lambda^{n+2} and writes
    lambda^n (16 B per DOF); with dJ/da: k_adj_fused with the forward stages
    recomputed in registers, every state kept (checkpoint interval 1, so no
    segment is recomputed), reads u^n and lambda^{n+1} and writes lambda^n
    (24 B per DOF)."""
    dofs = n_elem * 4
    out = {"n_elem": n_elem}
    for key, want, ckpt, per, bytes_dof, kern in (
            ("two_step_reverse", False, 64, 2, 16, "k_adj_fused2<p=3, rk4, upwind, two steps, R=2>"),
            ("one_step_reverse_with_speed", True, 1, 1, 24, "k_adj_fused<p=3, rk4, upwind, forward stages kept>")):
        ts = {}
        for n in (n1, n2):
            w = W.c5_adjoint_advection(n_elem=n_elem, n_steps=n)
            s = Solver(w, n_steps_record=n, ckpt_every=ckpt)
            u = s.initial_state()
            s.run(u, n, graph=True, record=True)
            stream = s.stream if s.stream is not None else torch.cuda.current_stream()
            reps = []
            for _ in range(3):
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                g, _ = s.adjoint(u, want_speed=want)
                e1.record(stream)
                torch.cuda.synchronize()
                reps.append(e0.elapsed_time(e1) / 1e3)
            ts[n] = statistics.median(reps)
            s.close()
            del u, g
            torch.cuda.empty_cache()
        launch = (ts[n2] - ts[n1]) / ((n2 - n1) / per)
        alg = bytes_dof * dofs
        ach = alg / launch / 1e9
        out[key] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "kernel": kern, "launch_us": launch * 1e6, "alg_bytes_per_launch": alg,
                    "adjoint_call_s": {str(n1): ts[n1], str(n2): ts[n2]}}
    return out


def bench_adjoint_burgers(torch, W, Solver, stage: bool, n_elem: int = 1 << 18, n_steps: int = 512):
    """Discrete adjoint of inviscid Burgers (LLF, ADG-AT q=3, p=2, SSP-RK3,
    PEs of 256, checkpoint every 64) over a window of n_steps steps, with
    J = 1/2 ||u(T) - u(0)||^2: dJ/du0 through the nonlinear reverse step (the
    forward stages recomputed in registers), and the per-stage reverse
    kernels on the same cotangent for comparison."""
    w = W.c5_adjoint_burgers(n_elem=n_elem, n_steps=n_steps)
    dofs = w.n_elem * (w.degree + 1)
    s = Solver(w, n_steps_record=n_steps, ckpt_every=64)
    u_init = s.initial_state()
    holder = {}

    def cot_of(u):
        holder["cot"] = u - u_init
        return holder["cot"]

    g, _, t_fwd, t_adj = _timed_adjoint(torch, s, n_steps, cot_of)
    s.close()
    out = {"workload": f"Burgers LLF ADG-AT(q=3) SSP-RK3 N_E={n_elem} p=2, PE size 256, {n_steps}-step window, "
                       f"checkpoint every 64, J = 1/2 ||u(T) - u(0)||^2",
           "reverse_dof_stage_per_s": dofs * 3 * n_steps / t_adj, "adjoint_s": t_adj, "recorded_forward_s": t_fwd,
           "grad_finite": bool(torch.isfinite(g).all().item())}
    if stage:
        s = Solver(w, kernel="stage", n_steps_record=n_steps, ckpt_every=64)
        g2, _, _, t2 = _timed_adjoint(torch, s, n_steps, lambda u: holder["cot"])
        s.close()
        out["stage_kernels"] = {"reverse_dof_stage_per_s": dofs * 3 * n_steps / t2, "adjoint_s": t2,
                                "grad_rel_l2_vs_fused": float(torch.linalg.vector_norm(g2 - g)
                                                              / torch.linalg.vector_norm(g))}
    return out


def bench_experiments():
    """Sec. 6.2 scaling experiments on the batched engine (Figs. 9 and 10),
    summarised: orders in N_E per P, the P-dependence of the asynchrony error,
    and the fit of <E-bar> against the AT remainder's delay moment."""
    from paper_2404_03399_amd import experiments as X
    t0 = time.perf_counter()
    f9a = X.error_vs_pe("at2", n_elems=(64, 128, 256, 512, 1024))
    f9b = X.error_vs_pe("at4", n_elems=(64, 128, 256, 512))
    f10a = X.error_vs_delay("at2", n_elem=512, delay_counts=(1, 2, 3, 4, 5))
    f10b = X.error_vs_delay("at4", n_elem=128, delay_counts=(1, 2, 3, 4))
    a9 = X.async_vs_pe("at4", n_elem=64, n_real=256)
    a10 = X.async_vs_delay("at4", n_elem=128, delay_counts=(1, 2, 3, 4))
    caa = X.error_caa("at2")
    vb = X.viscous_burgers_convergence()
    bc = X.burgers_convergence()
    def slim(r):
        return {k: r[k] for k in ("n_elem", "n_pe", "delay_counts", "mean", "delay_moment", "stable", "fit")}
    return {"wall_s": time.perf_counter() - t0, "n_real": f9a["n_real"],
            "fig9_at2": {"order_in_n_elem": f9a["order_in_n_elem"], "order_dg": f9a["order_in_n_elem_dg"],
                         "inset_n_elem": f9a["inset"]["n_elem"], "inset_mean": f9a["inset"]["mean"],
                         "slope_excess_vs_pe": f9a["inset"]["slope_excess_vs_pe"]},
            "fig9_at4": {"order_in_n_elem": f9b["order_in_n_elem"], "order_dg": f9b["order_in_n_elem_dg"],
                         "inset_n_elem": f9b["inset"]["n_elem"], "inset_excess_over_dg": f9b["inset"]["excess_over_dg"]},
            "fig10_at2": slim(f10a), "fig10_at4": slim(f10b),
            "fig9_at4_async_term": {k: a9[k] for k in ("n_elem", "n_real", "pe_counts", "async_mean", "async_std",
                                                       "slope_vs_pe", "slope_se")},
            "fig10_at4_async_term": {k: a10[k] for k in ("n_elem", "n_pe", "sigma", "n_real", "delay_counts",
                                                         "async_mean", "delay_moment", "stable", "ratio_to_moment")},
            "caa_at2": {k: caa[k] for k in ("n_elems", "order_caa", "order_dg", "ratio_to_dg")},
            "fig11_viscous_burgers": {k: vb[k] for k in ("n_elems", "n_ref", "t_final", "dg", "adg_at",
                                                           "order_dg", "order_adg_at")},
            "burgers_to_half": {k: bc[k] for k in ("n_elems", "t_final", "n_pe", "dg", "adg_at",
                                                    "order_dg", "order_adg_at")}}


def bench_burgers(torch, W, Solver, n_elem: int = 1 << 22, steps: int = 200):
    """Full-size inviscid Burgers window: 2^22 elements, p=2, LLF, ADG-AT
    (q=3), SSP-RK3, 16384 PEs of 256, on the fused kernel at its tuned shape."""
    w = W.c3_burgers(n_elem=n_elem, n_steps=steps)
    s = Solver(w, lane_elems="auto")
    K, R = s.opt.fused_steps or 2, s.opt.lane_elems or 1
    u = s.initial_state()
    g, reps, _ = time_solver(torch, s, u, steps, 20)
    finite = bool(torch.isfinite(u).all().item())
    s.close()
    dofs = w.n_elem * (w.degree + 1)
    rate = dofs * 3 * steps / g
    step_bytes = BYTES_PER_DOF_STEP_FUSED * dofs / K + ring_bytes_per_step(w)
    return {"workload": f"Burgers LLF ADG-AT(q=3) SSP-RK3, N_E={n_elem}, p=2, PE size 256", "lane_elems": R,
            "steps_per_launch": K, "dof_stage_per_s": rate, "us_per_step": g / steps * 1e6,
            "rep_us_per_step": [t / steps * 1e6 for t in reps],
            "hbm_frac": step_bytes / (g / steps) / 1e9 / HBM_PEAK_GBS, "state_finite": finite}


# Local DG per-stage kernels, Heun: q pass reads Y and writes q (16 B/DOF);
# the flux pass reads Y and q (16 B) and the Heun registers (stage 0 writes A
# and Y, stage 1 reads U and A and writes U: 20 B on average).
BYTES_PER_DOF_STAGE_LDG_HEUN = 52.0


def bench_viscous_burgers(torch, W, Solver, n_elem: int = 1 << 20, steps: int = 200):
    """Throughput of ALDG(2)-AT2-RK2 (viscous Burgers, P = n_elem / 256) on
    the fused local DG kernel (K steps per launch: 16 B per DOF and launch
    plus the two PE-face rings) and on the per-stage kernels."""
    w = W.viscous_burgers_workload(n_elem, "adg_at", 2, t_final=1e-3)
    from dataclasses import replace
    w = replace(w, pe_size=256)
    dofs = w.n_elem * (w.degree + 1)
    out = {"workload": f"viscous Burgers ALDG(2)-AT2-RK2, N_E={n_elem}, PE size 256, nu={w.viscosity}"}
    finite = True
    for kernel in ("fused", "stage"):
        s = Solver(w, kernel=kernel)
        K = (s.opt.fused_steps or 2) if kernel == "fused" else 1
        u = s.initial_state()
        g, _, _ = time_solver(torch, s, u, steps, 20)
        finite = finite and bool(torch.isfinite(u).all().item())
        s.close()
        rate = dofs * 2 * steps / g
        if kernel == "fused":
            step_bytes = BYTES_PER_DOF_STEP_FUSED * dofs / K + 2 * ring_bytes_per_step(w)
            out.update({"dof_stage_per_s": rate, "us_per_step": g / steps * 1e6, "steps_per_launch": K,
                        "hbm_frac": step_bytes / (g / steps) / 1e9 / HBM_PEAK_GBS})
        else:
            out["stage_kernels"] = {"dof_stage_per_s": rate, "us_per_step": g / steps * 1e6,
                                    "hbm_frac_at_52B_per_dof_stage":
                                        rate * BYTES_PER_DOF_STAGE_LDG_HEUN / 1e9 / HBM_PEAK_GBS}
    out["fused_over_stage"] = out["dof_stage_per_s"] / out["stage_kernels"]["dof_stage_per_s"]
    out["state_finite"] = finite
    return out


def bench_ensemble(torch, W, Solver, n_steps: int, n_real: int, plain: bool, lane_elems: int = -1):
    """Batched ensemble (12 meshes x n_real delay realizations, one context,
    one launch per degree per step) against one context per problem."""
    ws = W.c4_ensemble(n_real=n_real, n_steps=n_steps)
    group = [int(w.name.split("_")[1][1:]) for w in ws]
    dofs = sum(w.n_elem * (w.degree + 1) for w in ws)
    s = Solver(ws, lane_elems="auto") if lane_elems < 0 else Solver(ws, lane_elems=lane_elems, fused_steps=2)
    R, K = s.opt.lane_elems or 2, s.opt.fused_steps or 2

    def timed(sv, uu, init, reps):
        # the step graph is captured on this buffer first; every rep restarts
        # from the initial state (reset outside the events), so the timed
        # region holds graph replays only and the last rep's final state is
        # the state after n_steps; median over reps (HIP events)
        sv.capture_graph(uu)
        stream = sv.stream if sv.stream is not None else torch.cuda.current_stream()
        times = []
        for _ in range(reps):
            uu.copy_(init)
            sv.reset()
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            sv.run(uu, n_steps, graph=True)
            ev1.record(stream)
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1) / 1e3)
        return statistics.median(times), times

    u_init = s.initial_state()
    u = u_init.clone()
    t_batched, reps_batched = timed(s, u, u_init, 5)
    # roofline of one K-step advance of the whole ensemble (up to eight range
    # launches of the fused step kernel, one per degree and form)
    alg = sum(BYTES_PER_DOF_STEP_FUSED * w.n_elem * (w.degree + 1) + K * ring_bytes_per_step(w) for w in ws)
    adv_s = t_batched * K / n_steps
    ach = alg / adv_s / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": read_traffic(R, K, profile="pmc_fused_step_ensemble_c4.md"),
            "kernel": f"k_fused_step over all degree ranges of one {K}-step advance (R={R})",
            "alg_bytes_per_advance": alg, "advance_us": adv_s * 1e6, "steps_per_launch": K, "lane_elems": R,
            "note": f"state 2 x {8 * dofs / 1e9:.2f} GB: HBM-resident"}
    # reference: exact solution of each problem at its own final time
    ref = s.empty_state()
    for i, w in enumerate(ws):
        x = s.nodes(i) - w.speed * n_steps * w.dt
        v = torch.zeros_like(x)
        for k, a, ph in zip(w.ic.kappa, w.ic.amp, w.ic.phase):
            v = v + a * torch.sin(k * x + ph)
        s.view(ref, i).copy_(v)
    gstats = s.ensemble_stats(u, ref, group, max(group) + 1)
    # the asynchrony term of each realization: its state against the
    # synchronous run of its own mesh (both share the discretization error)
    from paper_2404_03399_amd import experiments as X
    twins = {}
    ref_dg = s.empty_state()
    for i, w in enumerate(ws):
        key = (w.n_elem, w.degree, w.dt)
        if key not in twins:
            sd = Solver(X.synchronous_twin(w))
            ud = sd.initial_state()
            sd.run(ud, n_steps, graph=False)
            twins[key] = sd.view(ud, 0).clone()
            sd.close()
        s.view(ref_dg, i).copy_(twins[key])
    astats = s.ensemble_stats(u, ref_dg, group, max(group) + 1)
    out = {"workload": f"{len(set(group))} meshes x {n_real} realizations ({len(ws)} problems), "
                       f"{dofs} DOFs, {n_steps} RK4 steps, ADG-AT q=p+1",
           "lane_elems": R, "steps_per_launch": K,
           "batched_dof_stage_per_s": dofs * 4 * n_steps / t_batched, "batched_s": t_batched,
           "batched_rep_s": reps_batched, "roofline": roof,
           "per_mesh": [{"n_elem": ws[group.index(g)].n_elem, "degree": ws[group.index(g)].degree,
                         "mean_err": st[0], "var_err": st[1], "mean_linf": st[2], "var_linf": st[3],
                         "async_mean": at[0], "async_var": at[1], "async_linf_mean": at[2],
                         "async_linf_var": at[3]}
                        for g, (st, at) in enumerate(zip(gstats, astats))]}
    # launch structure: one fused launch per degree range (the library's
    # default) against one launch over every range (ADG_OPT_ONE_LAUNCH), both
    # at two elements per lane, two steps per launch and no PE-face split (the
    # shape the one-launch kernel supports)
    launches = {}
    for one in (False, True):
        so = Solver(ws, lane_elems=2, fused_steps=2, pe_split=False, one_launch=one)
        uo = u_init.clone()
        t1, reps1 = timed(so, uo, u_init, 3)
        launches["one_launch" if one else "per_range"] = {
            "batched_s": t1, "rep_s": reps1, "advance_us": t1 * 2 / n_steps * 1e6,
            "launches_per_advance": 1 if one else len({(w.degree, w.flux == "upwind" and w.speed > 0) for w in ws}),
            "bitwise_equal_to_tuned": bool(torch.equal(uo, u))}
        so.close()
    out["launch_structure"] = launches
    if plain:
        # one context per problem, same problems and kernels, each at its own
        # tuned launch shape (context set-up, tuning and graph capture
        # excluded on both sides; each problem's run timed by HIP events, so
        # host time between problems is not counted against the plain side)
        total = 0.0
        max_diff = 0.0
        for i, w in enumerate(ws):
            sp = Solver(w, lane_elems="auto")  # each problem at its own tuned shape
            ui = sp.empty_state()
            sp.view(ui, 0).copy_(s.view(u_init, i))
            uu = ui.clone()
            total += timed(sp, uu, ui, 1)[0]
            max_diff = max(max_diff, float((sp.view(uu, 0) - s.view(u, i)).abs().max()))
            sp.close()
        out["plain_dof_stage_per_s"] = dofs * 4 * n_steps / total
        out["plain_s"] = total
        out["batched_over_plain"] = total / t_batched
        out["max_abs_diff_batched_vs_plain"] = max_diff
        for v in launches.values():
            v["batched_over_plain"] = total / v["batched_s"]
    s.close()
    return out


def bench_large(torch, W, Solver, steps: int, n_elem: int = 1 << 24):
    """Config 2 over the Infinity Cache: 2^24 elements (2 x 537 MB of state),
    everything else as the headline workload, fused kernel at its tuned
    launch shape; with its own roofline block."""
    wl = W.c2_advection_large("adg_at", n_elem=n_elem)
    so = Solver(wl, lane_elems="auto")
    R, K = so.opt.lane_elems or 1, so.opt.fused_steps or 2
    uu = so.initial_state()
    g, reps, _ = time_solver(torch, so, uu, steps, 16)
    finite = bool(torch.isfinite(uu).all().item())
    so.close()
    dofs = wl.n_elem * (wl.degree + 1)
    return {"workload": f"linear advection ADG-AT(q=4) RK4, N_E={n_elem}, p=3, PE size 256 (P={wl.n_pe}), "
                        f"delays as the headline", "steps": steps,
            "dof_stage_per_s": dofs * 4 * steps / g, "us_per_step": g / steps * 1e6,
            "rep_us_per_step": [t / steps * 1e6 for t in reps], "state_finite": finite,
            "roofline": fused_roofline(wl, g * K / steps, R, K, read_traffic(R, K, n_elem),
                                       f"state 2 x {8 * dofs / 1e6:.0f} MB: HBM-resident")}


def copy_bandwidth(torch, mib: int = 1024, reps: int = 5):
    """A plain device-to-device copy of `mib` MiB (read + write), median of
    reps: the practical ceiling of a read-and-write stream on this GPU."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) / 1e3)
    t = statistics.median(times)
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * n * 8, "GBs": 2 * n * 8 / t / 1e9, "frac_of_hbm_peak": 2 * n * 8 / t / 1e9 / HBM_PEAK_GBS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel", default="fused", choices=["fused", "stage"])
    ap.add_argument("--n-elem", type=int, default=1 << 20)
    ap.add_argument("--lane-elems", type=int, default=-1,
                    help="fused kernel elements per lane (default: autotuned together with --fused-steps)")
    ap.add_argument("--fused-steps", type=int, default=0, help="fused kernel time steps per launch (0: default)")
    ap.add_argument("--extras", action="store_true", help="also time DG/ADG and the per-stage kernel")
    ap.add_argument("--no-large", action="store_true", help="skip the HBM-resident 2^24-element line")
    ap.add_argument("--large-steps", type=int, default=64)
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--ensemble-real", type=int, default=256)
    ap.add_argument("--ensemble-lane-elems", type=int, default=-1,
                    help="ensemble: elements per lane with two steps per launch (default: autotuned)")
    ap.add_argument("--ensemble-steps", type=int, default=500)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-context-per-problem ensemble run")
    ap.add_argument("--no-adjoint-stage", action="store_true", help="skip the per-stage adjoint comparison")
    ap.add_argument("--no-experiments", action="store_true",
                    help="skip the Sec. 6.2 scaling experiments and the Burgers / viscous Burgers timings")
    ap.add_argument("--no-scaling", action="store_true",
                    help="skip only the Sec. 6.2 scaling experiments (keep the Burgers / viscous Burgers timings)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2404_03399_amd import workloads as W
    from paper_2404_03399_amd.solver import Solver

    w = W.c2_advection_large("adg_at", n_elem=args.n_elem)
    s = Solver(w, kernel=args.kernel, lane_elems="auto" if args.lane_elems < 0 else args.lane_elems,
               fused_steps=args.fused_steps)
    K = (s.opt.fused_steps or 2) if args.kernel == "fused" else 1
    R = s.opt.lane_elems or 1
    u = s.initial_state()
    gpu_s, rep_s, wall = time_solver(torch, s, u, args.steps, args.warmup)
    dofs = w.n_elem * (w.degree + 1)
    stages = 4
    value = dofs * stages * args.steps / gpu_s
    finite = bool(torch.isfinite(u).all().item())
    cache_note = ("working set 2 x 33.6 MB fits the 256 MB Infinity Cache (see large_mesh for an "
                  "HBM-resident size)" if args.n_elem <= (1 << 22) else "HBM-resident")
    if args.kernel == "fused":
        launch_s = gpu_s * K / args.steps
        roof = fused_roofline(w, launch_s, R, K, read_traffic(R, K, args.n_elem), cache_note)
    else:
        launch_s = gpu_s / (args.steps * stages)
        alg_bytes = BYTES_PER_DOF_STAGE_STAGEK["rk4"] * dofs + ring_bytes_per_step(w) / stages
        achieved = alg_bytes / launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_stage<RK4, upwind, s> (mean over stages)",
                "alg_bytes_per_launch": alg_bytes, "launch_us": launch_s * 1e6, "note": cache_note}
    # The same throughput expressed at the per-stage kernels' byte model (34 B
    # per DOF-stage for RK4): the bandwidth an unfused stepper would need to
    # match it.  Not a roofline fraction (it exceeds 1 because the fused
    # kernel moves 16 B per DOF per launch, not 136 B per DOF per step).
    sm = BYTES_PER_DOF_STAGE_STAGEK["rk4"] * value / 1e9
    roof["unfused_equivalent"] = {"bytes_per_dof_stage": BYTES_PER_DOF_STAGE_STAGEK["rk4"],
                                  "equivalent_GBs": sm, "equivalent_over_hbm_peak": sm / HBM_PEAK_GBS,
                                  "note": "not a roofline fraction"}

    out = {
        "metric": "DOF-stage updates/s (fwd, adjoint) vs HBM roofline; batched vs plain",
        "value": value,
        "unit": "DOF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_s / args.steps * 1e3,
        "rep_ms_per_step": [t / args.steps * 1e3 for t in rep_s],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"linear advection ADG-AT(q=4) RK4, N_E={w.n_elem}, p=3, "
                               f"PE size 256 (P={w.n_pe}), delays {{0..3}} p=(0.5,0.25,0.15,0.1) per stage",
                   "n_elem": w.n_elem, "degree": 3, "pe_size": 256, "rk": "rk4", "scheme": "adg_at",
                   "kernel": args.kernel, "dofs": dofs},
        "roofline": roof,
        "timing": f"median of {len(rep_s)} timed runs of {args.steps} steps (HIP events on the kernels' stream; "
                  f"graph captured and {args.warmup} warm-up steps before the first event)",
        "wall_s": wall,
        "state_finite": finite,
        "run_metrics": run_metrics(torch, s, w, u, args.warmup + len(rep_s) * args.steps),
    }
    if args.extras:
        ex = {}
        for scheme in ("dg", "adg"):
            ws = W.c2_advection_large(scheme, n_elem=args.n_elem)
            so = Solver(ws)
            uu = so.initial_state()
            g, _, _ = time_solver(torch, so, uu, args.steps // 2, 20)
            ex[f"{scheme}_dof_stage_per_s"] = dofs * stages * (args.steps // 2) / g
            so.close()
        so = Solver(w, kernel="stage")
        uu = so.initial_state()
        g, _, _ = time_solver(torch, so, uu, args.steps // 2, 20)
        ex["stage_kernel_dof_stage_per_s"] = dofs * stages * (args.steps // 2) / g
        so.close()
        out["extras"] = ex
    if not args.no_large:
        out["large_mesh"] = bench_large(torch, W, Solver, args.large_steps)
    out["hbm_copy"] = copy_bandwidth(torch)
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes_each_way"] = n * 8
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(torch, W, Solver, args.adjoint_steps, args.n_elem,
                                       not args.no_adjoint_stage, not args.no_large)
    if not args.no_ensemble:
        out["ensemble"] = bench_ensemble(torch, W, Solver, args.ensemble_steps, args.ensemble_real,
                                         not args.no_plain, args.ensemble_lane_elems)
    if not args.no_experiments:
        if not args.no_scaling:
            out["experiments"] = bench_experiments()
        out["viscous_burgers"] = bench_viscous_burgers(torch, W, Solver)
        out["burgers"] = bench_burgers(torch, W, Solver)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
        out["cpu_baseline"]["host"] = {"cpu_count": os.cpu_count()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
