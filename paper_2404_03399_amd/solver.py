"""PyTorch plumbing around the C ABI: device memory, streams, state packing.

torch supplies the device buffers (state, workspace) and the current HIP
stream; all arithmetic of the method runs in libadg's kernels.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import List, Sequence

import numpy as np
import torch

from . import adg


def delay_thresholds(probs: Sequence) -> List[int]:
    """Bin edges T_k = floor(2^53 (p_0 + ... + p_{k-1})), k = 1..L-1, from exact
    decimal/rational probabilities (delay = number of edges <= the uniform)."""
    ps = [Fraction(p) for p in probs]
    if any(p < 0 for p in ps) or sum(ps) != 1:
        raise ValueError("delay probabilities must be >= 0 and sum to 1")
    out, acc = [], Fraction(0)
    for p in ps[:-1]:
        acc += p
        out.append(math.floor(acc * (1 << 53)))
    return out


def to_problem(w) -> adg.adg_problem:
    """C descriptor of a workloads.Workload."""
    p = adg.adg_problem()
    p.abi_version = adg.ADG_ABI_VERSION
    p.equation = adg.EQUATION[w.equation]
    p.scheme = adg.SCHEME[w.scheme]
    p.flux = adg.FLUX[w.flux]
    p.rk = adg.RK[w.rk]
    p.degree = w.degree
    p.at_levels = w.at_levels if w.scheme == "adg_at" else 0
    p.n_delays = len(w.probs)
    p.delay_granularity = 2 if getattr(w, "caa", False) else (1 if w.per_stage else 0)
    p.reserved = 0
    p.n_elem = w.n_elem
    p.pe_size = w.pe_size
    p.seed = w.seed & ((1 << 64) - 1)
    thr = delay_thresholds(w.probs)
    for i, t in enumerate(thr):
        p.delay_threshold[i] = t
    p.x_left = w.x_left
    p.length = w.length
    p.speed = w.speed
    p.dt = w.dt
    p.viscosity = getattr(w, "viscosity", 0.0)
    return p


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Solver:
    """One context over one or more problems (batched when more than one)."""

    def __init__(self, workloads, kernel: str = "auto", n_steps_record: int = 0, ckpt_every: int = 0,
                 device: str = "cuda", stream=None, lane_elems=0, fused_steps: int = 0, scratch: bool = False,
                 pe_split=None, one_launch: bool = False):
        """scratch: take the library's static device workspace (adg_init_scratch)
        instead of allocating one; no recording horizon.  pe_split: None for
        the library's choice, True / False to force the fused kernel's
        PE-face split on (where the PE sizes allow it) or off.  one_launch:
        one fused launch over every degree range (ADG_OPT_ONE_LAUNCH)."""
        if not isinstance(workloads, (list, tuple)):
            workloads = [workloads]
        self.workloads = list(workloads)
        self.probs = [to_problem(w) for w in self.workloads]
        self.offsets, self.lds, self.total = adg.adg_state_layout(self.probs)
        self.opt = adg.adg_options()
        self.opt.kernel = adg.KERNEL[kernel]
        self.opt.ckpt_every = ckpt_every
        if lane_elems == "auto":
            # elements per lane and (unless given) steps per launch, tuned together
            from . import autotune
            fused = kernel in ("fused", "auto")
            lane_elems, k, split = autotune.tune(self.workloads) if fused else (0, 0, None)
            fused_steps = fused_steps or k
            if pe_split is None:
                pe_split = split
        self.opt.lane_elems = int(lane_elems)
        self.opt.fused_steps = int(fused_steps)
        if pe_split is not None:
            self.opt.flags = adg.ADG_OPT_PE_SPLIT_ON if pe_split else adg.ADG_OPT_PE_SPLIT_OFF
        if one_launch:
            self.opt.flags |= adg.ADG_OPT_ONE_LAUNCH
        self.ws_bytes = adg.adg_workspace_size(self.probs, self.opt, n_steps_record)
        self.stream = stream
        if scratch:
            if n_steps_record:
                raise ValueError("the static scratch workspace has no recording horizon")
            dev = torch.device(device)
            if dev.index is None:
                dev = torch.device(dev.type, torch.cuda.current_device())
            self.device = dev
            self.workspace = None
            with torch.cuda.device(dev):
                self.ctx = adg.adg_init_scratch(self.probs, self.opt, _stream_handle(stream))
        else:
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=torch.device(device))
            self.device = self.workspace.device  # with its index
            self.ctx = adg.adg_init(self.probs, self.opt, n_steps_record, self.workspace.data_ptr(),
                                    self.ws_bytes, _stream_handle(stream))

    def close(self):
        if getattr(self, "ctx", None) is not None:
            adg.adg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state_ptr(self, t: torch.Tensor, name: str = "u") -> int:
        """Device address of a state vector, after checking that it has this
        context's layout: float64, contiguous, on this context's device,
        exactly adg_state_layout's total length and 16-byte aligned.  The
        kernels index every node plane up to its padded leading dimension, so
        anything else would be read or written out of bounds (ValueError)."""
        if not torch.is_tensor(t):
            raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
        if t.dtype != torch.float64:
            raise ValueError(f"{name}: dtype must be torch.float64, got {t.dtype}")
        if t.device != self.device:
            raise ValueError(f"{name}: must be on {self.device}, got {t.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: must be contiguous")
        if t.numel() != self.total:
            raise ValueError(f"{name}: must hold {self.total} doubles (adg_state_layout), got {t.numel()}")
        ptr = t.data_ptr()
        if ptr % 16:
            raise ValueError(f"{name}: data must be 16-byte aligned")
        return ptr

    # ---- state packing ---------------------------------------------------
    def empty_state(self) -> torch.Tensor:
        return torch.zeros(self.total, dtype=torch.float64, device=self.device)

    def pack(self, arrays) -> torch.Tensor:
        """Per-problem (n_elem, degree+1) arrays -> device state vector."""
        if not isinstance(arrays, (list, tuple)):
            arrays = [arrays]
        host = np.zeros(self.total, dtype=np.float64)
        for w, off, ld, a in zip(self.workloads, self.offsets, self.lds, arrays):
            a = np.asarray(a, dtype=np.float64)
            view = host[off:off + ld * (w.degree + 1)].reshape(w.degree + 1, ld)
            view[:, :w.n_elem] = a.T
        return torch.from_numpy(host).to(self.device)

    def view(self, u: torch.Tensor, i: int = 0) -> torch.Tensor:
        """(degree+1, n_elem) view of problem i inside the state vector."""
        w = self.workloads[i]
        off, ld = self.offsets[i], self.lds[i]
        return u[off:off + ld * (w.degree + 1)].view(w.degree + 1, ld)[:, :w.n_elem]

    def unpack(self, u: torch.Tensor):
        host = u.detach().cpu().numpy()
        out = []
        for w, off, ld in zip(self.workloads, self.offsets, self.lds):
            out.append(host[off:off + ld * (w.degree + 1)].reshape(w.degree + 1, ld)[:, :w.n_elem].T.copy())
        return out

    def nodes(self, i: int = 0) -> torch.Tensor:
        """Physical node coordinates of problem i, (degree+1, n_elem), on the device."""
        w = self.workloads[i]
        xi = torch.tensor(adg.adg_nodes(w.degree), dtype=torch.float64, device=self.device)
        dx = w.length / w.n_elem
        e = torch.arange(w.n_elem, dtype=torch.float64, device=self.device)
        return w.x_left + e[None, :] * dx + (xi[:, None] + 1.0) * (dx / 2.0)

    def initial_state(self) -> torch.Tensor:
        """Nodal interpolation of each workload's multi-sine initial data."""
        u = self.empty_state()
        for i, w in enumerate(self.workloads):
            x = self.nodes(i)
            v = torch.full_like(x, w.ic.offset)
            for k, a, ph in zip(w.ic.kappa, w.ic.amp, w.ic.phase):
                v = v + a * torch.sin(k * x + ph)
            self.view(u, i).copy_(v)
        return u

    # ---- stepping ----------------------------------------------------------
    def reset(self):
        adg.adg_reset(self.ctx)

    def step(self, u: torch.Tensor):
        adg.adg_step(self.ctx, self.state_ptr(u))

    def run(self, u: torch.Tensor, n_steps: int, graph: bool = True, record: bool = False,
            check_finite: bool = False):
        flags = (adg.ADG_RUN_GRAPH if graph else 0) | (adg.ADG_RUN_RECORD if record else 0) | \
                (adg.ADG_RUN_CHECK_FINITE if check_finite else 0)
        adg.adg_run(self.ctx, self.state_ptr(u), n_steps, flags)

    def capture_graph(self, u: torch.Tensor):
        """Capture the step graph for buffer u without stepping (adg_run with
        zero steps and ADG_RUN_GRAPH), so that a later graph run replays it
        without the capture and instantiation cost."""
        adg.adg_run(self.ctx, self.state_ptr(u), 0, adg.ADG_RUN_GRAPH)

    def adjoint(self, cot: torch.Tensor, want_speed: bool = True):
        """dJ/du0 (device, state layout) and dJ/da per problem (host list, or
        None if want_speed is False) for the last recorded run, given
        cot = dJ/du(T)."""
        cot_ptr = self.state_ptr(cot, "cot")
        grad = torch.empty_like(cot)
        gs = adg.adg_adjoint(self.ctx, cot_ptr, self.state_ptr(grad, "grad"), len(self.probs), want_speed)
        return grad, gs

    def steps_taken(self) -> int:
        return adg.adg_step_count(self.ctx)

    def error_stats(self, u: torch.Tensor, ref: torch.Tensor):
        return adg.adg_error_stats(self.ctx, self.state_ptr(u), self.state_ptr(ref, "ref"), len(self.probs))

    def ensemble_stats(self, u: torch.Tensor, ref: torch.Tensor, group_of, n_groups: int):
        """Per group: (mean <E>, var <E>, mean max-err, var max-err)."""
        return adg.adg_ensemble_stats(self.ctx, self.state_ptr(u), self.state_ptr(ref, "ref"), list(group_of),
                                      n_groups)

    def exact_advection_state(self, t: float) -> torch.Tensor:
        """Nodal values of the exact linear-advection solution u0(x - a t)."""
        u = self.empty_state()
        for i, w in enumerate(self.workloads):
            x = self.nodes(i) - w.speed * t
            v = torch.full_like(x, w.ic.offset)
            for k, a, ph in zip(w.ic.kappa, w.ic.amp, w.ic.phase):
                v = v + a * torch.sin(k * x + ph)
            self.view(u, i).copy_(v)
        return u

    def exact_burgers_state(self, t: float, iters: int = 60) -> torch.Tensor:
        """Nodal values of the inviscid Burgers solution before the first
        shock, u(x, t) = u0(xi) with x = xi + u0(xi) t, by Newton's method on
        the characteristic foot xi (raises once characteristics cross)."""
        u = self.empty_state()
        for i, w in enumerate(self.workloads):
            x = self.nodes(i)

            def u0(z):
                v = torch.full_like(z, w.ic.offset)
                for k, a, ph in zip(w.ic.kappa, w.ic.amp, w.ic.phase):
                    v = v + a * torch.sin(k * z + ph)
                return v

            def du0(z):
                v = torch.zeros_like(z)
                for k, a, ph in zip(w.ic.kappa, w.ic.amp, w.ic.phase):
                    v = v + a * k * torch.cos(k * z + ph)
                return v

            xi = x - u0(x) * t
            for _ in range(iters):
                dg = 1.0 + du0(xi) * t
                if bool((dg <= 0).any()):
                    raise ValueError("characteristics crossed: a shock has formed")
                step = (xi + u0(xi) * t - x) / dg
                xi = xi - step
                if float(step.abs().max()) < 1e-15 * (1.0 + float(x.abs().max())):
                    break
            self.view(u, i).copy_(u0(xi))
        return u

    def delay_schedule(self, i: int, step0: int, n_steps: int):
        w = self.workloads[i]
        return adg.adg_delay_schedule(self.probs[i], step0, n_steps, adg.RK_STAGES[w.rk], w.n_pe)
