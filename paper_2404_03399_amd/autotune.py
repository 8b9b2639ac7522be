"""Autotuner for the fused step kernel's launch shape: elements per lane
(1, 2 or 4), time steps per launch (1 or 2) and, where the PE sizes allow
it, the PE-face split on or off.

The best pair depends on the problem set: register pressure grows with the
elements per lane (fewer resident waves), larger tiles cut the halo
recompute and the number of waves, and two steps per launch halve the state
traffic per step at the price of a wider halo.  The tuner times each
admissible pair on the caller's own problems (same kernels, a few
graph-replayed steps on a scratch copy of the initial state) and caches the
winner in a JSON file keyed by device, integrator, equation/flux, degrees
and size.  Every pair gives bitwise the same states (the kernels use
explicit FMAs with contraction off), so tuning never changes results.

    R, K, split = autotune.tune(workloads)        # tuned (or cached) shape
    R = autotune.lane_elems(workloads)            # its elements per lane
    Solver(workloads, lane_elems="auto")           # same, through the solver
"""
from __future__ import annotations

import json
import math
import os
import statistics
from typing import List, Optional, Tuple

CANDIDATES = (1, 2, 4)
STEPS_PER_LAUNCH = (1, 2)


def cache_path() -> str:
    return os.environ.get("ADG_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "adg_tune.json"))


def kernel_source_hash() -> str:
    """Hash of the kernel and library sources: a cached choice made on other
    kernels is not reused."""
    import hashlib
    from . import build
    h = hashlib.sha256()
    for name in sorted(os.listdir(build.CSRC)):
        h.update(name.encode())
        with open(os.path.join(build.CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _key(workloads, device_name: str) -> str:
    degrees = sorted({w.degree for w in workloads})
    total = sum(w.n_elem for w in workloads)
    bucket = int(round(math.log2(max(total, 1))))
    pes = min((w.pe_size for w in workloads if w.scheme != "dg" and w.n_elem // w.pe_size > 1), default=0)
    w0 = workloads[0]
    return "|".join(str(x) for x in (device_name, kernel_source_hash(), w0.rk, w0.equation, w0.flux, w0.scheme,
                                     degrees, bucket, len(workloads) > 1, min(pes, 4)))


def admissible(workloads) -> List[int]:
    """Elements per lane the library accepts for these problems (<= every
    asynchronous problem's PE size)."""
    pes = min((w.pe_size for w in workloads if w.scheme != "dg" and w.n_elem // w.pe_size > 1), default=1 << 30)
    return [r for r in CANDIDATES if r <= pes]


def split_possible(workloads, k: int) -> bool:
    """The PE-face split needs an asynchronous problem and, for every one, a
    PE size holding a window of 4 k S elements (k steps per launch, S
    stages)."""
    from .adg import RK_STAGES
    asyn = [w for w in workloads if w.scheme != "dg" and w.n_elem // w.pe_size > 1]
    if not asyn or workloads[0].equation == "viscous_burgers":
        return False
    return min(w.pe_size for w in asyn) >= 4 * k * RK_STAGES[workloads[0].rk]


def configs(workloads) -> List[Tuple[int, int, Optional[bool]]]:
    """Candidate (R, K, split): split None where the PE-face split does not
    apply (the library then has nothing to choose)."""
    out = []
    for r in admissible(workloads):
        for k in STEPS_PER_LAUNCH:
            if split_possible(workloads, k):
                out += [(r, k, False), (r, k, True)]
            else:
                out.append((r, k, None))
    return out


def tune(workloads, steps: int = 32, use_cache: bool = True, verbose: bool = False,
         reps: int = 3) -> Tuple[int, int, Optional[bool]]:
    """(elements per lane, steps per launch, PE-face split) with the shortest
    time per step: for each candidate the step graph is captured first
    (outside the timing), then `reps` runs of `steps` graph-replayed steps are
    timed with HIP events and the median is kept."""
    import torch
    from .solver import Solver

    if not isinstance(workloads, (list, tuple)):
        workloads = [workloads]
    workloads = list(workloads)
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    key = _key(workloads, dev)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache and "pe_split" in cache[key]:
            c = cache[key]
            return int(c["lane_elems"]), int(c["fused_steps"]), c["pe_split"]
    steps = max(16, steps - steps % 16)  # whole graph replays only
    timings = {}
    u_init = None  # the state layout does not depend on the launch shape
    for r, k, split in configs(workloads):
        s = Solver(workloads, lane_elems=r, fused_steps=k, pe_split=split)
        if u_init is None:
            u_init = s.initial_state()
        u = u_init.clone()
        s.capture_graph(u)
        s.run(u, 16, graph=True)  # warm-up replay
        stream = s.stream if s.stream is not None else torch.cuda.current_stream()
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            s.run(u, steps, graph=True)
            ev1.record(stream)
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1) / steps)
        timings[(r, k, split)] = statistics.median(times)
        s.close()
        del u
    best = min(timings, key=timings.get)
    if verbose:
        print(f"autotune {key}: " + ", ".join(f"R={r} K={k} split={sp}: {t * 1e3:.2f} us"
                                              for (r, k, sp), t in timings.items()), flush=True)
    if use_cache:
        cache[key] = {"lane_elems": best[0], "fused_steps": best[1], "pe_split": best[2],
                      "ms_per_step": {f"R={r},K={k},split={sp}": t for (r, k, sp), t in timings.items()}}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    return best


def lane_elems(workloads, steps: int = 24, use_cache: bool = True, verbose: bool = False) -> int:
    return tune(workloads, steps, use_cache, verbose)[0]
