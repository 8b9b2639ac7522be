"""Autotuner for the fused step kernel's elements per lane (1, 2 or 4).

The best value depends on the problem set: register pressure grows with the
elements per lane (fewer resident waves), while larger tiles cut the halo
recompute and the number of waves.  The tuner times each admissible
candidate on the caller's own problems (same kernels, a few graph-replayed
steps on a scratch copy of the initial state) and caches the winner in a
JSON file keyed by device, integrator, equation/flux, degrees and size.

    R = autotune.lane_elems(workloads)            # tuned (or cached) value
    Solver(workloads, lane_elems="auto")           # same, through the solver
"""
from __future__ import annotations

import json
import math
import os
from typing import Iterable, List

CANDIDATES = (1, 2, 4)


def cache_path() -> str:
    return os.environ.get("ADG_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "adg_tune.json"))


def _key(workloads, device_name: str) -> str:
    degrees = sorted({w.degree for w in workloads})
    total = sum(w.n_elem for w in workloads)
    bucket = int(round(math.log2(max(total, 1))))
    pes = min((w.pe_size for w in workloads if w.scheme != "dg" and w.n_elem // w.pe_size > 1), default=0)
    w0 = workloads[0]
    return "|".join(str(x) for x in (device_name, w0.rk, w0.equation, w0.flux, w0.scheme, degrees, bucket,
                                     len(workloads) > 1, min(pes, 4)))


def admissible(workloads) -> List[int]:
    pes = min((w.pe_size for w in workloads if w.scheme != "dg" and w.n_elem // w.pe_size > 1), default=1 << 30)
    return [r for r in CANDIDATES if r <= pes]


def lane_elems(workloads, steps: int = 24, use_cache: bool = True, verbose: bool = False) -> int:
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
        if key in cache:
            return int(cache[key]["lane_elems"])
    timings = {}
    for r in admissible(workloads):
        s = Solver(workloads, lane_elems=r)
        u = s.initial_state()
        s.run(u, 4, graph=False)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        s.run(u, steps, graph=True)
        ev1.record()
        torch.cuda.synchronize()
        timings[r] = ev0.elapsed_time(ev1) / steps
        s.close()
    best = min(timings, key=timings.get)
    if verbose:
        print(f"autotune {key}: " + ", ".join(f"R={r}: {t * 1e3:.2f} us" for r, t in timings.items()), flush=True)
    if use_cache:
        cache[key] = {"lane_elems": best, "ms_per_step": timings}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, default=str)
        os.replace(tmp, path)
    return best
