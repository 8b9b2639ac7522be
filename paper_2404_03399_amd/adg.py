"""ctypes binding of libadg.so: the C ABI of include/adg.h, same names.

Argument marshalling only.  Every step of the method runs in the HIP
kernels; if the library is missing this module raises on import of the
library (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

from . import build as _build

ADG_ABI_VERSION = 2

ADG_OK = 0
ADG_E_INVALID = -1
ADG_E_ABI = -2
ADG_E_WORKSPACE = -3
ADG_E_HIP = -4
ADG_E_STATE = -5
ADG_E_NONFINITE = -6
ADG_E_UNSUPPORTED = -7

EQUATION = {"advection": 0, "burgers": 1, "viscous_burgers": 2}
SCHEME = {"dg": 0, "adg": 1, "adg_at": 2}
FLUX = {"upwind": 0, "central": 1, "llf": 2}
RK = {"heun": 0, "ssprk3": 1, "rk4": 2, "lsrk3": 3, "lsrk4": 4}
RK_STAGES = {"heun": 2, "ssprk3": 3, "rk4": 4, "lsrk3": 3, "lsrk4": 5}
KERNEL = {"auto": 0, "stage": 1, "fused": 2}

ADG_SCRATCH_BYTES = 64 << 20

ADG_OPT_PE_SPLIT_OFF = 1
ADG_OPT_PE_SPLIT_ON = 2
ADG_OPT_ONE_LAUNCH = 4

ADG_RUN_GRAPH = 1
ADG_RUN_RECORD = 2
ADG_RUN_CHECK_FINITE = 4

SYMBOLS = [
    "adg_abi_version", "adg_last_error", "adg_build_id", "adg_nodes", "adg_state_layout", "adg_workspace_size",
    "adg_init", "adg_init_scratch", "adg_reset", "adg_step_count", "adg_step", "adg_run", "adg_adjoint",
    "adg_error_stats", "adg_ensemble_stats", "adg_delay_schedule", "adg_destroy",
]


class adg_problem(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("equation", C.c_uint32), ("scheme", C.c_uint32),
        ("flux", C.c_uint32), ("rk", C.c_uint32), ("degree", C.c_uint32),
        ("at_levels", C.c_uint32), ("n_delays", C.c_uint32), ("delay_granularity", C.c_uint32),
        ("reserved", C.c_uint32), ("n_elem", C.c_int64), ("pe_size", C.c_int64),
        ("seed", C.c_uint64), ("delay_threshold", C.c_uint64 * 7), ("x_left", C.c_double),
        ("length", C.c_double), ("speed", C.c_double), ("dt", C.c_double), ("viscosity", C.c_double),
    ]


class adg_options(C.Structure):
    _fields_ = [("ckpt_every", C.c_int64), ("kernel", C.c_int32), ("lane_elems", C.c_int32),
                ("flags", C.c_uint32), ("fused_steps", C.c_uint32)]


class AdgError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


_LIB = None


def library_path() -> str:
    """The in-tree libadg.so, or the build named by ADG_LIBRARY (e.g. the
    host-AddressSanitizer build)."""
    return os.environ.get("ADG_LIBRARY") or _build.LIB


def lib() -> C.CDLL:
    """Load libadg.so (built in-tree by paper_2404_03399_amd.build).  Raises
    ImportError if it is missing, or if it was built from sources other than
    the ones in this tree (its adg_build_id() differs from the hash of
    csrc/ and include/): a stale binary is never tested or timed."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"HIP library not built: {path} (run python -m paper_2404_03399_amd.build)")
        L = C.CDLL(path)
        P, I32, I64, U32, D = C.POINTER, C.c_int32, C.c_int64, C.c_uint32, C.c_double
        vp = C.c_void_p
        sig = {
            "adg_abi_version": ([], C.c_int),
            "adg_last_error": ([], C.c_char_p),
            "adg_build_id": ([], C.c_char_p),
            "adg_nodes": ([I32, P(D)], C.c_int),
            "adg_state_layout": ([P(adg_problem), I32, P(I64), P(I64), P(I64)], C.c_int),
            "adg_workspace_size": ([P(adg_problem), I32, P(adg_options), I64, P(I64)], C.c_int),
            "adg_init": ([P(vp), P(adg_problem), I32, P(adg_options), I64, vp, I64, vp], C.c_int),
            "adg_init_scratch": ([P(vp), P(adg_problem), I32, P(adg_options), vp], C.c_int),
            "adg_reset": ([vp], C.c_int),
            "adg_step_count": ([vp, P(I64)], C.c_int),
            "adg_step": ([vp, vp], C.c_int),
            "adg_run": ([vp, vp, I64, U32], C.c_int),
            "adg_adjoint": ([vp, vp, vp, P(D)], C.c_int),
            "adg_error_stats": ([vp, vp, vp, P(D)], C.c_int),
            "adg_ensemble_stats": ([vp, vp, vp, P(I32), I32, P(D)], C.c_int),
            "adg_delay_schedule": ([P(adg_problem), I64, I64, P(I32)], C.c_int),
            "adg_destroy": ([vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        if L.adg_abi_version() != ADG_ABI_VERSION:
            raise ImportError("libadg ABI version mismatch")
        built, here = L.adg_build_id().decode(), _build.source_hash()
        if built != here:
            raise ImportError(f"{path} was built from other sources (build id {built}, sources {here}): "
                              f"rebuild with python -m paper_2404_03399_amd.build")
        _LIB = L
    return _LIB


def check(code: int, where: str) -> None:
    if code != ADG_OK:
        raise AdgError(code, where, lib().adg_last_error().decode())


# ---- thin wrappers with the C names ------------------------------------------
def adg_abi_version() -> int:
    return lib().adg_abi_version()


def adg_nodes(degree: int):
    out = (C.c_double * (degree + 1))()
    check(lib().adg_nodes(degree, out), "adg_nodes")
    return list(out)


def adg_state_layout(probs):
    n = len(probs)
    arr = (adg_problem * n)(*probs)
    offs = (C.c_int64 * n)()
    lds = (C.c_int64 * n)()
    tot = C.c_int64()
    check(lib().adg_state_layout(arr, n, offs, lds, C.byref(tot)), "adg_state_layout")
    return list(offs), list(lds), tot.value


def adg_workspace_size(probs, opt: adg_options, n_steps_record: int = 0) -> int:
    n = len(probs)
    arr = (adg_problem * n)(*probs)
    out = C.c_int64()
    check(lib().adg_workspace_size(arr, n, C.byref(opt), n_steps_record, C.byref(out)), "adg_workspace_size")
    return out.value


def adg_init(probs, opt: adg_options, n_steps_record: int, d_workspace: int, workspace_bytes: int, stream: int):
    n = len(probs)
    arr = (adg_problem * n)(*probs)
    ctx = C.c_void_p()
    check(lib().adg_init(C.byref(ctx), arr, n, C.byref(opt), n_steps_record, C.c_void_p(d_workspace),
                         workspace_bytes, C.c_void_p(stream)), "adg_init")
    return ctx


def adg_init_scratch(probs, opt: adg_options, stream: int):
    n = len(probs)
    arr = (adg_problem * n)(*probs)
    ctx = C.c_void_p()
    check(lib().adg_init_scratch(C.byref(ctx), arr, n, C.byref(opt), C.c_void_p(stream)), "adg_init_scratch")
    return ctx


def adg_reset(ctx) -> None:
    check(lib().adg_reset(ctx), "adg_reset")


def adg_step_count(ctx) -> int:
    out = C.c_int64()
    check(lib().adg_step_count(ctx, C.byref(out)), "adg_step_count")
    return out.value


def adg_step(ctx, d_u: int) -> None:
    check(lib().adg_step(ctx, C.c_void_p(d_u)), "adg_step")


def adg_run(ctx, d_u: int, n_steps: int, flags: int = 0) -> None:
    check(lib().adg_run(ctx, C.c_void_p(d_u), n_steps, flags), "adg_run")


def adg_adjoint(ctx, d_cot: int, d_grad_u0: int, n_probs: int, want_speed: bool = True):
    """dJ/du0 into d_grad_u0; returns dJ/da per problem, or None when not
    requested (h_grad_speed = NULL)."""
    out = (C.c_double * n_probs)() if want_speed else None
    check(lib().adg_adjoint(ctx, C.c_void_p(d_cot), C.c_void_p(d_grad_u0), out), "adg_adjoint")
    return list(out) if want_speed else None


def adg_error_stats(ctx, d_u: int, d_ref: int, n_probs: int):
    out = (C.c_double * (3 * n_probs))()
    check(lib().adg_error_stats(ctx, C.c_void_p(d_u), C.c_void_p(d_ref), out), "adg_error_stats")
    return [tuple(out[3 * i:3 * i + 3]) for i in range(n_probs)]


def adg_ensemble_stats(ctx, d_u: int, d_ref: int, group_of, n_groups: int):
    n = len(group_of)
    g = (C.c_int32 * n)(*group_of)
    out = (C.c_double * (4 * n_groups))()
    check(lib().adg_ensemble_stats(ctx, C.c_void_p(d_u), C.c_void_p(d_ref), g, n_groups, out), "adg_ensemble_stats")
    return [tuple(out[4 * i:4 * i + 4]) for i in range(n_groups)]


def adg_delay_schedule(prob: adg_problem, step0: int, n_steps: int, n_stages: int, n_pe: int):
    import numpy as np
    out = np.zeros((n_steps, n_stages, max(n_pe, 1)), dtype=np.int32)
    check(lib().adg_delay_schedule(C.byref(prob), step0, n_steps,
                                   out.ctypes.data_as(C.POINTER(C.c_int32))), "adg_delay_schedule")
    return out


def adg_destroy(ctx) -> None:
    check(lib().adg_destroy(ctx), "adg_destroy")
