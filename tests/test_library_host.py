"""CPU tests of the C-ABI library: it loads, exports every symbol declared in
include/adg.h, and its host-side logic (validation, layout, nodes, delay
schedule) agrees with the oracle.  No kernel is launched here."""
import ctypes
import os
import re
from dataclasses import replace

import numpy as np
import pytest

from paper_2404_03399_amd import adg, solver, workloads as W
from oracle import basis, delays

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "adg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(adg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(adg.library_path()):
        from paper_2404_03399_amd import build
        build.build()
    return adg.lib()


def test_exports_every_declared_symbol(L):
    names = _declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(adg.SYMBOLS)


def test_abi_version(L):
    assert adg.adg_abi_version() == 2


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_nodes_match_oracle(L, p):
    np.testing.assert_allclose(adg.adg_nodes(p), basis.gll_nodes(p), atol=2e-16)


def test_struct_sizes(L):
    assert ctypes.sizeof(adg.adg_problem) == 40 + 16 + 8 + 56 + 40
    assert ctypes.sizeof(adg.adg_options) == 24


def test_thresholds_match_oracle():
    for probs in (["0.3", "0.4", "0.3"], ["0.5", "0.25", "0.15", "0.1"], ["1/3", "1/3", "1/3"], ["1"]):
        assert solver.delay_thresholds(probs) == delays.thresholds(probs)


def test_layout(L):
    ws = [W.c1_advection_small(), replace(W.c1_advection_small(), n_elem=100, pe_size=25, degree=3)]
    offs, lds, tot = adg.adg_state_layout([solver.to_problem(w) for w in ws])
    assert offs == [0, 64 * 3] and lds == [64, 128] and tot == 64 * 3 + 128 * 4


@pytest.mark.parametrize("rk,per_stage,scheme", [("rk4", True, "adg_at"), ("ssprk3", False, "adg_at"),
                                                  ("heun", True, "adg"), ("rk4", True, "dg"),
                                                  ("lsrk4", True, "adg_at")])
def test_delay_schedule_bit_exact_vs_oracle(L, rk, per_stage, scheme):
    w = replace(W.c2_advection_large(scheme, n_elem=4096), rk=rk, per_stage=per_stage, seed=12345)
    p = solver.to_problem(w)
    S = adg.RK_STAGES[rk]
    got = adg.adg_delay_schedule(p, 0, 20, S, w.n_pe)
    q = (w.degree + 1) if scheme == "adg_at" else 1
    ref = delays.schedule(w.seed, w.probs, 20, S, w.n_pe, per_stage, q)
    if scheme == "dg":
        ref[:] = 0
    assert np.array_equal(got, ref)
    # later window, large seed (batched realizations use seed = mesh << 32 | r)
    w2 = replace(w, seed=(11 << 32) | 255)
    got = adg.adg_delay_schedule(solver.to_problem(w2), 1000, 3, S, w.n_pe)
    ref = delays.schedule(w2.seed, w.probs, 3, S, w.n_pe, per_stage, q, step0=1000)
    if scheme == "dg":
        ref[:] = 0
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("rk,q", [("heun", 2), ("rk4", 4)])
def test_caa_schedule_bit_exact_vs_oracle(L, rk, q):
    w = replace(W.c2_advection_large("adg_at", n_elem=1024), rk=rk, caa=True, probs=W.DELAYS_UNIFORM3,
                degree=q - 1)
    S = adg.RK_STAGES[rk]
    got = adg.adg_delay_schedule(solver.to_problem(w), 0, 23, S, w.n_pe)
    ref = delays.schedule(w.seed, w.probs, 23, S, w.n_pe, w.per_stage, q, caa=True)
    assert np.array_equal(got, ref)
    # every face and stage of a step shares the cycle's delay
    assert all(len(np.unique(got[i])) == 1 for i in range(23))
    # communication-avoiding with L = 3 needs exactly three delay levels
    p = solver.to_problem(replace(w, probs=W.DELAYS_C2))
    with pytest.raises(adg.AdgError):
        adg.adg_workspace_size([p], adg.adg_options())


def test_viscous_burgers_options(L):
    w = W.Workload(name="ldg", equation="viscous_burgers", flux="llf", rk="heun", degree=2, n_elem=64,
                   pe_size=16, probs=("0.3", "0.4", "0.3"), viscosity=0.1, dt=1e-4)
    p = solver.to_problem(w)
    fused = adg.adg_workspace_size([p], adg.adg_options())              # AUTO -> fused, q kept on chip
    opt = adg.adg_options()
    opt.kernel = adg.KERNEL["stage"]
    assert adg.adg_workspace_size([p], opt) > fused                     # the q pass needs a buffer
    opt = adg.adg_options()
    opt.kernel = adg.KERNEL["fused"]
    opt.fused_steps = 1
    assert adg.adg_workspace_size([p], opt) > 0                         # one or two steps per launch
    for r in (2, 4):                                                    # several elements per lane
        opt.lane_elems = r
        assert adg.adg_workspace_size([p], opt) > 0
    opt.lane_elems = 32                                                 # more than the PE size
    with pytest.raises(adg.AdgError) as ei:
        adg.adg_workspace_size([p], opt)
    assert ei.value.code == adg.ADG_E_INVALID
    with pytest.raises(adg.AdgError) as ei:
        adg.adg_workspace_size([p], adg.adg_options(), 10)             # no adjoint for local DG
    assert ei.value.code == adg.ADG_E_UNSUPPORTED
    for bad in (dict(flux="central"), dict(viscosity=-1.0), dict(viscosity=float("nan"))):
        with pytest.raises(adg.AdgError):
            adg.adg_workspace_size([solver.to_problem(replace(w, **bad))], adg.adg_options())
    with pytest.raises(adg.AdgError):   # viscosity only for viscous Burgers
        adg.adg_workspace_size([solver.to_problem(replace(W.c1_advection_small(), viscosity=0.1))],
                               adg.adg_options())


def _bad(**kw):
    return solver.to_problem(replace(W.c1_advection_small(), **kw))


@pytest.mark.parametrize("mut", [
    dict(degree=5), dict(degree=0), dict(pe_size=7), dict(dt=-1.0), dict(flux="llf"),
    dict(equation="burgers"), dict(scheme="adg"), dict(length=0.0), dict(degree=4, scheme="adg_at", at_levels=6),
])
def test_validation_rejects(L, mut):
    p = _bad(**mut)
    if mut.get("scheme") == "adg":
        p.at_levels = 2          # AT levels set for a non-AT scheme
    if mut.get("at_levels") == 6:
        p.at_levels = 6
    with pytest.raises(adg.AdgError) as ei:
        adg.adg_workspace_size([p], adg.adg_options())
    assert ei.value.code == adg.ADG_E_INVALID


def test_validation_abi_and_thresholds(L):
    p = solver.to_problem(W.c1_advection_small())
    p.abi_version = 99
    with pytest.raises(adg.AdgError) as ei:
        adg.adg_workspace_size([p], adg.adg_options())
    assert ei.value.code == adg.ADG_E_ABI
    p = solver.to_problem(W.c1_advection_small())
    p.delay_threshold[0], p.delay_threshold[1] = 10, 5
    with pytest.raises(adg.AdgError):
        adg.adg_workspace_size([p], adg.adg_options())
    a = solver.to_problem(W.c1_advection_small())
    b = solver.to_problem(replace(W.c1_advection_small(), rk="heun"))
    with pytest.raises(adg.AdgError):
        adg.adg_workspace_size([a, b], adg.adg_options())


def test_workspace_size_grows_with_problems(L):
    one = adg.adg_workspace_size([solver.to_problem(W.c1_advection_small())], adg.adg_options())
    two = adg.adg_workspace_size([solver.to_problem(W.c1_advection_small())] * 2, adg.adg_options())
    assert two > one > 0


def test_autotune_admissible_candidates():
    from paper_2404_03399_amd import autotune
    w = W.c1_advection_small()
    assert autotune.admissible([w]) == [1, 2, 4]
    assert autotune.admissible([replace(w, pe_size=2, n_elem=64)]) == [1, 2]
    assert autotune.admissible([replace(w, scheme="dg", pe_size=1)]) == [1, 2, 4]


def _documented_valid(p, opt, n_rec) -> bool:
    """The constraints include/adg.h states for one problem and the options."""
    import math
    eq, sch, fl = p.equation, p.scheme, p.flux
    L_, q = p.n_delays, p.at_levels
    ok = (p.abi_version == adg.ADG_ABI_VERSION and eq in (0, 1, 2) and sch in (0, 1, 2) and p.rk in (0, 1, 2, 3, 4)
          and 1 <= p.degree <= 4 and 1 <= L_ <= 8 and p.delay_granularity in (0, 1, 2) and p.reserved == 0
          and p.n_elem >= 2 and p.pe_size >= 1 and p.n_elem % p.pe_size == 0
          and math.isfinite(p.length) and p.length > 0 and math.isfinite(p.dt) and p.dt > 0
          and math.isfinite(p.x_left))
    if not ok:
        return False
    if fl in (0, 1) and eq != 0:
        return False
    if fl == 2 and eq == 0:
        return False
    if fl not in (0, 1, 2):
        return False
    if eq == 0 and not (math.isfinite(p.speed) and p.speed != 0):
        return False
    if eq == 2 and not (math.isfinite(p.viscosity) and p.viscosity >= 0):
        return False
    if eq != 2 and p.viscosity != 0:
        return False
    if not (q == 0 or (1 <= q <= 5 and sch == 2)):
        return False
    if p.delay_granularity == 2 and L_ != 3:  # the communication-avoiding cycle
        return False
    thr = [p.delay_threshold[i] for i in range(L_ - 1)]
    if any(t > (1 << 53) for t in thr) or any(b < a for a, b in zip(thr, thr[1:])):
        return False
    if opt.ckpt_every < 0 or opt.kernel not in (0, 1, 2) or opt.flags != 0 or opt.fused_steps not in (0, 1, 2):
        return False
    if opt.lane_elems not in (0, 1, 2, 4):
        return False
    async_ = sch != 0 and p.n_elem // p.pe_size > 1
    if async_ and opt.lane_elems > p.pe_size:
        return False
    return 0 <= n_rec <= (1 << 28)


def test_random_descriptors_are_validated(L):
    """Random mutations of valid descriptors and options: adg_state_layout
    and adg_workspace_size return a documented status and never crash, a
    valid draw is accepted, and nothing outside the documented constraints
    is accepted."""
    import ctypes as C
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_gpu_random_configs import draw
    rng = np.random.default_rng(2024)
    ints = [0, 1, 2, 3, 4, 5, 7, 8, 9, 64, -1, 2 ** 31 - 1, 2 ** 32 - 1]
    dbls = [0.0, -0.0, 1.0, -1.0, 1e-300, 1e300, float("nan"), float("inf"), -float("inf")]
    fields_i = ["abi_version", "equation", "scheme", "flux", "rk", "degree", "at_levels", "n_delays",
                "delay_granularity", "reserved", "n_elem", "pe_size"]
    fields_d = ["x_left", "length", "speed", "dt", "viscosity"]
    codes = {0, adg.ADG_E_INVALID, adg.ADG_E_ABI, adg.ADG_E_UNSUPPORTED}
    accepted_invalid = []
    for it in range(3000):
        w, *_ = draw(int(rng.integers(400)))
        p = solver.to_problem(w)
        opt = adg.adg_options()
        opt.kernel = int(rng.choice([0, 1, 2]))
        opt.lane_elems = int(rng.choice([0, 1, 2, 4]))
        if w.scheme != "dg" and w.n_elem // w.pe_size > 1:
            opt.lane_elems = min(opt.lane_elems, 1 if w.pe_size < 2 else (2 if w.pe_size < 4 else opt.lane_elems))
        opt.fused_steps = int(rng.choice([0, 1, 2]))
        n_rec = 0
        mutate = it % 4 != 0  # every fourth draw stays valid
        if mutate:
            for _ in range(int(rng.integers(1, 4))):
                r = rng.random()
                if r < 0.55:
                    setattr(p, str(rng.choice(fields_i)), int(rng.choice(ints)) % (1 << 32)
                            if rng.random() < 0.9 else int(rng.integers(0, 1 << 31)))
                elif r < 0.85:
                    setattr(p, str(rng.choice(fields_d)), float(rng.choice(dbls)))
                elif r < 0.92:
                    p.delay_threshold[int(rng.integers(7))] = int(rng.choice([0, 1 << 52, (1 << 53) + 1, (1 << 64) - 1]))
                else:
                    opt.lane_elems = int(rng.choice([-1, 3, 8]))
                    opt.flags = int(rng.choice([0, 1]))
                    opt.ckpt_every = int(rng.choice([-1, 0, 5]))
                    opt.fused_steps = int(rng.choice([0, 3, -1])) % (1 << 32)
        arr = (adg.adg_problem * 1)(p)
        offs, lds, tot, out = (C.c_int64 * 1)(), (C.c_int64 * 1)(), C.c_int64(), C.c_int64()
        rc1 = L.adg_state_layout(arr, 1, offs, lds, C.byref(tot))
        rc2 = L.adg_workspace_size(arr, 1, C.byref(opt), n_rec, C.byref(out))
        assert rc1 in codes and rc2 in codes, (it, rc1, rc2)
        valid = _documented_valid(p, opt, n_rec)
        if not mutate:
            assert valid and rc2 == 0, (it, rc2, adg.adg_last_error())
        if rc2 == 0 and not valid:
            accepted_invalid.append((it, {f: getattr(p, f) for f in fields_i + fields_d}))
        if rc2 == 0:
            assert rc1 == 0 and out.value > 0 and tot.value > 0
    assert not accepted_invalid, accepted_invalid[:5]


def test_state_tensor_validation_rejects_wrong_layouts():
    """Solver.state_ptr, which every stepping, adjoint and statistics call
    uses for its device pointers, refuses tensors the kernels would index out
    of bounds: wrong dtype, device, length, non-contiguous or misaligned.
    Driven here with CPU tensors through a stand-in for the context."""
    import torch
    from types import SimpleNamespace
    from paper_2404_03399_amd.solver import Solver
    fake = SimpleNamespace(device=torch.device("cpu"), total=128)
    ok = torch.zeros(128, dtype=torch.float64)
    assert Solver.state_ptr(fake, ok) == ok.data_ptr()
    bad = {
        "float32": torch.zeros(128, dtype=torch.float32),
        "short": torch.zeros(127, dtype=torch.float64),
        "long": torch.zeros(129, dtype=torch.float64),
        "natural layout": torch.zeros(40, 3, dtype=torch.float64),
        "strided": torch.zeros(256, dtype=torch.float64)[::2],
        "misaligned": torch.zeros(129, dtype=torch.float64)[1:],
    }
    for name, t in bad.items():
        with pytest.raises(ValueError):
            Solver.state_ptr(fake, t, name)
    with pytest.raises(ValueError):
        Solver.state_ptr(SimpleNamespace(device=torch.device("meta"), total=128), ok)
    with pytest.raises(TypeError):
        Solver.state_ptr(fake, np.zeros(128))


def test_library_build_id_matches_sources(L):
    """The loaded library was compiled from the sources in this tree."""
    from paper_2404_03399_amd import build
    assert L.adg_build_id().decode() == build.source_hash()


def test_stale_library_is_refused(monkeypatch):
    """A library whose build id differs from the hash of csrc/ and include/
    is refused on load (a stale binary is never tested or timed)."""
    from paper_2404_03399_amd import build
    monkeypatch.setattr(build, "source_hash", lambda: "not-these-sources")
    monkeypatch.setattr(adg, "_LIB", None)
    with pytest.raises(ImportError, match="other sources"):
        adg.lib()


def test_scratch_init_rejects_oversized_problems(L):
    """adg_init_scratch refuses, before any device call, problems whose
    workspace exceeds the static scratch array."""
    w = W.c2_advection_large("adg_at", n_elem=1 << 24)
    p = solver.to_problem(w)
    assert adg.adg_workspace_size([p], adg.adg_options()) > adg.ADG_SCRATCH_BYTES
    with pytest.raises(adg.AdgError) as ei:
        adg.adg_init_scratch([p], adg.adg_options(), 0)
    assert ei.value.code == adg.ADG_E_WORKSPACE
    assert "static scratch" in str(ei.value)


def test_option_flags_validated(L):
    """adg_options.flags: the two PE-face split bits are accepted alone and
    refused together; the one-launch bit needs the fused kernel, two elements
    per lane and no forced split, and is refused for the local DG kernel; any
    other bit is refused; the split adds the window work lists to the
    workspace."""
    p = solver.to_problem(W.c2_advection_large("adg_at", n_elem=1 << 16))
    base = adg.adg_workspace_size([p], adg.adg_options())
    for f in (adg.ADG_OPT_PE_SPLIT_OFF, adg.ADG_OPT_PE_SPLIT_ON):
        opt = adg.adg_options()
        opt.flags = f
        assert adg.adg_workspace_size([p], opt) > 0
    off = adg.adg_options()
    off.flags = adg.ADG_OPT_PE_SPLIT_OFF
    assert adg.adg_workspace_size([p], off) < base  # PE size 256 splits by default
    for f in (adg.ADG_OPT_PE_SPLIT_OFF | adg.ADG_OPT_PE_SPLIT_ON, 8, 1 << 31,
              adg.ADG_OPT_ONE_LAUNCH | adg.ADG_OPT_PE_SPLIT_ON):
        opt = adg.adg_options()
        opt.flags = f
        with pytest.raises(adg.AdgError) as ei:
            adg.adg_workspace_size([p], opt)
        assert ei.value.code == adg.ADG_E_INVALID
    one = adg.adg_options()
    for f in (adg.ADG_OPT_ONE_LAUNCH, adg.ADG_OPT_ONE_LAUNCH | adg.ADG_OPT_PE_SPLIT_OFF):
        one.flags = f
        for lane_elems in (0, 2):
            one.lane_elems = lane_elems
            assert adg.adg_workspace_size([p], one) == adg.adg_workspace_size([p], off)  # never split
    for lane_elems, kernel in ((1, 0), (4, 0), (2, adg.KERNEL["stage"])):
        one.lane_elems, one.kernel = lane_elems, kernel
        with pytest.raises(adg.AdgError) as ei:
            adg.adg_workspace_size([p], one)
        assert ei.value.code == adg.ADG_E_INVALID
    one.lane_elems, one.kernel = 0, 0
    with pytest.raises(adg.AdgError) as ei:  # the local DG kernel runs one element per lane
        adg.adg_workspace_size([solver.to_problem(W.viscous_burgers_workload(1024))], one)
    assert ei.value.code in (adg.ADG_E_INVALID, adg.ADG_E_UNSUPPORTED)


def test_autotune_candidates_include_the_pe_split():
    """The tuner tries the PE-face split on and off where every asynchronous
    PE size holds a window of 4 K S elements, and leaves it to the library
    elsewhere (no asynchronous face, or the local DG kernel)."""
    from paper_2404_03399_amd import autotune
    w = W.c2_advection_large("adg_at", n_elem=4096)          # RK4, PE size 256
    c = autotune.configs([w])
    assert {(r, k) for r, k, _ in c} == {(1, 1), (1, 2), (2, 1), (2, 2), (4, 1), (4, 2)}
    assert all({(r, k, True), (r, k, False)} <= set(c) for r in (1, 2, 4) for k in (1, 2))
    small = replace(w, pe_size=24)                           # holds a one-step window (16), not a two-step one (32)
    c = autotune.configs([small])
    assert (1, 1, True) in c and (1, 2, None) in c and (1, 2, True) not in c
    assert all(sp is None for _, _, sp in autotune.configs([replace(w, scheme="dg")]))
