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
                                                  ("heun", True, "adg"), ("rk4", True, "dg")])
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
    opt.lane_elems = 2                                                  # one element per lane only
    with pytest.raises(adg.AdgError) as ei:
        adg.adg_workspace_size([p], opt)
    assert ei.value.code == adg.ADG_E_UNSUPPORTED
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
