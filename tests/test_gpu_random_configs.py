"""GPU parity over seeded random configurations: equation and flux, scheme,
integrator, degree, mesh and PE size (every divisor class: 1, odd, powers of
two, not a multiple of the lane group), AT levels, delay distribution and
granularity, the communication-avoiding cycle, speed sign and launch shape
(R elements per lane, K steps per launch, graph or direct); random batches,
adjoints, call sequences and statistics.  Each case is compared with the
oracle and, bitwise, with other launch shapes of the same problem.

The bar is relative L2 <= 1e-12, or 30 times the oracle's own response to a
relative input perturbation of 1e-16 where that is larger: some draws are
ill-conditioned (viscous Burgers with AT of high q on the local DG fluxes
turns rounding-level differences into 1e-12 to 1e-9), and no FP64
evaluation order can agree more closely than that; a wrong term or index
moves the result by orders of magnitude more.  Where even that response
exceeds 1e-8 (an unstable mode, two draws in 400) only the bitwise checks
are made.  The draws are fixed by their seeds, so every run checks the same
cases."""
import sys

import numpy as np
import pytest

# draws that blow up overflow in the oracle too; their non-finite results are
# handled explicitly (no oracle bar), so numpy's overflow warnings are noise
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

from paper_2404_03399_amd import workloads as W
from oracle import adjoint as oadj, stats, stepper
from parity_bars import TOL, derived_bars, pe_max_rel
ORACLE_BAR = 1e-8  # above this the oracle's own rounding response makes the comparison meaningless
N_CASES = 400
SIGMA = {1: 0.05, 2: 0.01, 3: 0.005, 4: 0.001}
PE_SIZES = (1, 2, 3, 4, 5, 7, 8, 9, 13, 16, 20, 31, 64, 100, 129)
DELAY_SETS = (W.DELAYS_C2, ("1/3", "1/3", "1/3"), ("0.3", "0.4", "0.3"), ("0.5", "0.5"), ("0", "0", "1"),
              ("1/8",) * 8, ("0", "0", "0", "0", "0", "0", "0", "1"), ("1",))


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def draw(case: int, large: bool = False):
    """One configuration, a pure function of the case number (large: meshes
    of 20000 to 100000 elements, so that a launch's waves start in several
    rounds and late waves meet what early ones wrote)."""
    rng = np.random.default_rng((31000 if large else 7000) + case)
    eq = str(rng.choice(["advection", "advection", "advection", "burgers", "burgers", "viscous_burgers"]))
    scheme = str(rng.choice(["dg", "adg", "adg_at", "adg_at"]))
    rk = str(rng.choice(["heun", "ssprk3", "rk4", "lsrk3"]))
    p = int(rng.integers(1, 5))
    pe = int(rng.choice(PE_SIZES))
    if large:
        n_pe = int(rng.integers(max(1, 20000 // pe), max(2, 100000 // pe) + 1))
    else:
        n_pe = int(rng.integers(1, max(2, 2000 // pe) + 1))
    ne = max(2, pe * n_pe)
    if ne % pe:
        pe = ne
    caa = scheme != "dg" and eq != "viscous_burgers" and rng.random() < 0.15
    probs = ("1/3", "1/3", "1/3") if caa else DELAY_SETS[int(rng.integers(len(DELAY_SETS)))]
    per_stage = False if caa else bool(rng.random() < 0.5)
    q = int(rng.integers(0, p + 2)) if scheme == "adg_at" else 0
    n_steps = int(rng.integers(4, 11)) if large else int(rng.integers(5, 26))
    graph = bool(rng.random() < 0.5)
    dx = W.TWO_PI / ne
    if eq == "advection":
        flux = str(rng.choice(["upwind", "upwind", "central"]))
        speed = float(rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 2.0))
        dt = SIGMA[p] * dx / abs(speed)
        ic, nu = W.PAPER_MULTISINE, 0.0
    elif eq == "burgers":
        flux, speed = "llf", 1.0
        dt = SIGMA[p] * dx / 1.5
        ic, nu = W.MultiSine((1, 2), (1.0, 0.5), (0.3, 0.9), offset=0.5), 0.0
    else:
        flux, speed = "llf", 1.0
        nu = float(rng.choice([0.02, 0.1]))
        dt = min(0.002 * dx * dx / nu, 0.01 * dx / 6.0)
        ic = W.PAPER_MULTISINE
    async_faces = scheme != "dg" and ne // pe > 1
    lanes = [r for r in (1, 2, 4) if not async_faces or r <= pe]
    R = int(rng.choice(lanes))
    K = int(rng.choice([1, 2]))
    w = W.Workload(name=f"rand{case}", equation=eq, scheme=scheme, flux=flux, rk=rk, degree=p, n_elem=ne,
                   pe_size=pe, probs=probs, seed=int(rng.integers(1 << 30)), per_stage=per_stage, caa=caa,
                   at_levels=q, speed=speed, viscosity=nu, dt=dt, ic=ic)
    return w, n_steps, R, K, graph


def same(a, b) -> bool:
    """Bitwise-equal states (a NaN of a blown-up draw matches a NaN)."""
    return np.array_equal(a, b, equal_nan=True)


def bars(w, u0, n, ref):
    """The bars for one case in both norms (relative L2, PE-face elements):
    TOL, or 30 x the oracle's own change under a rounding-level (1e-16
    relative) perturbation of the initial state; infinite where the oracle
    run itself blows up."""
    return derived_bars(w, u0, n, ref)


def tolerance(w, u0, n, ref) -> float:
    """The relative L2 bar of bars()."""
    return bars(w, u0, n, ref)[0]


def check_both(got, ref, w, tol, tol_pe):
    err = stats.rel_l2(got, ref)
    assert err <= tol, (err, tol)
    err_pe = pe_max_rel(got, ref, w)
    assert err_pe <= tol_pe, ("PE-face elements", err_pe, tol_pe)


def draw_batch(case: int):
    """Two to four problems that may share one context: the equation, flux,
    integrator, scheme and delay granularity of the first draw, each with its
    own degree, mesh, PE size, AT levels, delays, seed, speed and step."""
    rng = np.random.default_rng(9000 + case)
    first, n, _, K, graph = draw(1000 + 5 * case)
    ws = [first]
    for j in range(1, int(rng.integers(2, 5))):
        w, *_ = draw(1000 + 5 * case + j)
        q = min(w.at_levels, w.degree + 1) if first.scheme == "adg_at" else 0
        dx = W.TWO_PI / w.n_elem
        if first.equation == "advection":
            dt = SIGMA[w.degree] * dx / abs(w.speed)
        elif first.equation == "burgers":
            dt = SIGMA[w.degree] * dx / 1.5
        else:
            nu = first.viscosity
            dt = min(0.002 * dx * dx / nu, 0.01 * dx / 6.0)
        probs = first.probs if first.caa else w.probs
        ws.append(W.Workload(name=f"{first.name}_{j}", equation=first.equation, scheme=first.scheme,
                             flux=first.flux, rk=first.rk, degree=w.degree, n_elem=w.n_elem, pe_size=w.pe_size,
                             probs=probs, seed=w.seed, per_stage=first.per_stage, caa=first.caa, at_levels=q,
                             speed=w.speed if first.equation == "advection" else 1.0,
                             viscosity=first.viscosity, dt=dt, ic=first.ic))
    async_pes = [w.pe_size for w in ws if w.scheme != "dg" and w.n_elem // w.pe_size > 1]
    lanes = [r for r in (1, 2, 4) if r <= min(async_pes or [4])]
    R = int(rng.choice(lanes))
    return ws, n, R, K, graph


def _run(torch, w, u0, n, R, K, graph, kernel="fused", one_launch=False):
    from paper_2404_03399_amd.solver import Solver
    s = Solver(w, kernel=kernel, lane_elems=R, fused_steps=K, one_launch=one_launch)
    u = s.pack(u0)
    s.run(u, n, graph=graph)
    torch.cuda.synchronize()
    out = s.unpack(u)
    s.close()
    return out if isinstance(w, (list, tuple)) else out[0]


def test_batch_draws_share_what_a_context_requires():
    for c in range(N_BATCH):
        ws, n, R, K, _ = draw_batch(c)
        assert 2 <= len(ws) <= 4
        for w in ws:
            assert (w.equation, w.flux, w.rk, w.scheme, w.per_stage, w.caa) == \
                (ws[0].equation, ws[0].flux, ws[0].rk, ws[0].scheme, ws[0].per_stage, ws[0].caa)
            assert w.n_elem % w.pe_size == 0 and 0 <= w.at_levels <= w.degree + 1
            if w.scheme != "dg" and w.n_elem // w.pe_size > 1:
                assert R <= w.pe_size


def test_draws_are_valid_and_varied():
    """The draw covers every equation, scheme, integrator and launch shape."""
    ws = [draw(c) for c in range(N_CASES)]
    seen = {(w.equation, w.scheme, w.rk) for w, *_ in ws}
    assert {e for e, _, _ in seen} == {"advection", "burgers", "viscous_burgers"}
    assert {s for _, s, _ in seen} == {"dg", "adg", "adg_at"}
    assert {r for _, _, r in seen} == {"heun", "ssprk3", "rk4", "lsrk3"}
    assert {(R, K) for _, _, R, K, _ in ws} >= {(1, 1), (1, 2), (2, 1), (2, 2), (4, 1), (4, 2)}
    for w, n, R, K, _ in ws:
        assert w.n_elem % w.pe_size == 0 and n >= 5


def test_tolerance_is_tight_except_for_ill_conditioned_draws():
    """The relative L2 bar stays at 1e-12 for all but a few draws, all of them
    viscous Burgers with AT on the local DG fluxes (high q), where the oracle
    itself answers a rounding-level perturbation with 1e-12 or more; in two
    of them an unstable mode takes that to 1e-5 and only the bitwise checks
    remain meaningful.  The PE-face elementwise bar, which sees the AT
    weights' amplification undiluted, relaxes on a few more, all of them
    (viscous) Burgers."""
    relaxed, relaxed_pe = [], []
    for c in range(N_CASES):
        w, n, *_ = draw(c)
        u0 = stepper.initial_state(w)
        tol, tol_pe = bars(w, u0, n, stepper.Stepper(w).run(u0, n))
        if tol > TOL:
            relaxed.append((c, tol))
            assert w.equation == "viscous_burgers" and w.scheme == "adg_at", (c, tol)
        if tol_pe > TOL:
            relaxed_pe.append((c, tol_pe))
            assert w.equation in ("burgers", "viscous_burgers"), (c, tol_pe)
    assert len(relaxed) <= N_CASES // 20, relaxed
    assert len(relaxed_pe) <= N_CASES // 20, relaxed_pe
    assert sum(t > ORACLE_BAR for _, t in relaxed) <= N_CASES // 100, relaxed


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(N_CASES))
def test_random_config_matches_oracle(torch_cuda, case):
    w, n, R, K, graph = draw(case)
    _say(f"random case {case}: {w.equation} {w.flux} {w.scheme} {w.rk} p={w.degree} N={w.n_elem} "
         f"pe={w.pe_size} q={w.at_levels} L={w.n_delays} per_stage={w.per_stage} caa={w.caa} "
         f"a={w.speed:.3f} steps={n} R={R} K={K} graph={graph}")
    u0 = stepper.initial_state(w)
    ref = stepper.Stepper(w).run(u0, n)
    got = _run(torch_cuda, w, u0, n, R, K, graph)
    assert same(got, _run(torch_cuda, w, u0, n, 1, 1, False))
    assert same(got, _run(torch_cuda, w, u0, n, R, 3 - K, not graph))
    tol, tol_pe = bars(w, u0, n, ref)
    if tol <= ORACLE_BAR:
        check_both(got, ref, w, tol, tol_pe)
        # the per-stage kernels: the same map, rounded in their own order
        st = _run(torch_cuda, w, u0, n, 0, 0, graph, kernel="stage")
        check_both(st, ref, w, tol, tol_pe)


N_LS4 = 60


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(N_LS4))
def test_random_lsrk4_config_matches_oracle(torch_cuda, case):
    """Random draws run with the five-stage fourth-order 2N scheme (the other
    draws keep their own integrators, so their seeds stay fixed): launch
    shapes bitwise, both kernel families against the oracle."""
    from dataclasses import replace
    w, n, R, K, graph = draw(5000 + case)
    w = replace(w, rk="lsrk4", name=f"ls4_{case}")
    _say(f"random lsrk4 case {case}: {w.equation} {w.flux} {w.scheme} p={w.degree} N={w.n_elem} "
         f"pe={w.pe_size} q={w.at_levels} L={w.n_delays} per_stage={w.per_stage} caa={w.caa} "
         f"steps={n} R={R} K={K} graph={graph}")
    u0 = stepper.initial_state(w)
    ref = stepper.Stepper(w).run(u0, n)
    got = _run(torch_cuda, w, u0, n, R, K, graph)
    assert same(got, _run(torch_cuda, w, u0, n, 1, 1, False))
    assert same(got, _run(torch_cuda, w, u0, n, R, 3 - K, not graph))
    tol, tol_pe = bars(w, u0, n, ref)
    if tol <= ORACLE_BAR:
        check_both(got, ref, w, tol, tol_pe)
        st = _run(torch_cuda, w, u0, n, 0, 0, graph, kernel="stage")
        check_both(st, ref, w, tol, tol_pe)


N_LARGE = 24


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(N_LARGE))
def test_random_large_config_matches_oracle(torch_cuda, case):
    """Large meshes: the launch shapes still agree bitwise and the oracle
    still agrees, with waves dispatched over several rounds."""
    w, n, R, K, graph = draw(case, large=True)
    _say(f"random large case {case}: {w.equation} {w.flux} {w.scheme} {w.rk} p={w.degree} N={w.n_elem} "
         f"pe={w.pe_size} q={w.at_levels} L={w.n_delays} per_stage={w.per_stage} caa={w.caa} "
         f"steps={n} R={R} K={K} graph={graph}")
    u0 = stepper.initial_state(w)
    ref = stepper.Stepper(w).run(u0, n)
    got = _run(torch_cuda, w, u0, n, R, K, graph)
    assert same(got, _run(torch_cuda, w, u0, n, 1, 1, False))
    assert same(got, _run(torch_cuda, w, u0, n, R, 3 - K, not graph))
    tol, tol_pe = bars(w, u0, n, ref)
    if tol <= ORACLE_BAR:
        check_both(got, ref, w, tol, tol_pe)


N_BATCH = 80


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(N_BATCH))
def test_random_batch_matches_single_runs(torch_cuda, case):
    """A context over several different problems advances each exactly as a
    context of its own would (bitwise), at any launch shape; with two
    elements per lane also in one launch over every degree range."""
    ws, n, R, K, graph = draw_batch(case)
    _say(f"random batch {case}: {len(ws)} x {ws[0].equation} {ws[0].flux} {ws[0].scheme} {ws[0].rk}, "
         f"p={[w.degree for w in ws]} N={[w.n_elem for w in ws]} pe={[w.pe_size for w in ws]} "
         f"steps={n} R={R} K={K} graph={graph}")
    u0s = [stepper.initial_state(w) for w in ws]
    outs = _run(torch_cuda, ws, u0s, n, R, K, graph)
    for w, u0, got in zip(ws, u0s, outs):
        assert same(got, _run(torch_cuda, w, u0, n, 1, 1, False)), w.name
    if R == 2 and ws[0].equation != "viscous_burgers":
        one = _run(torch_cuda, ws, u0s, n, 2, K, not graph, one_launch=True)
        for w, a, b in zip(ws, outs, one):
            assert same(a, b), w.name


N_ADJ = 100


def draw_adjoint(case: int, large: bool = False):
    """A forward draw of an equation with an adjoint (not viscous Burgers),
    with a kernel family and a checkpoint interval."""
    rng = np.random.default_rng((23000 if large else 11000) + case)
    for attempt in range(20):
        w, n, R, K, graph = draw(2000 + 20 * case + attempt, large=large)
        if w.equation != "viscous_burgers":
            break
    kernel = "stage" if rng.random() < 0.3 else "fused"
    ckpt = int(rng.choice([1, 2, 5, 7, 64]))
    return w, n, R, K, graph, kernel, ckpt


def adjoint_tolerance(w, u0, n, ref, g_o, ga_o, ga_scale):
    """Bars for dJ/du0 and dJ/da.  dJ/du0: 1e-12, or 30 x the oracle's own
    change under a rounding-level perturbation of the initial state.
    dJ/da is a cancelling sum over every DOF, stage and step of lambda_K K / a
    (on large meshes 1e4 times smaller than the sum of |terms|, ga_scale), so
    per-term relative differences of lambda_K and K (1e-12 from the reverse
    sweep's own rounding) reach it undiminished: its bar is 1e-11 of the sum
    of |terms|, far below what a wrong term would cost."""
    rng = np.random.default_rng(54321)
    u1 = u0 * (1.0 + 1e-16 * rng.standard_normal(u0.shape))
    _, g1, ga1 = oadj.gradient(w, u1, n, oadj.misfit_cotangent(ref))
    tol_g = max(TOL, 30.0 * stats.rel_l2(g1, g_o))
    tol_a = max(1e-12 * max(1.0, abs(ga_o)), 1e-11 * ga_scale, 30.0 * abs(ga1 - ga_o))
    return tol_g, tol_a


def test_adjoint_draws_have_adjoints():
    kinds = set()
    for c in range(N_ADJ):
        w, n, R, K, graph, kernel, ckpt = draw_adjoint(c)
        assert w.equation in ("advection", "burgers")
        kinds.add((w.equation, kernel))
    assert kinds == {("advection", "fused"), ("advection", "stage"), ("burgers", "fused"), ("burgers", "stage")}


N_ADJ_LARGE = 12


@pytest.mark.gpu
@pytest.mark.parametrize("case,large", [(c, False) for c in range(N_ADJ)] + [(c, True) for c in range(N_ADJ_LARGE)])
def test_random_adjoint_matches_oracle(torch_cuda, case, large):
    """Recorded run (any launch shape, graph or not, any checkpoint interval)
    and adg_adjoint against the oracle's reverse mode; dJ/du0 without dJ/da
    is bitwise the full call's.  The large draws put the reverse sweep's
    waves over several dispatch rounds."""
    from paper_2404_03399_amd.solver import Solver
    w, n, R, K, graph, kernel, ckpt = draw_adjoint(case, large)
    _say(f"random adjoint {case} large={large}: {w.equation} {w.flux} {w.scheme} {w.rk} p={w.degree} N={w.n_elem} "
         f"pe={w.pe_size} q={w.at_levels} L={w.n_delays} per_stage={w.per_stage} caa={w.caa} a={w.speed:.3f} "
         f"steps={n} kernel={kernel} C={ckpt} R={R} K={K} graph={graph}")
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(case).standard_normal(u0.shape)
    ut_o, g_o, ga_o, ga_scale = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref), with_scale=True)
    fused = kernel == "fused"
    s = Solver(w, kernel=kernel, n_steps_record=n, ckpt_every=ckpt, lane_elems=R if fused else 0,
               fused_steps=K if fused else 0)
    u = s.pack(u0)
    s.run(u, n, graph=graph, record=True)
    ut = s.unpack(u)[0]
    cot = s.pack(ut - ref)
    g, gs = s.adjoint(cot)
    g2, gs2 = s.adjoint(cot, want_speed=False)
    torch_cuda.cuda.synchronize()
    gl, gl2 = s.unpack(g)[0], s.unpack(g2)[0]
    s.close()
    assert gs2 is None and same(gl, gl2)
    if tolerance(w, u0, n, ut_o) > ORACLE_BAR:
        return  # the forward run is ill-conditioned or blows up: only the bitwise check holds
    tol_g, tol_a = adjoint_tolerance(w, u0, n, ref, g_o, ga_o, ga_scale)
    assert stats.rel_l2(ut, ut_o) <= tolerance(w, u0, n, ut_o)
    assert stats.rel_l2(gl, g_o) <= tol_g, (stats.rel_l2(gl, g_o), tol_g)
    if w.equation == "advection":
        assert abs(gs[0] - ga_o) <= tol_a, (gs[0], ga_o, tol_a)


N_SEQ = 80


def draw_sequence(case: int):
    """A configuration and a random split of its steps into calls: single
    steps and runs of 1 to 40 steps, each with or without graph replay."""
    rng = np.random.default_rng(13000 + case)
    w, _, R, K, _ = draw(4000 + case)
    calls = []
    for _ in range(int(rng.integers(3, 9))):
        if rng.random() < 0.3:
            calls.append(("step", 1, False))
        else:
            calls.append(("run", int(rng.integers(1, 41)), bool(rng.random() < 0.5)))
    return w, R, K, calls


def test_sequence_draws_mix_calls():
    kinds = set()
    for c in range(N_SEQ):
        _, _, _, calls = draw_sequence(c)
        kinds |= {(k, g, m >= 16) for k, m, g in calls}
    assert {("step", False, False), ("run", True, True), ("run", False, True), ("run", True, False)} <= kinds


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(N_SEQ))
def test_random_call_sequence_equals_one_run(torch_cuda, case):
    """Steps split over any sequence of adg_step / adg_run calls (graph or
    direct, runs shorter or longer than the captured batch) give bitwise the
    state of one uninterrupted run, which matches the oracle (where the
    oracle's own rounding response stays below 1e-8: a few long viscous
    draws grow an unstable mode and only the bitwise check is meaningful)."""
    from paper_2404_03399_amd.solver import Solver
    w, R, K, calls = draw_sequence(case)
    total = sum(m for _, m, _ in calls)
    _say(f"random call sequence {case}: {w.equation} {w.flux} {w.scheme} {w.rk} p={w.degree} N={w.n_elem} "
         f"pe={w.pe_size} R={R} K={K} calls={calls}")
    u0 = stepper.initial_state(w)
    s = Solver(w, kernel="fused", lane_elems=R, fused_steps=K)
    u = s.pack(u0)
    for kind, m, graph in calls:
        if kind == "step":
            s.step(u)
        else:
            s.run(u, m, graph=graph)
    torch_cuda.cuda.synchronize()
    assert s.steps_taken() == total
    got = s.unpack(u)[0]
    s.close()
    assert same(got, _run(torch_cuda, w, u0, total, R, K, False))
    ref = stepper.Stepper(w).run(u0, total)
    tol, tol_pe = bars(w, u0, total, ref)
    if tol <= ORACLE_BAR:
        check_both(got, ref, w, tol, tol_pe)


N_STATS = 24


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(N_STATS))
def test_random_batch_statistics_match_oracle(torch_cuda, case):
    """adg_error_stats and adg_ensemble_stats on a random batch, after a
    run, against random reference states: per problem the spatial mean and
    maximum of |u - ref| and the integral of u (Sec. 6.2 error measure), and
    per random group of problems the two-pass mean and variance of both."""
    from paper_2404_03399_amd.solver import Solver
    ws, n, R, K, graph = draw_batch(200 + case)
    rng = np.random.default_rng(17000 + case)
    n_groups = int(rng.integers(1, min(3, len(ws)) + 1))
    group = [int(g) for g in rng.integers(0, n_groups, len(ws))]
    group[:n_groups] = list(range(n_groups))  # no empty group
    _say(f"random statistics {case}: {len(ws)} x {ws[0].equation} {ws[0].scheme}, N={[w.n_elem for w in ws]} "
         f"groups={group} steps={n} R={R} K={K}")
    s = Solver(ws, kernel="fused", lane_elems=R, fused_steps=K)
    u = s.pack([stepper.initial_state(w) for w in ws])
    s.run(u, n, graph=graph)
    refs = [rng.standard_normal((w.n_elem, w.degree + 1)) for w in ws]
    r = s.pack(refs)
    got = s.error_stats(u, r)
    ens = s.ensemble_stats(u, r, group, n_groups)
    torch_cuda.cuda.synchronize()
    outs = s.unpack(u)
    s.close()
    per = []
    for w, o, rf, g in zip(ws, outs, refs, got):
        m, mx = stats.mean_abs(o, rf), stats.max_abs(o, rf)
        assert abs(g[0] - m) <= 1e-13 * max(1.0, m) and g[1] == mx
        assert abs(g[2] - stepper.Stepper(w).integral(o)) <= 1e-12 * max(1.0, np.abs(o).max() * w.length)
        per.append((m, mx))
    for gi in range(n_groups):
        vals = [per[i] for i in range(len(ws)) if group[i] == gi]
        m0, v0 = stats.ensemble_mean_var([v[0] for v in vals])
        m1, v1 = stats.ensemble_mean_var([v[1] for v in vals])
        assert abs(ens[gi][0] - m0) <= 1e-13 * m0 and abs(ens[gi][2] - m1) <= 1e-13 * m1
        assert abs(ens[gi][1] - v0) <= 1e-12 * (m0 * m0 + v0)
        assert abs(ens[gi][3] - v1) <= 1e-12 * (m1 * m1 + v1)
