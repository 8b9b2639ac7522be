"""GPU discrete adjoint (adg_adjoint through the C ABI) against the oracle's
reverse-mode gradient, plus properties that hold at any size: the
dot-product identity (linear advection) and central differences of the GPU
forward map."""
import sys
from dataclasses import replace

import numpy as np
import pytest

from paper_2404_03399_amd import workloads as W
from oracle import adjoint as oadj, stats, stepper

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu_grad(torch, w, u0, n, cot_fn, kernel="fused", ckpt=5):
    from paper_2404_03399_amd.solver import Solver
    s = Solver(w, kernel=kernel, n_steps_record=n, ckpt_every=ckpt)
    u = s.pack(u0)
    s.run(u, n, graph=True, record=True)
    ut = s.unpack(u)[0]
    cot = s.pack(cot_fn(ut))
    g, gs = s.adjoint(cot)
    torch.cuda.synchronize()
    out = s.unpack(g)[0], gs[0], ut
    s.close()
    return out


CASES = [
    ("adg_at", "rk4", 2, "upwind", 96, 12),
    ("adg_at", "ssprk3", 3, "upwind", 100, 20),
    ("adg", "heun", 1, "central", 64, 16),
    ("dg", "rk4", 4, "upwind", 70, 7),
    ("adg_at", "rk4", 3, "central", 300, 25),
    ("adg_at", "lsrk3", 2, "upwind", 90, 9),
    ("adg_at", "lsrk4", 3, "upwind", 120, 12),
    ("adg_at", "lsrk4", 2, "central", 96, 8),
    ("adg_at", "rk4", 1, "upwind", 96, 2),  # a PE face every other element: several job passes per wave
]


@pytest.mark.parametrize("kernel", ["fused", "stage"])
@pytest.mark.parametrize("scheme,rk,p,flux,ne,pe", CASES)
def test_adjoint_matches_oracle(torch_cuda, kernel, scheme, rk, p, flux, ne, pe):
    dt = {1: 0.05, 2: 0.02, 3: 0.005, 4: 0.002}[p] * W.TWO_PI / ne
    w = W.Workload(name="adj", scheme=scheme, rk=rk, degree=p, n_elem=ne, pe_size=pe, flux=flux,
                   probs=W.DELAYS_C2, seed=11, dt=dt, speed=1.3, ic=W.PAPER_MULTISINE)
    n = 23
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(4).standard_normal(u0.shape)
    _say(f"adjoint {scheme} {rk} p={p} {flux} N={ne} pe={pe} steps={n} kernel={kernel}")
    ut_o, g_o, ga_o = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    g, ga, ut = _gpu_grad(torch_cuda, w, u0, n, lambda x: x - ref, kernel=kernel, ckpt=5)
    assert stats.rel_l2(ut, ut_o) <= 1e-12
    assert stats.rel_l2(g, g_o) <= 1e-12, stats.rel_l2(g, g_o)
    assert abs(ga - ga_o) <= 1e-12 * max(1.0, abs(ga_o)), (ga, ga_o)


@pytest.mark.parametrize("n", [22, 23])
@pytest.mark.parametrize("scheme,rk,p,flux,ne,pe", CASES)
def test_two_step_reverse_matches_oracle(torch_cuda, scheme, rk, p, flux, ne, pe, n):
    """dJ/du0 alone for linear advection: with two fused steps per launch the
    reverse sweep takes two steps per launch too (no forward recomputation).
    It matches the oracle and, bitwise, the one-step reverse sweep; an odd
    step count leaves one single step at the end."""
    from paper_2404_03399_amd.solver import Solver
    dt = {1: 0.05, 2: 0.02, 3: 0.005, 4: 0.002}[p] * W.TWO_PI / ne
    w = W.Workload(name="adj2", scheme=scheme, rk=rk, degree=p, n_elem=ne, pe_size=pe, flux=flux,
                   probs=W.DELAYS_C2, seed=11, dt=dt, speed=1.3, ic=W.PAPER_MULTISINE)
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(4).standard_normal(u0.shape)
    _say(f"two-step reverse {scheme} {rk} p={p} {flux} N={ne} pe={pe} steps={n}")
    _, g_o, _ = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    out = {}
    for K in (1, 2):
        s = Solver(w, kernel="fused", n_steps_record=n, ckpt_every=5, fused_steps=K)
        u = s.pack(u0)
        s.run(u, n, graph=True, record=True)
        cot = s.pack(s.unpack(u)[0] - ref)
        g, gs = s.adjoint(cot, want_speed=False)
        torch_cuda.cuda.synchronize()
        assert gs is None
        out[K] = s.unpack(g)[0]
        s.close()
    assert np.array_equal(out[1], out[2])
    assert stats.rel_l2(out[2], g_o) <= 1e-12, stats.rel_l2(out[2], g_o)


@pytest.mark.parametrize("kernel", ["fused", "stage"])
@pytest.mark.parametrize("rk,p,per_stage", [("ssprk3", 2, True), ("ssprk3", 2, False), ("rk4", 3, True),
                                            ("heun", 1, False), ("lsrk3", 2, True), ("lsrk4", 2, True)])
def test_burgers_adjoint_matches_oracle(torch_cuda, kernel, rk, p, per_stage):
    # N = 128 spans several fused-adjoint tiles (64 - 2(2S - 1) elements each)
    w = replace(W.c3_burgers(n_elem=128, n_steps=0, sigma=0.02), pe_size=16, per_stage=per_stage, rk=rk,
                degree=p)
    n = 30
    u0 = stepper.initial_state(w)
    ref = 0.25 * np.ones_like(u0)
    _say(f"burgers adjoint N=128 {rk} p={p} steps={n} per_stage={per_stage} kernel={kernel}")
    _, g_o, _ = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    g, _, _ = _gpu_grad(torch_cuda, w, u0, n, lambda x: x - ref, kernel=kernel, ckpt=7)
    assert stats.rel_l2(g, g_o) <= 1e-12


@pytest.mark.parametrize("kernel", ["fused", "stage"])
def test_checkpoint_interval_does_not_change_gradient(torch_cuda, kernel):
    # fused: segments are recomputed by the fused step kernel from the
    # checkpointed state and PE-face records, so the states, and with them the
    # gradients, are bitwise those of the recorded run for any interval.
    # stage: the per-stage recompute rounds differently from the recorded
    # run's kernel only in the order of operations: equal to rounding.
    w = W.c2_advection_large("adg_at", n_elem=2048)
    u0 = stepper.initial_state(w)
    _say(f"checkpoint intervals 1, 7, 64 on N=2048, 40 steps, kernel={kernel}")
    outs = [_gpu_grad(torch_cuda, w, u0, 40, lambda x: x, kernel=kernel, ckpt=c) for c in (1, 7, 64)]
    for g, ga, _ in outs[1:]:
        if kernel == "fused":
            assert np.array_equal(g, outs[0][0]) and ga == outs[0][1]
        else:
            assert stats.rel_l2(g, outs[0][0]) <= 1e-13
            assert abs(ga - outs[0][1]) <= 1e-13 * max(1.0, abs(ga))
    # same interval twice: bitwise reproducible
    again = _gpu_grad(torch_cuda, w, u0, 40, lambda x: x, kernel=kernel, ckpt=7)
    assert np.array_equal(again[0], outs[1][0]) and again[1] == outs[1][1]


@pytest.mark.parametrize("lane_elems", [1, 2, 4])
def test_fused_adjoint_lane_elems_and_batch(torch_cuda, lane_elems):
    """A batched recording (degrees 1..4, different speeds, meshes and PE
    sizes, forward with R elements per lane) against the oracle problem by
    problem; the reverse step with dJ/da runs one element per lane.  dJ/du0
    without dJ/da (two reverse steps per launch, min(R, 2) elements per lane)
    is bitwise the same."""
    from paper_2404_03399_amd.solver import Solver
    specs = [(1, 90, 15, 1.3, "ssprk3"), (2, 128, 16, 0.7, "ssprk3"), (3, 75, 5, -1.1, "ssprk3"),
             (4, 64, 8, 2.0, "ssprk3")]
    ws = []
    for p, ne, pe, a, rk in specs:
        dt = {1: 0.05, 2: 0.02, 3: 0.005, 4: 0.002}[p] * W.TWO_PI / ne / abs(a)
        ws.append(W.Workload(name=f"b{p}", scheme="adg_at", rk=rk, degree=p, n_elem=ne, pe_size=pe,
                             flux="upwind", probs=W.DELAYS_C2, seed=100 + p, dt=dt, speed=a,
                             ic=W.PAPER_MULTISINE))
    n = 17
    _say(f"batched fused adjoint, 4 problems, R={lane_elems}, {n} steps")
    s = Solver(ws, n_steps_record=n, ckpt_every=6, lane_elems=lane_elems)
    u0s = [stepper.initial_state(w) for w in ws]
    refs = [np.random.default_rng(7 + i).standard_normal(u.shape) for i, u in enumerate(u0s)]
    u = s.pack(u0s)
    s.run(u, n, graph=True, record=True)
    uts = s.unpack(u)
    cot = s.pack([ut - r for ut, r in zip(uts, refs)])
    g, gs = s.adjoint(cot)
    # dJ/du0 alone: two reverse steps per launch over the batch's degree groups
    g2, _ = s.adjoint(cot, want_speed=False)
    torch_cuda.cuda.synchronize()
    gl, gl2 = s.unpack(g), s.unpack(g2)
    s.close()
    for i in range(len(ws)):
        assert np.array_equal(gl[i], gl2[i]), i
    for i, w in enumerate(ws):
        ut_o, g_o, ga_o = oadj.gradient(w, u0s[i], n, oadj.misfit_cotangent(refs[i]))
        assert stats.rel_l2(uts[i], ut_o) <= 1e-12
        assert stats.rel_l2(gl[i], g_o) <= 1e-12, (i, stats.rel_l2(gl[i], g_o))
        assert abs(gs[i] - ga_o) <= 1e-12 * max(1.0, abs(ga_o)), (i, gs[i], ga_o)


@pytest.mark.parametrize("rk,p,flux,ne,pe", [("rk4", 3, "upwind", 1000, 40), ("lsrk4", 2, "central", 1030, 10),
                                             ("ssprk3", 4, "upwind", 777, 7), ("heun", 1, "upwind", 2048, 2),
                                             ("lsrk3", 2, "upwind", 130, 13)])
def test_two_step_reverse_lane_elems(torch_cuda, rk, p, flux, ne, pe):
    """The two-step reverse with two elements per lane (tiles of R (64 - 2H)
    elements, halo H = 2S / R lanes) is bitwise the one-element reverse, over
    several tiles with a ragged last one, an odd mesh (a lane's two elements
    straddle the periodic wrap), a PE face every other element, and a mesh
    shorter than one wave's extent; both match the oracle."""
    from paper_2404_03399_amd.solver import Solver
    dt = {1: 0.05, 2: 0.02, 3: 0.005, 4: 0.002}[p] * W.TWO_PI / ne
    w = W.Workload(name="adj2r", scheme="adg_at", rk=rk, degree=p, n_elem=ne, pe_size=pe, flux=flux,
                   probs=W.DELAYS_C2, seed=21, dt=dt, speed=0.9, ic=W.PAPER_MULTISINE)
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(5).standard_normal(u0.shape)
    n = 22
    _say(f"two-step reverse R=1 vs 2: {rk} p={p} {flux} N={ne} pe={pe} steps={n}")
    out = {}
    for R in (1, 2):
        s = Solver(w, kernel="fused", n_steps_record=n, ckpt_every=5, fused_steps=2, lane_elems=R)
        u = s.pack(u0)
        s.run(u, n, graph=True, record=True)
        cot = s.pack(s.unpack(u)[0] - ref)
        g, _ = s.adjoint(cot, want_speed=False)
        torch_cuda.cuda.synchronize()
        out[R] = s.unpack(g)[0]
        s.close()
    assert np.array_equal(out[1], out[2])
    _, g_o, _ = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    assert stats.rel_l2(out[2], g_o) <= 1e-12, stats.rel_l2(out[2], g_o)


@pytest.mark.parametrize("kernel", ["fused", "stage"])
@pytest.mark.parametrize("equation", ["advection", "burgers"])
def test_gradient_without_speed_is_identical(torch_cuda, kernel, equation):
    """adg_adjoint with h_grad_speed = NULL (linear advection: no forward
    recomputation) gives bitwise the same dJ/du0, and a second adjoint call
    on the same recording repeats the first bitwise."""
    from paper_2404_03399_amd.solver import Solver
    if equation == "advection":
        w = replace(W.c2_advection_large("adg_at", n_elem=700), pe_size=10)
    else:
        w = replace(W.c3_burgers(n_elem=300, n_steps=0, sigma=0.02), pe_size=12)
    n = 37
    _say(f"adjoint without dJ/da, {equation}, kernel={kernel}")
    s = Solver(w, kernel=kernel, n_steps_record=n, ckpt_every=9)
    u = s.initial_state()
    s.run(u, n, graph=True, record=True)
    cot = s.pack(np.random.default_rng(3).standard_normal((w.n_elem, w.degree + 1)))
    g1, gs1 = s.adjoint(cot)
    g2, gs2 = s.adjoint(cot, want_speed=False)
    g3, gs3 = s.adjoint(cot)
    torch_cuda.cuda.synchronize()
    assert gs2 is None
    a1, a2, a3 = s.unpack(g1)[0], s.unpack(g2)[0], s.unpack(g3)[0]
    assert np.array_equal(a1, a2) and np.array_equal(a1, a3) and gs1 == gs3
    s.close()


@pytest.mark.parametrize("kernel", ["fused", "stage"])
def test_adjoint_with_communication_avoiding_cycle(torch_cuda, kernel):
    w = W.Workload(name="adj_caa", scheme="adg_at", rk="rk4", degree=2, n_elem=120, pe_size=10,
                   probs=W.DELAYS_UNIFORM3, caa=True, per_stage=False, dt=0.01 * W.TWO_PI / 120,
                   speed=1.1, ic=W.PAPER_MULTISINE)
    n = 21
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(8).standard_normal(u0.shape)
    _say(f"adjoint with the communication-avoiding cycle, kernel={kernel}")
    _, g_o, ga_o = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    g, ga, _ = _gpu_grad(torch_cuda, w, u0, n, lambda x: x - ref, kernel=kernel, ckpt=4)
    assert stats.rel_l2(g, g_o) <= 1e-12
    assert abs(ga - ga_o) <= 1e-12 * max(1.0, abs(ga_o))


def test_stepping_after_adjoint_continues_the_run(torch_cuda):
    """adg_adjoint restores the PE-face records of the current step: stepping
    on afterwards gives bitwise the run that never called the adjoint."""
    from paper_2404_03399_amd.solver import Solver
    w = W.c2_advection_large("adg_at", n_elem=1000)
    w = replace(w, pe_size=8)
    _say("continue after adjoint, N=1000, 30 + 21 steps")
    s = Solver(w, n_steps_record=30, ckpt_every=8)
    u = s.initial_state()
    s.run(u, 30, graph=True, record=True)
    s.adjoint(u.clone())
    s.run(u, 21, graph=False)
    ref = Solver(w)
    v = ref.initial_state()
    ref.run(v, 51, graph=False)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(s.unpack(u)[0], ref.unpack(v)[0])
    s.close()
    ref.close()


def test_autograd_function(torch_cuda):
    torch = torch_cuda
    from paper_2404_03399_amd.autograd import ADGFunction
    from paper_2404_03399_amd.solver import Solver
    w = W.c2_advection_large("adg_at", n_elem=1024)
    n = 20
    u0 = stepper.initial_state(w)
    ref = np.zeros_like(u0)
    _, g_o, ga_o = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    s = Solver(w)
    x = s.pack(u0).requires_grad_(True)
    speed = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    _say("autograd ADG-AT N=1024 20 steps")
    ut = ADGFunction.apply(x, speed, w, n)
    loss = 0.5 * (ut ** 2).sum()
    loss.backward()
    g = s.unpack(x.grad)[0]
    assert stats.rel_l2(g, g_o) <= 1e-12
    # dJ/da is one scalar summed over ~10^6 terms of both signs; its rounding
    # error is bounded relative to the summands' scale, not to the result
    assert abs(float(speed.grad) - ga_o) <= 1e-11 * max(1.0, abs(ga_o))
    s.close()


def test_full_size_dot_product_and_speed_fd(torch_cuda):
    """2^20 elements, p=3, RK4, ADG-AT, checkpoint every 64 steps (the
    adjoint workload's shape, 200 steps): <G v, c> = <v, G^T c> and dJ/da
    against a central difference of the GPU forward map."""
    torch = torch_cuda
    from paper_2404_03399_amd.solver import Solver
    w = W.c5_adjoint_advection(n_steps=200)
    n = 200
    rng = np.random.default_rng(0)
    _say("full-size adjoint dot product, N=2^20, 200 steps")
    s = Solver(w, n_steps_record=n, ckpt_every=64)
    v = s.initial_state()
    c = s.pack(rng.standard_normal((w.n_elem, w.degree + 1)))
    u = v.clone()
    s.run(u, n, graph=True, record=True)
    gtc, ga = s.adjoint(c)
    torch.cuda.synchronize()
    lhs = float((u * c).sum())
    rhs = float((v * gtc).sum())
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs)), (lhs, rhs)
    # J = <u_T, c> is linear in u0; its speed derivative by central differences
    def J(speed):
        so = Solver(replace(w, speed=speed))
        uu = v.clone()
        so.run(uu, n, graph=True)
        val = float((uu * c).sum())
        so.close()
        return val
    h = 1e-4
    fd = (J(1.0 + h) - J(1.0 - h)) / (2 * h)
    assert abs(ga[0] - fd) <= 1e-6 * max(1.0, abs(fd)), (ga[0], fd)
    s.close()


def test_adjoint_past_2gib_planes(torch_cuda):
    """2^26 elements, p=3 (planes of one state span 2 GiB, so every kernel
    takes its 64-bit-address path instead of the buffer resources): the
    dot-product identity <G v, c> = <v, G^T c> for the one-step and the
    two-step reverse, and both give bitwise the same dJ/du0."""
    torch = torch_cuda
    from paper_2404_03399_amd.solver import Solver
    w = W.c5_adjoint_advection(n_elem=1 << 26, n_steps=6)
    n = 6
    assert (w.degree + 1) * w.n_elem * 8 >= 1 << 31
    _say("adjoint past 2 GiB planes, N=2^26, 6 steps, one- and two-step reverse")
    out = {}
    for K in (1, 2):
        s = Solver(w, n_steps_record=n, ckpt_every=3, fused_steps=K)
        v = s.initial_state()
        c = torch.sin(3.0 * v) + 0.25
        u = v.clone()
        s.run(u, n, graph=False, record=True)
        gtc, _ = s.adjoint(c, want_speed=False)
        torch.cuda.synchronize()
        lhs = float((u * c).sum())
        rhs = float((v * gtc).sum())
        assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs)), (K, lhs, rhs)
        out[K] = gtc.clone()
        s.close()
        del v, c, u, gtc
        torch.cuda.empty_cache()
    assert torch.equal(out[1], out[2])


def test_burgers_gradient_against_central_difference(torch_cuda):
    """Burgers (p=2, LLF, ADG-AT q=3, SSP-RK3) on 2^10 elements over 100
    steps, checkpoint every 16: <dJ/du0, v> against a central difference of
    the GPU forward map along a random direction v, J = 1/2 ||u(T)||^2."""
    torch = torch_cuda
    from paper_2404_03399_amd.solver import Solver
    w = replace(W.c5_adjoint_burgers(n_elem=1 << 10, n_steps=100), pe_size=64)
    n = 100
    rng = np.random.default_rng(1)
    _say("Burgers gradient vs central difference, N=1024, 100 steps")
    s = Solver(w, n_steps_record=n, ckpt_every=16)
    u0 = s.initial_state()
    v = s.pack(rng.standard_normal((w.n_elem, w.degree + 1)))
    u = u0.clone()
    s.run(u, n, graph=True, record=True)
    g, _ = s.adjoint(u.clone(), want_speed=False)
    torch.cuda.synchronize()
    s.close()

    def J(x0):
        so = Solver(w)
        uu = x0.clone()
        so.run(uu, n, graph=True)
        torch.cuda.synchronize()
        so.close()
        return 0.5 * float((uu * uu).sum())
    h = 1e-6
    fd = (J(u0 + h * v) - J(u0 - h * v)) / (2 * h)
    ad = float((g * v).sum())
    assert abs(ad - fd) <= 1e-6 * max(1.0, abs(fd)), (ad, fd)
