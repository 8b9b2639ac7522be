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


@pytest.mark.parametrize("per_stage", [True, False])
def test_burgers_adjoint_matches_oracle(torch_cuda, per_stage):
    w = replace(W.c3_burgers(n_elem=128, n_steps=0, sigma=0.02), pe_size=16, per_stage=per_stage)
    n = 30
    u0 = stepper.initial_state(w)
    ref = 0.25 * np.ones_like(u0)
    _say(f"burgers adjoint N=128 steps={n} per_stage={per_stage}")
    _, g_o, _ = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    g, _, _ = _gpu_grad(torch_cuda, w, u0, n, lambda x: x - ref, ckpt=7)
    assert stats.rel_l2(g, g_o) <= 1e-12


def test_checkpoint_interval_does_not_change_gradient(torch_cuda):
    # segments are recomputed with the per-stage kernel, the recorded run used
    # the fused one: the gradients agree to rounding, not bitwise
    w = W.c2_advection_large("adg_at", n_elem=2048)
    u0 = stepper.initial_state(w)
    _say("checkpoint intervals 1, 7, 64 on N=2048, 40 steps")
    outs = [_gpu_grad(torch_cuda, w, u0, 40, lambda x: x, ckpt=c) for c in (1, 7, 64)]
    for g, ga, _ in outs[1:]:
        assert stats.rel_l2(g, outs[0][0]) <= 1e-13
        assert abs(ga - outs[0][1]) <= 1e-13 * max(1.0, abs(ga))
    # same interval twice: bitwise reproducible
    again = _gpu_grad(torch_cuda, w, u0, 40, lambda x: x, ckpt=7)
    assert np.array_equal(again[0], outs[1][0]) and again[1] == outs[1][1]


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
