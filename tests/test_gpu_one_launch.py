"""One fused launch over every degree range (ADG_OPT_ONE_LAUNCH) against one
launch per range: bitwise the same states, and both meet the oracle bars.
Batches mix degrees 1-4, the a > 0 upwind form and the general form (a < 0),
PE sizes from 2 up, a problem without asynchronous faces, and odd step counts
(a batch's last step takes the one-step launch)."""
import sys

import numpy as np
import pytest

from paper_2404_03399_amd import workloads as W
from oracle import stats, stepper
from parity_bars import TOL, pe_max_rel

pytestmark = pytest.mark.gpu

SIG = {1: 0.05, 2: 0.01, 3: 0.005, 4: 0.001}


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _batch(equation, flux, rk, scheme, specs):
    ws = []
    for i, (p, ne, pe, a) in enumerate(specs):
        ic = W.MultiSine((1, 3), (1.0, 0.5), (0.2, 1.3), offset=0.5 if equation == "burgers" else 0.0)
        ws.append(W.Workload(name=f"one{i}", equation=equation, scheme=scheme, flux=flux, rk=rk, degree=p,
                             n_elem=ne, pe_size=pe, probs=W.DELAYS_C2, seed=40 + i, speed=a, ic=ic,
                             dt=SIG[4] * W.TWO_PI / 2048))
    return ws


def _run(torch, ws, u0s, n, one, graph, K=2):
    from paper_2404_03399_amd.solver import Solver
    s = Solver(ws, kernel="fused", lane_elems=2, fused_steps=K, one_launch=one, pe_split=False if one else None)
    u = s.pack(u0s)
    s.run(u, n, graph=graph)
    torch.cuda.synchronize()
    out = s.unpack(u)
    s.close()
    return out


BATCHES = {  # one equation, flux, integrator and scheme per context
    "upwind_both_forms": ("advection", "upwind", "rk4", "adg_at",
                          [(1, 640, 64, 1.0), (2, 512, 2, -0.7), (3, 1000, 40, 1.3), (4, 768, 256, 0.9),
                           (4, 330, 33, -1.1), (3, 256, 256, 1.0), (2, 900, 30, 1.0)]),  # (3, 256, 256): one PE
    "central_lsrk4": ("advection", "central", "lsrk4", "adg_at",
                      [(2, 600, 20, 1.0), (4, 500, 50, -1.0), (1, 1024, 128, 0.8)]),
    "burgers_ssprk3": ("burgers", "llf", "ssprk3", "adg",
                       [(3, 700, 70, 1.0), (1, 512, 16, 1.0), (2, 1001, 13, 1.0)]),
}


@pytest.mark.parametrize("name", list(BATCHES))
@pytest.mark.parametrize("n,graph", [(21, True), (16, False)])
def test_one_launch_bitwise_equals_per_range(torch_cuda, name, n, graph):
    ws = _batch(*BATCHES[name])
    u0s = [stepper.initial_state(w) for w in ws]
    _say(f"one launch vs per range: {name}, {len(ws)} problems, steps={n} graph={graph}")
    one = _run(torch_cuda, ws, u0s, n, True, graph)
    per = _run(torch_cuda, ws, u0s, n, False, graph)
    for w, u0, a, b in zip(ws, u0s, one, per):
        assert np.array_equal(a, b), w.name
        ref = stepper.Stepper(w).run(u0, n)
        assert stats.rel_l2(a, ref) <= TOL, w.name
        assert pe_max_rel(a, ref, w) <= TOL, w.name


def test_one_launch_single_step_launches(torch_cuda):
    """One step per launch: the K = 1 one-launch kernel."""
    ws = _batch(*BATCHES["upwind_both_forms"])
    u0s = [stepper.initial_state(w) for w in ws]
    n = 9
    _say(f"one launch, one step per launch, {len(ws)} problems, steps={n}")
    one = _run(torch_cuda, ws, u0s, n, True, True, K=1)
    per = _run(torch_cuda, ws, u0s, n, False, True, K=2)
    for w, a, b in zip(ws, one, per):
        assert np.array_equal(a, b), w.name


def test_one_launch_adjoint_bitwise(torch_cuda):
    """The adjoint's checkpoint segments are recomputed by the fused step:
    with one launch over every range the recorded states, and so dJ/du0 and
    dJ/da, are bitwise those of the per-range launches."""
    from paper_2404_03399_amd.solver import Solver
    ws = _batch(*BATCHES["upwind_both_forms"])
    u0s = [stepper.initial_state(w) for w in ws]
    n = 13
    _say(f"one launch, recorded run and adjoint, {len(ws)} problems, steps={n}")
    res = {}
    for one in (True, False):
        s = Solver(ws, kernel="fused", lane_elems=2, fused_steps=2, n_steps_record=n, ckpt_every=4,
                   one_launch=one, pe_split=False if one else None)
        u = s.pack(u0s)
        s.run(u, n, graph=True, record=True)
        cot = s.pack([np.cos(x) for x in s.unpack(u)])
        g, ga = s.adjoint(cot)
        torch_cuda.cuda.synchronize()
        res[one] = (s.unpack(u), s.unpack(g), list(ga))
        s.close()
    for i, w in enumerate(ws):
        assert np.array_equal(res[True][0][i], res[False][0][i]), w.name
        assert np.array_equal(res[True][1][i], res[False][1][i]), w.name
    assert res[True][2] == res[False][2]
