"""PE-face split of the fused step kernel: a launch with the PE-face paths
compiled out over every tile, then a launch over windows of 4 K S elements
centred on the PE faces that owns the 2 K S elements each face's delayed
flux can reach.  Each element is computed with the same instructions as in
the unsplit kernel, so the split and unsplit runs agree bitwise; both meet
the oracle bars.  Cases cover every integrator (the five-stage scheme fits one
window per wave, the others two or four), both launch shapes, windows that
wrap around the periodic end, a last wave with unused windows, the a > 0
upwind form and the general form, Burgers, the communication-avoiding cycle,
batches mixing degrees and a single-PE problem, and the adjoint (whose
segment recompute runs the split kernel)."""
import sys

import numpy as np
import pytest

from paper_2404_03399_amd import workloads as W
from oracle import adjoint as oadj, stats, stepper
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


def _w(ne, pe, p, rk, phys, scheme="adg_at", per_stage=True, speed=1.0, caa=False, seed=3):
    eq = "burgers" if phys == "llf" else "advection"
    ic = W.MultiSine((1, 3), (1.0, 0.5), (0.2, 1.3), offset=0.5 if eq == "burgers" else 0.0)
    probs = W.DELAYS_UNIFORM3 if caa else W.DELAYS_C2
    return W.Workload(name=f"split_{ne}_{pe}_{p}_{rk}_{phys}", equation=eq, scheme=scheme, flux=phys, rk=rk,
                      degree=p, n_elem=ne, pe_size=pe, probs=probs, seed=seed, per_stage=per_stage and not caa,
                      caa=caa, speed=speed if eq == "advection" else 1.0, ic=ic,
                      dt=SIG[p] * W.TWO_PI / ne / (1.5 if eq == "burgers" else abs(speed)))


def _run(torch, w, u0, n, split, R, K, graph):
    from paper_2404_03399_amd.solver import Solver
    s = Solver(w, kernel="fused", lane_elems=R, fused_steps=K, pe_split=split)
    u = s.pack(u0)
    s.run(u, n, graph=graph)
    torch.cuda.synchronize()
    out = s.unpack(u)
    s.close()
    return out if isinstance(w, (list, tuple)) else out[0]


CASES = [
    # ne, pe, p, rk, phys, R, K, extra
    (4096, 256, 3, "rk4", "upwind", 2, 2, {}),
    (960, 32, 3, "rk4", "upwind", 1, 2, {}),            # PE size = one two-step RK4 window
    (1320, 40, 3, "rk4", "upwind", 2, 2, {}),           # 33 PEs: the last wave has one unused window
    (1320, 40, 3, "rk4", "upwind", 4, 1, {}),
    (600, 50, 2, "ssprk3", "central", 2, 2, {}),
    (600, 50, 2, "ssprk3", "central", 1, 1, {}),
    (2000, 100, 4, "lsrk4", "upwind", 2, 2, {}),        # window 40: one per wave
    (800, 40, 3, "lsrk4", "central", 1, 1, {}),
    (700, 70, 1, "heun", "llf", 2, 2, {}),
    (900, 45, 2, "lsrk3", "llf", 1, 2, {}),
    (1024, 64, 3, "rk4", "upwind", 2, 2, {"speed": -1.3}),  # general form (a < 0)
    (1000, 50, 2, "rk4", "upwind", 2, 2, {"caa": True}),
    (1000, 50, 2, "rk4", "upwind", 2, 2, {"per_stage": False}),
    (1000, 50, 2, "rk4", "upwind", 2, 2, {"scheme": "adg"}),
]


@pytest.mark.parametrize("ne,pe,p,rk,phys,R,K,extra", CASES)
def test_split_bitwise_equals_unsplit(torch_cuda, ne, pe, p, rk, phys, R, K, extra):
    w = _w(ne, pe, p, rk, phys, **extra)
    u0 = stepper.initial_state(w)
    n = 21
    _say(f"PE split: N={ne} pe={pe} p={p} {rk} {phys} R={R} K={K} {extra} steps={n}")
    on = _run(torch_cuda, w, u0, n, True, R, K, graph=True)
    off = _run(torch_cuda, w, u0, n, False, R, K, graph=False)
    assert np.array_equal(on, off)
    ref = stepper.Stepper(w).run(u0, n)
    assert stats.rel_l2(on, ref) <= TOL
    assert pe_max_rel(on, ref, w) <= TOL


def test_split_batch_mixed(torch_cuda):
    """A batch of degrees 1-4, PE sizes from one window up, and a problem
    with a single PE: split and unsplit agree bitwise problem by problem."""
    ws = [_w(1280, 64, 1, "rk4", "upwind", seed=1), _w(960, 32, 2, "rk4", "upwind", seed=2),
          _w(2048, 256, 3, "rk4", "upwind", seed=3), _w(640, 80, 4, "rk4", "upwind", seed=4),
          _w(512, 512, 3, "rk4", "upwind", seed=5)]  # one PE: no asynchronous face
    ws = [W.replace(w, dt=SIG[4] * W.TWO_PI / 2048) for w in ws]  # one step for all
    u0s = [stepper.initial_state(w) for w in ws]
    n = 19
    _say(f"PE split batch of {len(ws)} problems, steps={n}")
    on = _run(torch_cuda, ws, u0s, n, True, 2, 2, graph=True)
    off = _run(torch_cuda, ws, u0s, n, False, 2, 2, graph=True)
    for w, u0, a, b in zip(ws, u0s, on, off):
        assert np.array_equal(a, b), w.name
        assert stats.rel_l2(a, stepper.Stepper(w).run(u0, n)) <= TOL


@pytest.mark.parametrize("phys,rk,p", [("upwind", "rk4", 3), ("llf", "ssprk3", 2)])
def test_split_adjoint_bitwise(torch_cuda, phys, rk, p):
    """Recorded run and discrete adjoint (segments recomputed by the split
    kernel from checkpoints): gradients bitwise equal with and without the
    split, and equal to the oracle's reverse mode."""
    torch = torch_cuda
    from paper_2404_03399_amd.solver import Solver
    w = _w(1280, 64, p, rk, phys, seed=7)
    u0 = stepper.initial_state(w)
    ref = np.random.default_rng(4).standard_normal(u0.shape)
    n = 23
    _say(f"PE split adjoint: {phys} {rk} p={p} N=1280 pe=64 steps={n}")
    out = {}
    for split in (True, False):
        s = Solver(w, kernel="fused", n_steps_record=n, ckpt_every=5, fused_steps=2, pe_split=split)
        u = s.pack(u0)
        s.run(u, n, graph=True, record=True)
        cot = s.pack(s.unpack(u)[0] - ref)
        g, gs = s.adjoint(cot)
        torch.cuda.synchronize()
        out[split] = (s.unpack(g)[0], gs[0])
        s.close()
    assert np.array_equal(out[True][0], out[False][0]) and out[True][1] == out[False][1]
    _, g_o, _ = oadj.gradient(w, u0, n, oadj.misfit_cotangent(ref))
    assert stats.rel_l2(out[True][0], g_o) <= 1e-12
