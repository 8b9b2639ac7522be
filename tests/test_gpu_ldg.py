"""Viscous Burgers in local DG form against the FP64 oracle, on the fused
kernel (q on chip, one launch per step) and on the per-stage kernels (q pass
+ flux pass): synchronous LDG, ALDG with AT2 and AT(p+1) on both PE-face
values, plain ALDG, per-step and per-stage delays, every integrator, ragged
and tiny meshes, and a batch with different viscosities."""
import sys
from dataclasses import replace

import numpy as np
import pytest

from paper_2404_03399_amd import workloads as W
from oracle import stats, stepper

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


def _w(p, rk, scheme, q, per_stage, ne=300, pe=20, nu=0.1, seed=3):
    dx = W.TWO_PI / ne
    return W.Workload(name=f"ldg_{p}_{rk}_{scheme}", equation="viscous_burgers", flux="llf", rk=rk, degree=p,
                      n_elem=ne, pe_size=pe, probs=("0.3", "0.4", "0.3"), scheme=scheme, at_levels=q,
                      per_stage=per_stage, seed=seed, viscosity=nu,
                      dt=min(0.002 * dx * dx / nu, 0.01 * dx / 6.0),  # diffusive and advective limits
                      ic=W.PAPER_MULTISINE)


CASES = [(2, "heun", "adg_at", 2, False), (2, "heun", "dg", 0, False), (1, "rk4", "adg_at", 0, True),
         (3, "ssprk3", "adg", 0, True), (2, "lsrk3", "adg_at", 3, False), (4, "rk4", "adg_at", 2, True),
         (3, "lsrk4", "adg_at", 2, True)]


@pytest.mark.parametrize("kernel", ["fused", "stage"])
@pytest.mark.parametrize("p,rk,scheme,q,per_stage", CASES)
def test_ldg_matches_oracle(torch_cuda, p, rk, scheme, q, per_stage, kernel):
    from paper_2404_03399_amd.solver import Solver
    w = _w(p, rk, scheme, q, per_stage)
    n = 17
    _say(f"viscous Burgers LDG {kernel} p={p} {rk} {scheme} q={q} per_stage={per_stage} N=300 steps={n}")
    u0 = stepper.initial_state(w)
    ref = stepper.Stepper(w).run(u0, n)
    for graph in (False, True):
        s = Solver(w, kernel=kernel)
        u = s.pack(u0)
        s.run(u, n, graph=graph)
        torch_cuda.cuda.synchronize()
        got = s.unpack(u)[0]
        s.close()
        assert stats.rel_l2(got, ref) <= 1e-12, stats.rel_l2(got, ref)
        # the solution really moved (the viscous and delayed terms acted)
        assert stats.rel_l2(got, u0) > 1e-6


@pytest.mark.parametrize("kernel", ["fused", "stage"])
def test_ldg_edge_meshes_and_batch(torch_cuda, kernel):
    from paper_2404_03399_amd.solver import Solver
    ws = [replace(_w(2, "heun", "adg_at", 2, False, ne=ne, pe=pe, nu=nu, seed=ne), name=f"b{ne}")
          for ne, pe, nu in ((7, 1, 0.05), (64, 64, 0.1), (130, 13, 0.2), (2, 1, 0.1), (1001, 7, 0.1))]
    n = 11
    _say(f"viscous Burgers LDG batch ({kernel}): N = 7, 64 (one PE), 130, 2, 1001; nu = 0.05..0.2")
    u0s = [stepper.initial_state(w) for w in ws]
    s = Solver(ws, kernel=kernel)
    u = s.pack(u0s)
    s.run(u, n, graph=False)
    torch_cuda.cuda.synchronize()
    got = s.unpack(u)
    s.close()
    for w, u0, g in zip(ws, u0s, got):
        assert stats.rel_l2(g, stepper.Stepper(w).run(u0, n)) <= 1e-12, w.name


def test_viscous_burgers_convergence(torch_cuda):
    """Fig. 11(b): LDG(2)-RK2 and ALDG(2)-AT2-RK2 converge at third order
    (against a synchronous run on an 8x finer mesh) with nearly equal errors."""
    from paper_2404_03399_amd import experiments as X
    _say("viscous Burgers convergence, N_E = 32, 64, 128, reference 1024, T = 0.1")
    r = X.viscous_burgers_convergence()
    assert r["order_dg"] <= -2.8 and r["order_adg_at"] <= -2.8, r
    assert all(a < 1.5 * d for a, d in zip(r["adg_at"], r["dg"])), r


@pytest.mark.parametrize("p,rk,scheme,q,per_stage", [(2, "heun", "adg_at", 2, False), (1, "rk4", "adg_at", 0, True)])
def test_ldg_fused_equals_stage(torch_cuda, p, rk, scheme, q, per_stage):
    """The fused kernel and the per-stage kernels agree to rounding on a mesh
    of several tiles with a ragged tail, over enough steps that every delay
    level and ring slot is used (configurations that stay stable: ALDG with
    AT(p+1), p = 3 and per-stage delays grows at the PE faces within 40
    steps here, in the oracle as on the GPU)."""
    from paper_2404_03399_amd.solver import Solver
    w = _w(p, rk, scheme, q, per_stage, ne=4080, pe=40, seed=11)
    n = 40
    _say(f"viscous Burgers LDG fused vs stage N={w.n_elem} steps={n}")
    u0 = stepper.initial_state(w)
    out = {}
    for kernel in ("fused", "stage"):
        s = Solver(w, kernel=kernel)
        u = s.pack(u0)
        s.run(u, n)
        torch_cuda.cuda.synchronize()
        out[kernel] = s.unpack(u)[0]
        s.close()
    # the increments over the run (the diffusive step limit keeps them small
    # against u itself), compared to rounding
    d_f, d_s = out["fused"] - u0, out["stage"] - u0
    assert stats.rel_l2(d_s, np.zeros_like(d_s)) > 1e-6
    assert stats.rel_l2(d_f, d_s) <= 1e-9
    ref = stepper.Stepper(w).run(u0, n)
    assert stats.rel_l2(out["fused"], ref) <= 1e-12
    assert stats.rel_l2(d_f, ref - u0) <= 1e-9


@pytest.mark.parametrize("p,rk,scheme,q,per_stage,ne,pe", [
    (2, "heun", "adg_at", 2, False, 300, 20), (1, "rk4", "adg_at", 0, True, 130, 13),
    (3, "ssprk3", "adg", 0, True, 97, 1), (2, "lsrk3", "adg_at", 3, False, 200, 8), (4, "heun", "dg", 0, False, 64, 16),
    (2, "lsrk4", "adg_at", 2, True, 150, 15)])
def test_ldg_two_steps_per_launch_bitwise(torch_cuda, p, rk, scheme, q, per_stage, ne, pe):
    """Two time steps per fused local DG launch (halo 2S; the second step's AT
    sums formed from the ring plus each lane's own level-n values) give
    bitwise the one-step results, and both match the oracle."""
    from paper_2404_03399_amd.solver import Solver
    w = _w(p, rk, scheme, q, per_stage, ne=ne, pe=pe, seed=ne + p)
    u0 = stepper.initial_state(w)
    _say(f"viscous Burgers LDG two-step launches p={p} {rk} {scheme} q={q} N={ne} pe={pe}")
    out = {}
    for K in (1, 2):
        for n, graph in ((19, False), (32, True)):
            s = Solver(w, fused_steps=K)
            u = s.pack(u0)
            s.run(u, n, graph=graph)
            torch_cuda.cuda.synchronize()
            out[K, n] = s.unpack(u)[0]
            s.close()
    assert np.array_equal(out[1, 19], out[2, 19])
    assert np.array_equal(out[1, 32], out[2, 32])
    assert stats.rel_l2(out[2, 19], stepper.Stepper(w).run(u0, 19)) <= 1e-12


@pytest.mark.parametrize("p,rk,scheme,q,per_stage,ne,pe", [
    (2, "heun", "adg_at", 2, False, 600, 20), (1, "rk4", "adg_at", 0, True, 130, 13),
    (3, "ssprk3", "adg", 0, True, 200, 2), (2, "lsrk3", "adg_at", 3, False, 800, 8),
    (4, "heun", "dg", 0, False, 64, 16), (2, "lsrk4", "adg_at", 2, True, 150, 15),
    (3, "heun", "adg_at", 3, False, 36, 4)])
def test_ldg_lane_elems_bitwise(torch_cuda, p, rk, scheme, q, per_stage, ne, pe):
    """Two and four elements per lane (tiles of R (64 - 2H) elements, halo
    H = K S / R lanes; a PE face every other element; odd meshes whose lanes
    straddle the periodic wrap; a mesh shorter than one wave's extent) give
    bitwise the one-element results at one and two steps per launch, and
    match the oracle."""
    from paper_2404_03399_amd.solver import Solver
    w = _w(p, rk, scheme, q, per_stage, ne=ne, pe=pe, seed=ne + 7 * p)
    u0 = stepper.initial_state(w)
    n = 21
    _say(f"viscous Burgers LDG lane counts p={p} {rk} {scheme} q={q} N={ne} pe={pe} steps={n}")
    out = {}
    for R in (1, 2, 4):
        if scheme != "dg" and R > pe:
            continue
        for K in (1, 2):
            s = Solver(w, kernel="fused", lane_elems=R, fused_steps=K)
            u = s.pack(u0)
            s.run(u, n, graph=(R + K) % 2 == 0)
            torch_cuda.cuda.synchronize()
            out[R, K] = s.unpack(u)[0]
            s.close()
    for key, v in out.items():
        assert np.array_equal(v, out[1, 1]), key
    assert stats.rel_l2(out[1, 1], stepper.Stepper(w).run(u0, n)) <= 1e-12


@pytest.mark.parametrize("scheme,q,probs", [("adg", 0, ("0", "0", "1")), ("adg_at", 1, ("0", "0", "0", "1")),
                                            ("adg_at", 2, ("0", "0", "1")), ("adg_at", 3, ("0", "1"))])
def test_two_step_launch_reads_no_level_written_in_it(torch_cuda, scheme, q, probs):
    """Every PE face at the largest delay L-1 with q AT levels: a two-step
    launch reads the ring down to level n + 2 - L - q from every wave holding
    the face while the owner writes levels n and n + 1.  With a small
    viscosity the time step is large enough for neighbouring levels to
    differ visibly, so a slot shared by a written and a read level would show
    against the oracle and between one and two steps per launch."""
    from paper_2404_03399_amd.solver import Solver
    w = replace(_w(2, "heun", scheme, q, False, ne=600, pe=2, nu=0.005), probs=probs)
    n = 20
    _say(f"viscous Burgers, every face at delay {len(probs) - 1}, {scheme} q={q}, N=600 pe=2 steps={n}")
    u0 = stepper.initial_state(w)
    ref = stepper.Stepper(w).run(u0, n)
    outs = []
    for K in (1, 2):
        s = Solver(w, kernel="fused", fused_steps=K)
        u = s.pack(u0)
        s.run(u, n, graph=False)
        torch_cuda.cuda.synchronize()
        outs.append(s.unpack(u)[0])
        s.close()
    assert np.array_equal(outs[0], outs[1])
    assert stats.rel_l2(outs[1], ref) <= 1e-12, stats.rel_l2(outs[1], ref)
