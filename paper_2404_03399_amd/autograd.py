"""torch.autograd.Function around the recorded forward run and the discrete
adjoint of libadg (delay schedule held fixed, dt held fixed).

    uT = ADGFunction.apply(u0, speed, workload, n_steps)

u0 is a state vector in the library's layout (Solver.pack / initial_state)
and speed a 0-d float64 tensor (the advection speed a).  backward() returns
dJ/du0 and dJ/da from adg_adjoint; when speed needs no gradient the adjoint
is asked for dJ/du0 only (for linear advection that skips the forward
recomputation).
"""
from __future__ import annotations

from dataclasses import replace

import torch

from .solver import Solver


class ADGFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, speed, workload, n_steps, ckpt_every=64, kernel="fused"):
        w = replace(workload, speed=float(speed.detach().cpu()) if torch.is_tensor(speed) else float(speed))
        s = Solver(w, kernel=kernel, n_steps_record=n_steps, ckpt_every=ckpt_every, device=u0.device)
        u = u0.detach().clone().contiguous()
        s.run(u, n_steps, graph=True, record=True)
        ctx.solver = s
        ctx.speed_is_tensor = torch.is_tensor(speed)
        ctx.speed_device = speed.device if torch.is_tensor(speed) else None
        return u

    @staticmethod
    def backward(ctx, grad_out):
        want_speed = ctx.speed_is_tensor and ctx.needs_input_grad[1]
        g, gs = ctx.solver.adjoint(grad_out.contiguous(), want_speed=want_speed)
        gspeed = None
        if want_speed:
            gspeed = torch.tensor(gs[0], dtype=torch.float64, device=ctx.speed_device)
        ctx.solver.close()
        ctx.solver = None
        return g, gspeed, None, None, None, None


def solve_with_grad(u0, speed, workload, n_steps, ckpt_every=64, kernel="fused"):
    return ADGFunction.apply(u0, speed, workload, n_steps, ckpt_every, kernel)
