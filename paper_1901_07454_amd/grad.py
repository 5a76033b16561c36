"""torch.autograd.Function over the library's discrete adjoint.

`SomaTrace.apply(theta, sim, n_steps, ckpt_every)` maps per-region channel
densities theta[cells, regions, 3] = (gbar_na, gbar_k, g_pas) (S/cm^2) to the
soma voltage of every cell after each step, trace[cells, n_steps] (mV).
Forward and backward both run in the HIP library (arb_grad_forward /
arb_grad_backward); this class only moves tensors across the ABI.

Each forward starts from the sim's state captured when the GradSim was made,
so repeated evaluations (an optimisation loop) are independent.
"""
from __future__ import annotations

import numpy as np
import torch

from . import arbmi


class GradSim:
    """A Simulation built for gradients, remembering its initial state."""

    def __init__(self, m: dict, **kw):
        kw["flags"] = kw.get("flags", 0) | arbmi.ARB_FLAG_GRADIENTS
        self.sim = arbmi.Simulation(m, **kw)
        self.state0 = self.sim.get_state()
        self.n_cells = self.sim.info["n_cells"]
        self.n_regions = len(m["cell_n_branch"]) + int(np.sum(m["cell_n_branch"]))

    def close(self):
        self.sim.close()


class SomaTrace(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, gs: GradSim, n_steps: int, ckpt_every: int):
        sim = gs.sim
        sim.set_state(gs.state0)
        sim.set_params(theta.detach().to("cpu", torch.float64).numpy())
        trace = torch.empty(gs.n_cells, n_steps, dtype=torch.float64, device=sim.stream.device)
        arbmi.arb_grad_forward(sim.h, n_steps, ckpt_every, trace)
        ctx.gs = gs
        ctx.theta_shape = theta.shape
        ctx.theta_device = theta.device
        return trace

    @staticmethod
    def backward(ctx, g):
        sim = ctx.gs.sim
        g = g.to(torch.float64).contiguous()
        if g.device != sim.stream.device:
            g = g.to(sim.stream.device)
        out = torch.empty(3 * ctx.gs.n_regions, dtype=torch.float64, device=sim.stream.device)
        arbmi.arb_grad_backward(sim.h, g, out)
        return out.view(ctx.theta_shape).to(ctx.theta_device), None, None, None


def soma_trace(theta, gs: GradSim, n_steps: int, ckpt_every: int = 100):
    return SomaTrace.apply(theta, gs, n_steps, ckpt_every)
