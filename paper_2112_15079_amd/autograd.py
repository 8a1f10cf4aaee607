"""torch.autograd.Function for a whole velocity-Verlet trajectory.

Forward runs Eqs. (3)-(4) on the GPU; backward calls the library's discrete
adjoint (reverse sweep with checkpoint-and-recompute every K steps), which
returns the exact gradient of the discrete trajectory with respect to the
initial positions, velocities and the masses.
"""
from __future__ import annotations

import torch

from . import nbody


class VerletRun(torch.autograd.Function):
    """(r0, v0, m) -> (r_T, v_T) after ``steps`` FP64 steps of size ``dt``."""

    @staticmethod
    def forward(ctx, r0, v0, m, G, dt, steps, checkpoint_every=100):
        r = r0.detach().clone().contiguous()
        v = v0.detach().clone().contiguous()
        md = m.detach().contiguous()
        nbody.verlet_run(r, v, md, G, dt, steps, "fp64")
        ctx.save_for_backward(r0.detach(), v0.detach(), md)
        ctx.G, ctx.dt, ctx.steps, ctx.K = float(G), float(dt), int(steps), int(checkpoint_every)
        return r, v

    @staticmethod
    def backward(ctx, grad_r, grad_v):
        r0, v0, m = ctx.saved_tensors
        if grad_r is None:
            grad_r = torch.zeros_like(r0)
        if grad_v is None:
            grad_v = torch.zeros_like(v0)
        gr, gv, gm, _, _ = nbody.verlet_adjoint(r0, v0, m, ctx.G, ctx.dt, ctx.steps, ctx.K,
                                                grad_r.contiguous(), grad_v.contiguous())
        return gr, gv, gm, None, None, None, None


def verlet(r0, v0, m, G, dt, steps, checkpoint_every=100):
    """Differentiable trajectory end point (r_T, v_T)."""
    return VerletRun.apply(r0, v0, m, G, dt, steps, checkpoint_every)
