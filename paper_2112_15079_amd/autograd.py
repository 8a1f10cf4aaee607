"""torch.autograd.Function for a whole velocity-Verlet trajectory.

Forward runs Eqs. (3)-(4) on the GPU and keeps the run's checkpoints (r, v)
every K steps; backward runs the library's discrete adjoint from those
checkpoints (reverse sweep, recomputing each K-step segment), which returns
the exact gradient of the discrete trajectory with respect to the initial
positions, velocities and the masses.  The forward trajectory is computed
once.
"""
from __future__ import annotations

import torch

from . import nbody


class VerletRun(torch.autograd.Function):
    """(r0, v0, m) -> (r_T, v_T) after ``steps`` FP64 steps of size ``dt``."""

    @staticmethod
    def forward(ctx, r0, v0, m, G, dt, steps, checkpoint_every=100):
        md = m.detach().contiguous()
        r, v, ck = nbody.verlet_checkpoints(r0.detach().contiguous(), v0.detach().contiguous(),
                                            md, G, dt, steps, checkpoint_every)
        ctx.save_for_backward(ck, md)
        ctx.G, ctx.dt, ctx.steps, ctx.K = float(G), float(dt), int(steps), int(checkpoint_every)
        return r, v

    @staticmethod
    def backward(ctx, grad_r, grad_v):
        ck, m = ctx.saved_tensors
        if grad_r is None:
            grad_r = torch.zeros((3, m.shape[0]), dtype=m.dtype, device=m.device)
        if grad_v is None:
            grad_v = torch.zeros((3, m.shape[0]), dtype=m.dtype, device=m.device)
        gr, gv, gm = nbody.verlet_adjoint_from_checkpoints(ck, m, ctx.G, ctx.dt, ctx.steps, ctx.K,
                                                           grad_r.contiguous(), grad_v.contiguous())
        return gr, gv, gm, None, None, None, None


def verlet(r0, v0, m, G, dt, steps, checkpoint_every=100):
    """Differentiable trajectory end point (r_T, v_T)."""
    return VerletRun.apply(r0, v0, m, G, dt, steps, checkpoint_every)
