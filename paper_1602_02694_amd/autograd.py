"""torch.autograd binding of the RK3 trajectory and its hand-written adjoint.

``WLSENOSteps.apply(u0, solver, dt, n_steps, ckpt_every)`` returns u(T) after
``n_steps`` TVD RK3 steps of the WLS-ENO scheme, keeping checkpoints
(``wlseno_step_record``); its backward runs the library's reverse sweep over
them (``wlseno_step_adjoint_recorded``), or the full checkpointed adjoint if
the solver recorded another trajectory in between.  Both directions run in
the HIP kernels; this module only moves tensors.
"""

from __future__ import annotations

import torch


class WLSENOSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, dt, n_steps, ckpt_every=10):
        u = u0.detach().clone().contiguous()
        solver.step_record(u, dt, n_steps, ckpt_every)
        solver._record_tag = object()
        ctx.tag = solver._record_tag
        ctx.solver = solver
        ctx.args = (float(dt), int(n_steps), int(ckpt_every))
        ctx.save_for_backward(u0.detach().contiguous())
        return u

    @staticmethod
    def backward(ctx, gT):
        (u0,) = ctx.saved_tensors
        dt, n_steps, ckpt_every = ctx.args
        if getattr(ctx.solver, "_record_tag", None) is ctx.tag:
            g0 = ctx.solver.step_adjoint_recorded(gT.contiguous())
        else:
            g0 = ctx.solver.step_adjoint(u0, dt, n_steps, gT.contiguous(), ckpt_every)
        return g0, None, None, None, None


def trajectory(u0, solver, dt, n_steps, ckpt_every=10):
    """u(T) with gradients flowing to u0 through the hand-written adjoint."""
    return WLSENOSteps.apply(u0, solver, dt, n_steps, ckpt_every)
