"""torch.autograd.Function around the STMG solve and its adjoint.

`STMGFunction.apply(u0, nu, prob, options)` returns u(T) = U_{N,M}, the end
value of the space-time solution for initial data u0 and diffusion
coefficient nu.  Its backward pass solves the transposed space-time system
backward in time with the same V-cycle kernels (stmg_adjoint) and returns
dL/du0 and dL/dnu.  With options["mem_budget"] smaller than the trajectory the
forward pass keeps only window checkpoints (stmg_solve_end) and the backward
pass recomputes one window at a time.

Each forward keeps its handle (workspace included: about five FP64
trajectories, or the window buffers) alive until its backward has run or the
graph is freed.  The backward releases them, so a second backward through the
same graph (retain_graph=True) raises a RuntimeError.

All numerical work runs in libstmg.so; this module only moves tensors.
"""
import torch

from . import stmg


class STMGFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, nu, prob, options=None):
        options = dict(options or {})
        p = dict(prob, nu=float(nu))
        h = stmg.Handle(p, device=u0.device, **options)
        u0c = u0.detach().to(torch.float64).contiguous()
        if h.num_windows() > 0:
            uT, _ = h.solve_end(u0c)
            ctx.save_for_backward(u0c)
            ctx.traj = None
        else:
            U, _ = h.solve(u0c)
            uT = U[-1, -1].clone()
            ctx.save_for_backward(u0c)
            ctx.traj = U
        ctx.handle = h
        return uT

    @staticmethod
    def backward(ctx, g):
        (u0c,) = ctx.saved_tensors
        h = ctx.handle
        if h is None:
            raise RuntimeError(
                "STMGFunction: backward was already run for this forward; the "
                "solver handle and trajectory are released after the first backward")
        gT = g.detach().to(torch.float64).contiguous()
        gu0, gnu, _ = h.adjoint(ctx.traj, gT, u0=u0c)
        ctx.handle = None
        ctx.traj = None
        return gu0, torch.tensor(gnu, dtype=torch.float64, device=gu0.device), None, None


def end_value(u0, nu, prob, **options):
    """u(T) as a differentiable function of (u0, nu)."""
    if not torch.is_tensor(nu):
        nu = torch.tensor(float(nu), dtype=torch.float64, device=u0.device)
    return STMGFunction.apply(u0, nu, prob, options)
