"""torch.autograd.Function over the unrolled iteration (C, b) -> u_T.

forward runs T iterations of Algorithm 1 (fixed rho, from X_k = Lambda_k = 0)
through sdp_unrolled_forward with checkpoints every `ckpt_every` iterations;
backward calls sdp_vjp, the hand-written reverse sweep.  Tensors use the
concatenated compact layout of the batch (c and u: lower pattern values of
every instance one after the other; b: the m_i right-hand sides).  Gradients
are Euclidean on these vectors, as autograd expects.
"""
import torch

from ._native import Solver


class UnrolledADMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, b, solver: Solver, T: int, ckpt_every: int):
        c = c.detach().contiguous()
        b = b.detach().contiguous()
        solver.update_data(c, b)
        u = torch.empty(solver.total_nnz, dtype=torch.float64, device=c.device)
        solver.unrolled_forward(T, ckpt_every, u)
        ctx.solver = solver
        return u

    @staticmethod
    def backward(ctx, u_bar):
        s = ctx.solver
        u_bar = u_bar.contiguous()
        c_bar = torch.empty(s.total_nnz, dtype=torch.float64, device=u_bar.device)
        b_bar = torch.empty(s.total_m, dtype=torch.float64, device=u_bar.device)
        s.vjp(u_bar, c_bar, b_bar, euclidean=True)
        return c_bar, b_bar, None, None, None


def unrolled_admm(c, b, solver: Solver, T: int = 200, ckpt_every: int = 20):
    """u_T as a differentiable function of (c, b)."""
    return UnrolledADMM.apply(c, b, solver, T, ckpt_every)
