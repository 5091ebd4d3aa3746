"""torch.autograd bridge for K steps of the quasi-orthogonal scheme (Sec. 4.1, Algorithm 1
of Sec. 5 with a fixed step): L(V, U_0) = loss(U_K) with U_K = Phi^K(U_0; V), where the
loss is the energy E of Sec. 2.2 or the sum of the Ritz values of span U_K.

Forward and backward both run in the HIP library (qo_tape_forward / qo_tape_backward):
the forward keeps one checkpoint per step, the backward recomputes each step from its
checkpoint and applies the adjoint of the step.  This module only moves tensors."""
from __future__ import annotations

import torch


class QOStepsLoss(torch.autograd.Function):
    """L = loss(Phi^K(U_0; V)).  V: (Ng,) CUDA tensor; U0: (N, Ng) CUDA block; either may
    be float32 (a trainable float32 potential, say): the steps and the adjoint run in FP64
    and the gradients come back in each input's dtype.  solver: a binding.Solver of the
    same grid and N (precision fp64); it holds the tape between forward and backward, so
    it serves one graph at a time."""

    @staticmethod
    def forward(ctx, V, U0, solver, tau, K, loss):
        solver.set_potential(V.detach().to(torch.float64))
        solver.set_state(U0.detach().to(torch.float64).contiguous())
        L = solver.tape_forward(tau, K, loss)
        ctx.solver = solver
        ctx.dtypes = (V.dtype, U0.dtype)
        return torch.tensor(L, dtype=torch.float64, device=V.device)

    @staticmethod
    def backward(ctx, gL):
        gV, gU = ctx.solver.tape_backward(float(gL))
        return gV.to(ctx.dtypes[0]), gU.to(ctx.dtypes[1]), None, None, None, None


def steps_loss(V, U0, solver, tau, K, loss="energy"):
    """Differentiable loss of K steps; see QOStepsLoss."""
    return QOStepsLoss.apply(V, U0, solver, float(tau), int(K), loss)
