"""torch.autograd.Function around the forward and adjoint sweeps.

``NPOGain.apply(u0, solver)`` returns the final perturbation energy
E(u^N) = <u^N, u^N>_W / 2 (the numerator of the gain, Sec. 2) as a 0-d
float64 tensor; its backward runs the checkpointed exact adjoint sweep
(Sec. 2, adjoint equations; Sec. 2.4 checkpoints) and returns the gradient
with respect to the real and imaginary parts of the stored coefficients.
All arithmetic runs in libnpo; this module only sequences the calls.
"""
import torch

from . import npo


class Solver:
    """A plan, its workspace and a checkpoint arena of ``n_ckpt`` slots."""

    def __init__(self, nr, ntheta, nz, lz, re, wo, amp, dt, t0, nsteps, n_ckpt, device="cuda"):
        self.plan = npo.Plan(nr, ntheta, nz, lz, re, wo, amp, dt, t0, nsteps, device=device)
        self.nsteps = nsteps
        self.n_ckpt = max(1, min(int(n_ckpt), nsteps))
        self.arena = self.plan.arena(self.n_ckpt)
        self.scal = torch.zeros(4, dtype=torch.float64, device=device)
        self.last_recompute = 0

    @property
    def shape(self):
        return self.plan.shape

    def checkpoint_bytes(self):
        return self.arena.numel() * 16


class NPOGain(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver):
        P = solver.plan
        u0c = u0.detach().contiguous()
        uN = P.field()
        npo.npo_forward_run(P.handle, P.ws, solver.arena, solver.n_ckpt, u0c, uN)
        npo.npo_inner(P.handle, P.ws, uN, uN, solver.scal)
        ctx.solver = solver
        ctx.save_for_backward(uN)
        return 0.5 * solver.scal[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        solver = ctx.solver
        P = solver.plan
        (uN,) = ctx.saved_tensors
        lam0 = P.field()
        solver.last_recompute = npo.npo_adjoint_run(P.handle, P.ws, solver.arena, solver.n_ckpt, uN, lam0)
        g = P.field()
        npo.npo_euclid_grad(P.handle, lam0, 1.0, g)
        return g * gJ.to(g.dtype), None


def gain_energy(u0, solver):
    """E(u^N) of the forward sweep from u0, differentiable in u0."""
    return NPOGain.apply(u0, solver)
