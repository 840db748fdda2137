"""Differentiable multi-step heat solve (torch.autograd) with a hand-written adjoint.

Forward: T backward-Euler steps A(kappa) u_n = u_{n-1}, each solved by FAS V-cycles to
a relative residual `tol`; states at every `ckpt`-th step are kept.

Backward, for an upstream gradient lambda_T = dLoss/du_T, segment by segment from the
end: the segment's states are recomputed from its checkpoint (the kernels are
deterministic, so they equal the forward states bit for bit), then for n = end..start+1

    mu_n = A^{-T} lambda_n            transposed V-cycles to `tol` (fas_solve_transposed)
    g_kappa -= mu_n^T (dA/dkappa) u_n    (fas_kappa_grad, harmonic-mean face weights)
    lambda_{n-1} = mu_n

and the gradient with respect to u0 is lambda_0.  Every step above runs in libfas; this
module only sequences the calls and owns the tensors.
"""
import torch

from .api import Grid


def _step(grid, u, rhs, dt, kappa, kappa_cell, tol, nu1, nu2):
    rhs.copy_(u)
    st = grid.solve(rhs, u, dt, kappa, kappa_cell, tol, nu1, nu2)
    if st != 0:
        raise RuntimeError("heat step did not converge within kmax cycles")


class HeatSolveFn(torch.autograd.Function):
    """u_T = HeatSolveFn.apply(u0, kappa_cell, grid, steps, dt, ckpt, tol, nu1, nu2).

    kappa_cell: cell diffusivity (grid dtype and shape; the grid must be created with
    variable_kappa=True), or None for kappa = 1 (then only u0 gets a gradient)."""

    @staticmethod
    def forward(ctx, u0, kappa_cell, grid, steps, dt, ckpt=4, tol=1e-10, nu1=2, nu2=2):
        if steps < 1 or ckpt < 1:
            raise ValueError("steps and ckpt must be >= 1")
        u = u0.detach().clone().contiguous()
        kc = None if kappa_cell is None else kappa_cell.detach().contiguous()
        rhs = torch.empty_like(u)
        checkpoints = [u.clone()]
        for n in range(1, steps + 1):
            _step(grid, u, rhs, dt, 1.0, kc, tol, nu1, nu2)
            if n % ckpt == 0 and n < steps:
                checkpoints.append(u.clone())
        ctx.grid, ctx.steps, ctx.dt, ctx.ckpt = grid, steps, dt, ckpt
        ctx.tol, ctx.nu1, ctx.nu2 = tol, nu1, nu2
        ctx.has_kappa = kc is not None
        ctx.save_for_backward(*(([kc] if kc is not None else []) + checkpoints))
        return u

    @staticmethod
    def backward(ctx, grad_uT):
        saved = ctx.saved_tensors
        kc = saved[0] if ctx.has_kappa else None
        checkpoints = saved[1:] if ctx.has_kappa else saved
        grid, steps, dt, ckpt = ctx.grid, ctx.steps, ctx.dt, ctx.ckpt
        lam = grad_uT.detach().contiguous().clone()
        gk = torch.zeros_like(kc) if kc is not None else None
        mu = torch.empty_like(lam)
        for seg in reversed(range(len(checkpoints))):
            start = seg * ckpt
            end = min(start + ckpt, steps)
            states = recompute_segment(grid, checkpoints[seg], end - start, dt, kc, ctx.tol, ctx.nu1, ctx.nu2)
            for n in range(end, start, -1):
                mu.zero_()
                # transposed cycles: the library swaps the sweep counts and colour order
                st = grid.solve(lam, mu, dt, 1.0, kc, ctx.tol, ctx.nu1, ctx.nu2, transposed=True)
                if st != 0:
                    raise RuntimeError("adjoint solve did not converge within kmax cycles")
                if gk is not None:
                    grid.kappa_grad(dt, kc, mu, states[n - start], gk)
                lam, mu = mu, lam
        return lam, gk, None, None, None, None, None, None, None


def recompute_segment(grid, u_start, count, dt, kappa_cell, tol, nu1, nu2):
    """States u_start, u_{start+1}, ..., u_{start+count} of one checkpoint segment."""
    u = u_start.clone()
    rhs = torch.empty_like(u)
    states = [u_start]
    for _ in range(count):
        _step(grid, u, rhs, dt, 1.0, kappa_cell, tol, nu1, nu2)
        states.append(u.clone())
    return states


def heat_loss_and_grads(u0, kappa_cell, u_target, steps, dt, ckpt=4, tol=1e-10, nu1=2, nu2=2, coarsest=4, grid=None):
    """Loss ||u_T - u_target||^2 and its gradients with respect to u0 and kappa_cell."""
    if grid is None:
        n = tuple(reversed(u0.shape))
        grid = Grid(n, 1.0 / n[0], dtype=u0.dtype, coarsest=coarsest, variable_kappa=kappa_cell is not None,
                    device=u0.device)
    a = u0.detach().clone().requires_grad_(True)
    k = None if kappa_cell is None else kappa_cell.detach().clone().requires_grad_(True)
    uT = HeatSolveFn.apply(a, k, grid, steps, dt, ckpt, tol, nu1, nu2)
    loss = ((uT - u_target) ** 2).sum()
    loss.backward()
    return loss.item(), a.grad, (k.grad if k is not None else None)
