"""torch.autograd wrapper of the time stepper, with adjoint-solve backward.

rollout(solver, u0, V, steps) returns u^steps of the starter followed by
steps - 1 three-level steps (Sec. 2.1, 2.2; the starter is the dt/2 system)
on `solver`'s operator, with D = rho dt |u^n|^2 + dt V.  Its backward runs the
reverse mode of every step through the C ABI (fnls_step_backward,
fnls_first_step_backward): one adjoint GMRES solve per step, A being complex
symmetric so that A^H = conj(A).  Gradients follow PyTorch's convention for
complex tensors (dL/dRe z + i dL/dIm z).

Checkpointing: the forward keeps the level pair (u^{k-1}, u^k) every
`checkpoint` steps; the backward recomputes the levels of one segment at a
time from its checkpoint, so memory is O(checkpoint) vectors instead of
O(steps).  All arithmetic runs in the library's kernels; this module only
orders the calls and holds the tensors.
"""
from __future__ import annotations

import torch

from .fnls import Solver


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, V, solver, steps, checkpoint, tol):
        if steps < 1:
            raise ValueError("steps must be >= 1")
        if checkpoint < 1:
            raise ValueError("checkpoint must be >= 1")
        solver.set_potential(V)
        u_prev = u0.detach().contiguous()
        u_cur, _ = solver.first_step(u_prev, tol=tol)
        ckpt = {1: (u_prev, u_cur)}         # k -> (u^{k-1}, u^k)
        for k in range(1, steps):
            un, _ = solver.step(u_prev, u_cur, tol=tol)
            u_prev, u_cur = u_cur, un
            if (k + 1) % checkpoint == 0 and k + 1 < steps:
                ckpt[k + 1] = (u_prev, u_cur)
        ctx.solver, ctx.steps, ctx.tol, ctx.ckpt, ctx.V = solver, steps, tol, ckpt, V
        return u_cur.clone()

    @staticmethod
    def backward(ctx, g_out):
        solver, N, tol, ckpt, V = ctx.solver, ctx.steps, ctx.tol, ctx.ckpt, ctx.V
        solver.set_potential(V)
        g = {N: g_out.detach().to(torch.complex128).contiguous().clone()}
        gV = torch.zeros_like(V) if (V is not None and ctx.needs_input_grad[1]) else None

        def grad(k):
            if k not in g:
                g[k] = torch.zeros_like(g_out, dtype=torch.complex128)
            return g[k]

        starts = sorted(ckpt)
        ends = starts[1:] + [N]
        for k0, k1 in reversed(list(zip(starts, ends))):
            # levels u^{k0-1} .. u^{k1} of this segment
            lev = {k0 - 1: ckpt[k0][0], k0: ckpt[k0][1]}
            for k in range(k0, k1):
                if k + 1 not in lev:
                    lev[k + 1], _ = solver.step(lev[k - 1], lev[k], tol=tol)
            for k in range(k1 - 1, k0 - 1, -1):
                if k == 0:
                    continue
                # step k: (u^{k-1}, u^k) -> u^{k+1}
                solver.step_backward(lev[k - 1], lev[k], lev[k + 1], g[k + 1], grad(k - 1), grad(k), gV,
                                     tol=tol)
                del g[k + 1]
        # starter u^0 -> u^1
        u0, u1 = ckpt[1]
        solver.first_step_backward(u0, u1, g[1], grad(0), gV, tol=tol)
        return g[0], gV, None, None, None, None


def rollout(solver: Solver, u0: torch.Tensor, V: torch.Tensor | None = None, steps: int = 20,
            checkpoint: int = 5, tol: float = 1e-10) -> torch.Tensor:
    """u^steps from u^0 (and the potential V), differentiable in u0 and V."""
    return _Rollout.apply(u0, V, solver, steps, checkpoint, tol)
