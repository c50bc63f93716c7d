"""torch.autograd wrapper of K Jacobi sweeps (2D) with the hand-written adjoint.

JacobiK.apply(f, U0, solver, K, h2, chunk) -> u_K (full state, ring included)

  f       source over the interior (n_y, n_x), solver dtype, on the solver's device
  U0      full initial state (n_y+2, n_x+2): ring = Dirichlet values g,
          interior = u_0
  solver  a paper_2303_02543_amd.Solver for this grid (its workspace is reused)
  K       number of sweeps; h2 = h^2 (b = h2 * f)
  chunk   checkpoint interval C: the forward pass records the state every C
          sweeps (kept on the context as `checkpoints`, for inspection or to
          resume) and the backward pass runs its adjoint sweeps in segments of
          C; the gradients do not depend on C.

backward(dL/du_K) returns dL/df = h^2 * sum_k w lam_k and dL/dU0 whose ring
entries are dL/dg and whose interior is dL/du_0 (corners 0), computed by the
library's adjoint passes (FP64 accumulation).  No PyTorch arithmetic touches the
sweep: torch only provides the tensors.
"""
import torch


class JacobiK(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, U0, solver, K, h2, chunk=None):
        K = int(K)
        chunk = int(chunk) if chunk else K
        solver.set_source(f.detach().contiguous(), h2)
        solver.set_state(U0.detach().contiguous())
        checkpoints = [U0.detach().clone()]
        left = K
        while left > 0:
            step = min(chunk, left)
            solver.sweep(step)
            left -= step
            if left > 0:
                checkpoints.append(solver.get_state())
        uK = solver.get_state()
        ctx.solver = solver
        ctx.K = K
        ctx.h2 = float(h2)
        ctx.chunk = chunk
        ctx.checkpoints = checkpoints
        ctx.f_dtype = f.dtype
        ctx.u_dtype = U0.dtype
        return uK

    @staticmethod
    def backward(ctx, grad_uK):
        s = ctx.solver
        lam = grad_uK.detach().to(s.torch_dtype).contiguous()
        gb, gU0 = s.adjoint(lam, ctx.K, ctx.h2, chunk=ctx.chunk)
        # s.adjoint returns h2-scaled dL/df in place of dL/db
        grad_f = gb.to(ctx.f_dtype)
        grad_U0 = gU0.to(ctx.u_dtype)
        return grad_f, grad_U0, None, None, None, None


def jacobi_k(f, U0, solver, K, h2, chunk=None):
    """Differentiable u_K = Jacobi^K(U0; b = h2 f)."""
    return JacobiK.apply(f, U0, solver, K, h2, chunk)
