"""torch.autograd wrapper of K Jacobi sweeps (2D) with the hand-written adjoint.

JacobiK.apply(f, U0, solver, K, h2, chunk, keep_checkpoints) -> u_K (full
state, ring included)

  f       source over the interior (n_y, n_x), solver dtype, on the solver's device
  U0      full initial state (n_y+2, n_x+2): ring = Dirichlet values g,
          interior = u_0
  solver  a paper_2303_02543_amd.Solver for this grid (its workspace is reused)
  K       number of sweeps; h2 = h^2 (b = h2 * f)
  chunk   checkpoint interval C: the forward sweeps run as jacobi_forward_ckpt
          segments of C and the adjoint sweeps as segments of C; the
          gradients do not depend on C.
  keep_checkpoints
          keep the forward states after 0, C, 2C, ... sweeps (one device
          tensor on the context, `checkpoints`), e.g. to restart the forward
          run; off by default because the adjoint of this affine sweep reads
          no forward state.

backward(dL/du_K) is one library call, jacobi_adjoint: dL/df = h^2 * sum_k
w lam_k, and dL/dU0 with interior dL/du_0 = lam_0 and ring dL/dg -- the
gradient that flows through the sweeps plus dL/du_K on the ring itself,
because the sweeps copy the ring into u_K (corners get only the latter).
All arithmetic runs in the library (FP64 accumulation); this module only
moves tensors, and casts the FP64 gradients to the inputs' dtypes as
autograd requires.
"""
import torch


class JacobiK(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, U0, solver, K, h2, chunk=None, keep_checkpoints=False):
        K = int(K)
        chunk = int(chunk) if chunk else max(K, 1)
        solver.set_source(f.detach().contiguous(), h2)
        solver.set_state(U0.detach().contiguous())
        ctx.checkpoints = solver.forward_ckpt(K, chunk, keep=bool(keep_checkpoints))
        uK = solver.get_state()
        ctx.solver = solver
        ctx.K = K
        ctx.h2 = float(h2)
        ctx.chunk = chunk
        ctx.f_dtype = f.dtype
        ctx.u_dtype = U0.dtype
        return uK

    @staticmethod
    def backward(ctx, grad_uK):
        s = ctx.solver
        lam = grad_uK.detach().to(s.torch_dtype).contiguous()
        gf, gU0 = s.adjoint(lam, ctx.K, ctx.h2, chunk=ctx.chunk)
        return gf.to(ctx.f_dtype), gU0.to(ctx.u_dtype), None, None, None, None, None


def jacobi_k(f, U0, solver, K, h2, chunk=None, keep_checkpoints=False):
    """Differentiable u_K = Jacobi^K(U0; b = h2 f)."""
    return JacobiK.apply(f, U0, solver, K, h2, chunk, keep_checkpoints)
