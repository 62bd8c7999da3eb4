"""torch.autograd binding of the split-CTMRG free energy.

``free_energy(A, beta, chi, ...)`` returns f(beta, A) (Eq. free energy
expression) as a 0-dim tensor that is differentiable in A.  The forward pass
converges the environments of both networks inside the HIP library and keeps
them resident on the device (the checkpoint); the backward pass is the
hand-written adjoint of the converged environment, Eq. (gradient
expression): it recomputes the half-patch contractions around the bra tensor
from the stored environments (``ctm_grad``) instead of differentiating
through the iteration, and returns g = df/dA, projected onto the D4 subspace.

All arithmetic runs in the library; this module only moves tensors.  A may be
float32 or float64 on the GPU (the library works in float64; the gradient is
returned in A's dtype).
"""
import torch

from . import ctm


class SplitCTMFreeEnergy(torch.autograd.Function):
    """f(beta, A); backward: the converged-environment adjoint of the library."""

    @staticmethod
    def forward(ctx, A, beta, chi, max_iter, tol, precision, refine, context):
        A64 = A.detach().to(torch.float64).contiguous()
        stream = torch.cuda.current_stream(A.device).cuda_stream if A.is_cuda else None
        if context is not None:
            # warm restart: the environments of the previous point are the start
            c = context
            c.reset_tensor(beta, A64)
        else:
            c = ctm.SplitCTM(beta, A64, chi, max_iter=max_iter, tol=tol, precision=precision,
                             refine=refine, stream=stream)
        done, delta, conv = c.iterate(0)
        f, _, _ = c.free_energy()
        ctx.ctm = c
        ctx.owned = context is None
        ctx.a_dtype = A.dtype
        ctx.info = dict(iters=done, delta=delta, converged=conv)
        return torch.tensor(f, dtype=A.dtype, device=A.device)

    @staticmethod
    def backward(ctx, grad_f):
        c = ctx.ctm
        if grad_f.is_cuda:
            g = torch.empty((2,) + (c.D,) * 4, dtype=torch.float64, device=grad_f.device)
            c.grad(g)
        else:
            g = torch.from_numpy(c.grad())
        if ctx.owned:
            c.close()
        ctx.ctm = None
        return (grad_f * g).to(ctx.a_dtype), None, None, None, None, None, None, None


def free_energy(A, beta, chi, max_iter=200, tol=1e-9, precision=ctm.CTM_FP64, refine=False,
                context=None):
    """f(beta, A) with autograd support (see the module docstring).

    ``context``: an existing ``ctm.SplitCTM`` of the same D and chi to warm-start
    from (its environments are reused and updated); otherwise a context is
    created for this call and released after the backward pass."""
    return SplitCTMFreeEnergy.apply(A, float(beta), int(chi), int(max_iter), float(tol),
                                    int(precision), bool(refine), context)
