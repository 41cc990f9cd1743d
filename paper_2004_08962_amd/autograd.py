"""The HICU objective as a differentiable torch function.

J(x) = ||H_S(x) F||_F^2 (THEORY section, Eq. 2 for a fixed filter bank F)
with a hand-written backward: the gradient 2 H_S'(H_S(x) F F^H), i.e. the
adjoint convolution, computed by the library's kernels.  Nothing from the
forward pass is kept except x and F: the backward recomputes the residual
Y = H_S(x) F tile by tile before the adjoint, so no patch matrix is ever
stored.

PyTorch's convention for a real loss of complex inputs is
grad = 2 dL/d(conj x), which is exactly the library's gradient g, so the
backward returns grad_J * g.  With a sampling mask the gradient is projected
(zero at observed locations, the hard data matching of the method);
without one it is the plain derivative.  F receives no gradient.
"""
import torch

from . import api


class HicuObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, F, kdims, lo=None, hi=None, mask=None, prec="fp32"):
        if F.requires_grad:
            raise NotImplementedError("HicuObjective differentiates with respect to x only")
        api._shape_checks(x.shape, kdims, F, mask)
        J, _, _ = api.objective_grad(x.detach(), None, F.detach(), kdims, lo, hi, prec=prec, want_grad=False)
        ctx.save_for_backward(x.detach(), F.detach())
        ctx.args = (tuple(kdims), lo, hi, mask, prec)
        return J

    @staticmethod
    def backward(ctx, grad_J):
        x, F = ctx.saved_tensors
        kdims, lo, hi, mask, prec = ctx.args
        _, g, _ = api.objective_grad(x, mask, F, kdims, lo, hi, prec=prec, want_grad=True)
        gx = g * grad_J.to(torch.float32)
        return gx, None, None, None, None, None, None


def hicu_objective(x, F, kdims, lo=None, hi=None, mask=None, prec="fp32"):
    """J = ||H_S(x) F||_F^2 (0-dim float64 CUDA tensor), differentiable in x."""
    return HicuObjective.apply(x, F, kdims, lo, hi, mask, prec)
