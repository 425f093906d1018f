"""Differentiable NFFT: torch.autograd functions over the library's transforms.

For a real loss L and PyTorch's complex-gradient convention (the gradient of
z is 2 dL/d conj(z)):

* forward  fhat = A(x) f:  grad_f = A^H g,
  grad_x[j, d] = Re(conj(g_j) dA_d f_j),  dA_d f_j = sum_n (-2 pi i n_d) f_n e^{-2 pi i n.x_j};
* adjoint  y = A(x)^H fhat:  grad_fhat = A g,
  grad_x[j, d] = Re(conj(fhat_j) dA_d g_j);

with g the incoming gradient.  dA_d f is the library's nfft_forward_deriv: with
the polynomial window (D <= 3) the derivative of the NFFT itself -- the
oversampled spectrum interpolated with the derivative of the window along axis
d, so the gradients are exact for the function the forward pass computes;
otherwise the forward NFFT of the coefficients -2 pi i n_d f_n (the derivative
of the NDFT, subsection "NDFT" of "Mathematical Description", evaluated with the
NFFT approximation).  Both agree with the NDFT's derivative to about the
transform's accuracy.

The nodes are fixed when a plan is built; the functions here take the plan
and the node tensor it was built from (the tensor carries the gradient).
"""
import torch

from .nfft import Plan


class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, x, plan):
        ctx.plan = plan
        ctx.save_for_backward(f)
        return plan.forward(f.contiguous())

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        (f,) = ctx.saved_tensors
        g = g.contiguous()
        grad_f = plan.adjoint(g) if ctx.needs_input_grad[0] else None
        grad_x = None
        if ctx.needs_input_grad[1]:
            grad_x = plan.node_grad(g, plan.forward_deriv(f.contiguous()))
        return grad_f, grad_x, None


class _Adjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fhat, x, plan):
        ctx.plan = plan
        ctx.save_for_backward(fhat)
        return plan.adjoint(fhat.contiguous())

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        (fhat,) = ctx.saved_tensors
        g = g.contiguous()
        grad_fhat = plan.forward(g) if ctx.needs_input_grad[0] else None
        grad_x = None
        if ctx.needs_input_grad[1]:
            grad_x = plan.node_grad(fhat.contiguous(), plan.forward_deriv(g))
        return grad_fhat, grad_x, None


def nfft(x, f, plan=None, m=4, sigma=2.0):
    """Differentiable forward NFFT (with respect to f and the nodes x).  ``plan`` must have
    been built from the current values of x; without one, a plan is built here."""
    if plan is None:
        plan = Plan(x.detach(), tuple(f.shape), m=m, sigma=sigma)
    return _Forward.apply(f, x, plan)


def nfft_adjoint(x, N, fhat, plan=None, m=4, sigma=2.0):
    """Differentiable adjoint NFFT (with respect to fhat and the nodes x); the argument order
    is that of the package's nfft_adjoint."""
    if plan is None:
        plan = Plan(x.detach(), tuple(N), m=m, sigma=sigma)
    return _Adjoint.apply(fhat, x, plan)
