"""Differentiable prediction: model image -> visibilities, with the gridding
adjoint as its hand-written backward.

Section 6 notes that the separable approximation serves prediction as well as
imaging, which Cotton-Schwab major cycles need.  For a real model image x the
forward operator is the prediction equation (Section 2) on the pixel grid,
    A x = degrid( F-[ x / (n c1 c1) ] )          (sepw_degrid, SEPW_DIV_N)
and, because 1/(n c1 c1) is real and diagonal, its adjoint is
    A^H r = F+[ grid(r) ] / (n c1 c1)             (sepw_grid, SEPW_DIV_N, weights 1).
For a real loss L of complex V = A x, PyTorch hands backward the gradient
g = dL/dV* (e.g. 2 W (V - Vt) for L = sum W |V - Vt|^2), and
dL/dx = Re(A^H g).  Both directions run in the library's kernels.
"""
import torch

from . import _lib


class Predict(torch.autograd.Function):
    """V = Predict.apply(x, plan): x real (N, N) float32 on the GPU."""

    @staticmethod
    def forward(ctx, x, plan):
        if x.dtype != torch.float32 or x.dim() != 2:
            raise TypeError("x must be a real float32 (N, N) tensor")
        ctx.plan = plan
        # the real model goes in as it is (no complex copy)
        return _lib.degrid(plan, x.contiguous(), flags=_lib.DIV_N | _lib.REAL)

    @staticmethod
    def backward(ctx, grad_v):
        plan = ctx.plan
        g = grad_v.contiguous()
        if g.dtype != torch.complex64:
            g = g.to(torch.complex64)
        # only the real part of the adjoint image is the gradient
        return _lib.grid(plan, g, None, flags=_lib.DIV_N | _lib.REAL), None


def predict(x, plan):
    return Predict.apply(x, plan)


def chi2(V, Vt, W):
    """sum_i W_i |V_i - Vt_i|^2, reduced in float64."""
    r = (V - Vt).to(torch.complex128)
    return torch.sum(W.to(torch.float64) * (r.real ** 2 + r.imag ** 2))
