"""torch.autograd wrapper of the collision integral.

Forward and backward both run in the HIP library (sb2_collision and
sb2_collision_backward); this module only routes tensors.  Gradients follow
torch's complex convention (dL/dRe z + i dL/dIm z); v is treated as an
unconstrained real tensor and h as an unconstrained complex matrix.  The
adjoint is float64 whatever precision the forward used.
"""
from __future__ import annotations

import torch

from . import _lib


class Sb2Collision(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, h, rho_hist, dt, prec):
        ctx.save_for_backward(v, h, rho_hist)
        ctx.dt = float(dt)
        return _lib.sb2_collision(v.contiguous(), h.contiguous(), rho_hist.contiguous(), dt, prec)

    @staticmethod
    def backward(ctx, grad_i):
        v, h, rho = ctx.saved_tensors
        gv, gh, gr = _lib.sb2_collision_backward(v.contiguous(), h.contiguous(), rho.contiguous(), ctx.dt,
                                                 grad_i.contiguous(), "fp64")
        return gv, gh, gr, None, None


def collision(v, h, rho_hist, dt, prec="fp64"):
    """Differentiable I_ns(t) (N, N) complex128."""
    return Sb2Collision.apply(v, h, rho_hist, dt, prec)


def correlation_observable(v, h, rho_hist, dt, prec="fp64"):
    """The scalar L = Im tr[h I_ns] (differentiable in v, h and rho_hist)."""
    i_ns = collision(v, h, rho_hist, dt, prec)
    return torch.diagonal(h @ i_ns).sum().imag
