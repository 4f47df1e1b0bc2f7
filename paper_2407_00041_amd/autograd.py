"""torch.autograd.Function for y = D(U) x.

backward returns dL/dx = D^H g (the adjoint apply: Eq. (1.13) with the
projectors swapped) and, when the links require a gradient,
dL/dU = G = dL/dRe U + i dL/dIm U from the library's force kernel, i.e. the
derivative of Re<g, D(U) x> (torch's convention for complex tensors).
"""
from __future__ import annotations

import torch

from . import DiracOp


class DiracApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, links, op, dims, m0, csw, antiperiodic_t):
        """x: [nrhs, V, 12] complex128 (canonical, on the GPU); links: [V, 4, 3, 3]."""
        if op is None:
            op = DiracOp(dims, links, m0, csw, antiperiodic_t=antiperiodic_t, precisions=("f64",))
        ctx.op = op
        ctx.save_for_backward(x)
        return op.apply(x, "f64")

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        op = ctx.op
        gx = gU = None
        g = g.contiguous()
        nrhs = x.numel() // (12 * op.V)
        if ctx.needs_input_grad[0]:
            gx = op.apply(g, "f64", dagger=True)
        if ctx.needs_input_grad[1]:
            gn = op.pack(g.reshape(nrhs, op.V, 12), "f64")
            xn = op.pack(x.reshape(nrhs, op.V, 12), "f64")
            gU = op.force(gn, xn, nrhs, raw=True)
        return gx, gU, None, None, None, None, None


def dirac_apply(x, links, dims, op: DiracOp | None = None, m0: float = 0.0, csw: float = 0.0,
                antiperiodic_t: bool = False):
    """Differentiable y = D(U) x.

    Pass a prebuilt ``op`` (created from these ``links``) for speed; without one
    the operator is rebuilt from ``links`` on every call (needed when the links
    themselves are perturbed, e.g. by finite-difference checks).
    """
    return DiracApply.apply(x, links, op, tuple(dims), m0, csw, antiperiodic_t)
