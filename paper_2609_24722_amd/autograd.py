"""Energy as a torch.autograd.Function whose backward is the force kernel and
whose double backward is the Hessian-vector-product kernel.

Positions are one (2, N) float64 tensor (row 0 = x, row 1 = y) on a GPU.

    E = CoulombEnergy.apply(xy, precision)
    g, = torch.autograd.grad(E, xy, create_graph=True)   # g = dE/dxy = -F
    Hv, = torch.autograd.grad(g, xy, v)                    # Hessian-vector product
"""
from __future__ import annotations

import torch

from . import MIXED
from . import ops


class CoulombGrad(torch.autograd.Function):
    """xy -> dE/dxy = -F (coulomb_forces); backward = H v (coulomb_hvp),
    valid because the Hessian is symmetric."""

    @staticmethod
    def forward(ctx, xy, precision=MIXED):
        fx, fy, _ = ops.forces(xy[0].contiguous(), xy[1].contiguous(), precision, with_energy=False)
        ctx.save_for_backward(xy)
        ctx.precision = precision
        return torch.stack([-fx, -fy])

    @staticmethod
    def backward(ctx, v):
        (xy,) = ctx.saved_tensors
        hx, hy = ops.hvp(xy[0].contiguous(), xy[1].contiguous(), v[0].contiguous(),
                         v[1].contiguous(), ctx.precision)
        return torch.stack([hx, hy]), None


class CoulombEnergy(torch.autograd.Function):
    """xy -> E (coulomb_energy); backward = dE/dxy through CoulombGrad."""

    @staticmethod
    def forward(ctx, xy, precision=MIXED):
        E = ops.energy(xy[0].contiguous(), xy[1].contiguous(), precision)
        ctx.save_for_backward(xy)
        ctx.precision = precision
        return E.reshape(())

    @staticmethod
    def backward(ctx, gE):
        (xy,) = ctx.saved_tensors
        g = CoulombGrad.apply(xy, ctx.precision)
        return gE * g, None


def energy(xy, precision=MIXED):
    return CoulombEnergy.apply(xy, precision)
