"""torch.autograd.Function over the forward solve and its hand-written adjoint.

The free surface is zeta(alpha) = alpha + xt(alpha) + i yt(alpha) with periodic
displacements xt, yt sampled on the M_0 surface nodes; zeta' and zeta'' are
their spectral derivatives (Sec. 2 parameterization, Sec. 3.4 symbols).  The
bottom and the obstacles are held fixed.  Forward: surface samples, then the
velocity-potential solve for U (Sec. 3).  Backward: the adjoint entry point
(one transpose GMRES solve plus the derivative of every kernel entry touching
the surface) followed by the chain rule through the spectral derivatives.
All arithmetic runs in the HIP library; torch only holds the buffers.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import wwbi


class SurfaceProblem:
    """Fixed walls and flow data; device buffers for the concatenated geometry."""

    def __init__(self, ctx: wwbi.Context, geom, device="cuda:0", **opts):
        self.ctx = ctx
        self.opts = opts
        self.M0 = geom.M[0]
        self.dg = wwbi.DeviceGeometry.from_synth(geom, device)

    @classmethod
    def from_synth(cls, ctx, geom, device="cuda:0", **opts) -> "SurfaceProblem":
        return cls(ctx, geom, device, **opts)

    def fill(self, xt: torch.Tensor, yt: torch.Tensor) -> wwbi.DeviceGeometry:
        """Write the surface samples (positions and spectral derivatives) into
        the first M_0 entries of the concatenated node arrays."""
        d = self.dg
        m = self.M0
        outs = [d.x[:m], d.y[:m], d.dx[:m], d.dy[:m], d.ddx[:m], d.ddy[:m]]
        self.ctx.surface_fill(xt.detach(), yt.detach(), outs)
        return d


class NormalVelocity(torch.autograd.Function):
    """U = NormalVelocity.apply(xt, yt, phi, problem)."""

    @staticmethod
    def forward(fctx, xt, yt, phi, problem: SurfaceProblem):
        geom = problem.fill(xt, yt)
        U, omega, _, rep = problem.ctx.solve_phi(geom, phi.detach(), **problem.opts)
        fctx.problem = problem
        fctx.save_for_backward(xt, yt, omega)
        return U

    @staticmethod
    def backward(fctx, gU):
        xt, yt, omega = fctx.saved_tensors
        problem = fctx.problem
        geom = problem.fill(xt, yt)
        grads, _ = problem.ctx.adjoint_phi(geom, omega, gU.contiguous(), **problem.opts)
        gxt, gyt = problem.ctx.surface_fill_adjoint(
            [grads["x"], grads["y"], grads["dx"], grads["dy"], grads["ddx"], grads["ddy"]])
        return gxt, gyt, grads["phi"], None


def normal_velocity(xt: torch.Tensor, yt: torch.Tensor, phi: torch.Tensor,
                    problem: SurfaceProblem) -> torch.Tensor:
    return NormalVelocity.apply(xt, yt, phi, problem)
