"""torch.autograd.Function over the hand-written adjoint (paper Sec. 2.2).

FPMLoss.apply(O, coeffs, z_um, geom, gamma, ctx) returns the batch loss as a
float64 scalar tensor; its backward returns the gradients libfpm computed in
the same call (fpm_loss_grad), scaled by the incoming gradient. Complex
gradients follow torch's convention for a real loss, dL/dRe + i dL/dIm.

    ctx = LossContext(plan, grid, leds, meas_amp)
    loss = FPMLoss.apply(O, coeffs, z_um, geom, gamma, ctx)
    loss.backward()   # fills O.grad, coeffs.grad, z_um.grad, geom.grad, gamma.grad
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import fpm


@dataclass
class LossContext:
    plan: fpm.Plan
    grid: fpm.LedGrid
    leds: object          # host int32 LED ids of the batch
    meas_amp: torch.Tensor


class FPMLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, O, coeffs, z_um, geom, gamma, lctx: LossContext):
        g = lctx.plan.loss_grad(lctx.grid, O.detach(), lctx.leds, lctx.meas_amp,
                                coeffs=None if coeffs is None else coeffs.detach(),
                                z_um=None if z_um is None else z_um.detach(),
                                geom=None if geom is None else geom.detach(),
                                gamma=None if gamma is None else gamma.detach())
        fctx.grads = (g["g_O"],
                      None if coeffs is None else g["g_par"][:fpm.N_ZERN].to(coeffs.dtype),
                      None if z_um is None else g["g_par"][fpm.N_ZERN:].to(z_um.dtype),
                      None if geom is None else g["g_geom"].to(geom.dtype),
                      None if gamma is None else g["g_gamma"].to(gamma.dtype))
        fctx.oob = g["oob"]
        return g["loss"][0]

    @staticmethod
    def backward(fctx, grad_out):
        out = []
        for gr in fctx.grads:
            out.append(None if gr is None else gr * grad_out.to(gr.real.dtype))
        return (*out, None)
