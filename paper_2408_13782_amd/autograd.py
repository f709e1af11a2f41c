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

import numpy as np
import torch

from . import fpm

MAX_GROUP = 64   # LEDs per fpm_loss_grad call


@dataclass
class LossContext:
    plan: fpm.Plan
    grid: fpm.LedGrid
    leds: object          # host int32 LED ids of the batch
    meas_amp: torch.Tensor


class FPMLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, O, coeffs, z_um, geom, gamma, lctx: LossContext):
        plan = lctx.plan
        # the scalar accumulators in one buffer: loss | g_par (16) | g_geom (4) | g_gamma
        n = plan.n_led
        flat = torch.zeros(1 + fpm.N_PAR + 4 + n, dtype=torch.float64, device=O.device)
        grads = {"loss": flat[:1], "g_par": flat[1:1 + fpm.N_PAR],
                 "g_geom": flat[1 + fpm.N_PAR:5 + fpm.N_PAR], "g_gamma": flat[5 + fpm.N_PAR:],
                 "g_O": torch.zeros_like(O, memory_format=torch.contiguous_format),
                 "oob": torch.zeros(1, dtype=torch.int32, device=O.device)}
        # fpm_loss_grad takes up to 64 LEDs and adds into the accumulators: a
        # larger batch (up to the full gradient of Eq. 6) is summed in groups
        leds = np.ascontiguousarray(np.asarray(lctx.leds, np.int32).reshape(-1))
        for b0 in range(0, max(leds.size, 1), MAX_GROUP):
            g = plan.loss_grad(lctx.grid, O.detach(), leds[b0:b0 + MAX_GROUP], lctx.meas_amp,
                               coeffs=None if coeffs is None else coeffs.detach(),
                               z_um=None if z_um is None else z_um.detach(),
                               geom=None if geom is None else geom.detach(),
                               gamma=None if gamma is None else gamma.detach(), grads=grads)
        fctx.flat, fctx.g_O = flat, g["g_O"]
        fctx.dtypes = tuple(None if t is None else t.dtype for t in (coeffs, z_um, geom, gamma))
        fctx.oob = g["oob"]
        return flat[0].clone()

    @staticmethod
    def backward(fctx, grad_out):
        c_t, z_t, g_t, gm_t = fctx.dtypes
        go = grad_out.to(torch.float64)
        flat = fctx.flat * go                    # every scalar group in one kernel
        par = flat[1:1 + fpm.N_PAR]
        out = [fctx.g_O * go.to(torch.float32),
               None if c_t is None else par[:fpm.N_ZERN].to(c_t),
               None if z_t is None else par[fpm.N_ZERN:].to(z_t),
               None if g_t is None else flat[1 + fpm.N_PAR:5 + fpm.N_PAR].to(g_t),
               None if gm_t is None else flat[5 + fpm.N_PAR:].to(gm_t)]
        return (*out, None)
