"""torch.autograd.Function over flood_adjoint.

``FloodAdjointFn.apply(n_field, rain_mult, ens, spec)`` returns the gauge-misfit
loss of one catchment's ensemble run from its current state, and its backward
returns the gradients with respect to the shared Manning field and the
per-member rain multipliers.  The forward pass calls ``flood_adjoint`` once
(it computes the loss and both gradients); the ensemble's state is restored
afterwards from a device snapshot held by the handle, so the function can be
evaluated repeatedly without any host transfer of the state.  Torch only
carries the tensors; all arithmetic runs in libflood.
"""
from __future__ import annotations

import numpy as np
import torch

from .flood import FloodEnsemble, flood_set_params


class FloodAdjointFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n_field: torch.Tensor, rain_mult: torch.Tensor, ens: FloodEnsemble, spec: dict):
        c = spec.get("catchment", 0)
        n_np = n_field.detach().cpu().numpy().astype(np.float32)
        mu_np = rain_mult.detach().cpu().numpy().astype(np.float64)
        flood_set_params(ens.h, c, manning=n_np, rain_mult=mu_np)
        ens.snapshot()
        try:
            loss, gn, gm = ens.adjoint(c, spec["t_end"], spec["sample_dt"], spec["gauges"], spec["obs"],
                                       spec.get("ckpt_every", 100))
        finally:
            ens.restore()
        ctx.save_for_backward(torch.as_tensor(gn, dtype=n_field.dtype, device=n_field.device),
                              torch.as_tensor(gm, dtype=rain_mult.dtype, device=rain_mult.device))
        return torch.tensor(loss, dtype=torch.float64, device=n_field.device)

    @staticmethod
    def backward(ctx, grad_out):
        gn, gm = ctx.saved_tensors
        g = grad_out.to(gn.dtype)
        return g * gn, g * gm, None, None
