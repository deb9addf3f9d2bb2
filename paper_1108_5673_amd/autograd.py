"""torch.autograd.Function over pwa_nll_grad: the forward call returns the NLL
and keeps the analytic gradient computed in the same pass over the events, so
backward costs no further evaluation."""
from __future__ import annotations

import numpy as np
import torch


class NLLFunction(torch.autograd.Function):
    """NLL(v) for v = [Re V_0, Im V_0, ...] (float64, 2W), gradient from the library.

    Usage: ``loss = NLLFunction.apply(v, model)``.
    """

    @staticmethod
    def forward(ctx, v, model):
        nll, g = model.nll_grad(v.detach().cpu().numpy())
        ctx.save_for_backward(torch.from_numpy(np.asarray(g)).to(device=v.device, dtype=v.dtype))
        return torch.tensor(nll, dtype=v.dtype, device=v.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None
