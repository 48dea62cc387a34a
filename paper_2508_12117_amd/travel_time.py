"""TravelTime: torch.autograd.Function over the HIP travel-time kernel.

forward(x_src, s) -> T runs the network forward and the hand-written
reverse-mode source gradient in one kernel (Sec. 3.2: gradients by
reverse-mode differentiation; activations recomputed on chip, never stored)
and keeps dT/dx for backward, which returns grad_T * dT/dx for x_src and
nothing for the receiver.  No torch autograd graph is built for the network.
"""
from __future__ import annotations

import torch

from . import spider


class TravelTime(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x_src, s, sctx, net_id, precision):
        x_src = x_src.detach().to(torch.float64).contiguous()
        s = s.detach().to(torch.float64).contiguous()
        rows = x_src.shape[0]
        T = torch.empty(rows, dtype=torch.float64, device=x_src.device)
        g = torch.empty(rows, 3, dtype=torch.float64, device=x_src.device)
        sctx.travel_time(net_id, x_src, s, T, g, precision=precision)
        ctx.save_for_backward(g)
        return T

    @staticmethod
    def backward(ctx, grad_T):
        (g,) = ctx.saved_tensors
        return grad_T[:, None] * g, None, None, None, None


def travel_time(x_src, s, sctx: "spider.Context", net_id: int, precision=spider.FP32):
    return TravelTime.apply(x_src, s, sctx, net_id, precision)
