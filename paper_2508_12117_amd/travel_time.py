"""TravelTime: torch.autograd.Function over the HIP travel-time calls.

forward(x_src, s) -> T calls spider_tt_forward; backward(grad_T) calls
spider_tt_backward, which evaluates the network again at the saved points
and returns the vector-Jacobian product grad_T * dT/dx for the source
(reverse-mode differentiation, Sec. 3.2), and nothing for the receiver.  No
torch autograd graph is built for the network and every arithmetic step,
including the product with grad_T, runs in the library; this wrapper only
allocates the outputs and passes pointers.
"""
from __future__ import annotations

import torch

from . import spider


class TravelTime(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x_src, s, sctx, net_id, precision):
        x_src = x_src.detach().to(torch.float64).contiguous()
        s = s.detach().to(torch.float64).contiguous()
        T = torch.empty(x_src.shape[0], dtype=torch.float64, device=x_src.device)
        sctx.tt_forward(net_id, x_src, s, T, precision=precision)
        ctx.save_for_backward(x_src, s)
        ctx.sctx, ctx.net_id, ctx.precision = sctx, net_id, precision
        return T

    @staticmethod
    def backward(ctx, grad_T):
        x_src, s = ctx.saved_tensors
        grad_T = grad_T.detach().to(torch.float64).contiguous()
        grad_x = torch.empty_like(x_src)
        ctx.sctx.tt_backward(ctx.net_id, x_src, s, grad_T, grad_x, precision=ctx.precision)
        return grad_x, None, None, None, None


def travel_time(x_src, s, sctx: "spider.Context", net_id: int, precision=spider.FP32):
    return TravelTime.apply(x_src, s, sctx, net_id, precision)
