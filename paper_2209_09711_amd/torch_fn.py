"""PyTorch autograd wrapper: R(p) with dR/dp from the same enumeration sweep.

PyTorch supplies device memory and the stream only.  The forward pass calls
``bat_reliability_grad_async`` on the current stream: one launch of the HIP
sweep produces R, the feasible count and T1_i - T0_i for every arc (Eq. 1 is
multilinear in p, so these are exactly dR/dp_i).  The backward pass scales
the saved gradient by the incoming gradient; it launches no second sweep.
"""
from __future__ import annotations

import numpy as np
import torch

from . import bat_reliability_grad_async


class BatReliability(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p: torch.Tensor, n_nodes: int, arcs, s: int, t: int):
        if p.dtype != torch.float64 or not p.is_cuda:
            raise TypeError("p must be a float64 tensor on the GPU")
        p = p.contiguous()
        m = p.shape[0]
        arcs = np.ascontiguousarray(np.asarray(arcs, dtype=np.int32).reshape(-1, 2))
        if arcs.shape[0] != m:
            raise ValueError("p and arcs disagree in length")
        dev = p.device
        R = torch.empty((), dtype=torch.float64, device=dev)
        cnt = torch.empty((), dtype=torch.int64, device=dev)
        g = torch.empty(max(m, 1), dtype=torch.float64, device=dev)
        status = torch.empty((), dtype=torch.int32, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        bat_reliability_grad_async(n_nodes, arcs, p.data_ptr(), s, t, R.data_ptr(), cnt.data_ptr(),
                                   g.data_ptr(), None, None, status.data_ptr(), stream)
        ctx.save_for_backward(g[:m])
        ctx.mark_non_differentiable(cnt)
        return R, cnt

    @staticmethod
    def backward(ctx, grad_R, grad_cnt):
        (g,) = ctx.saved_tensors
        return grad_R * g, None, None, None, None


def reliability(p: torch.Tensor, n_nodes: int, arcs, s: int, t: int):
    """Differentiable exact reliability: returns (R, count) tensors."""
    return BatReliability.apply(p, n_nodes, arcs, s, t)
