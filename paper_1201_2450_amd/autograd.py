"""Differentiable TNLM energy: torch.autograd.Function over the C ABI.

Forward: tnlm_energy with u = f, keeping only the O(N) per-voxel statistics
(log-normaliser and e for each voxel and direction), never the O(W N) weight
tensor. Backward: tnlm_grad(EXACT) rebuilds the weights from those
statistics and returns dE/df + dE/du, the gradient of E(f; f) through both
the image terms and the weights (Eqs. (2)-(3) with the weights of Eq. (9)
taken from f itself).
"""
from __future__ import annotations

import torch

from . import ops


class TNLMEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, d, M, h):
        e, stats = ops.energy(f, d=d, M=M, h=h, want_stats=True)
        ctx.save_for_backward(f, stats)
        ctx.geo = (d, M, h)
        return (e[0] + e[1]).reshape(())

    @staticmethod
    def backward(ctx, gE):
        f, stats = ctx.saved_tensors
        d, M, h = ctx.geo
        g = ops.grad(f, d=d, M=M, h=h, mode="exact", stats=stats, total=True)
        gf = (g * gE).to(f.dtype)
        return gf, None, None, None


def tnlm_energy(f, d, M, h):
    """E(f; f) as a differentiable 0-dim float32 tensor."""
    return TNLMEnergy.apply(f, d, M, h)
