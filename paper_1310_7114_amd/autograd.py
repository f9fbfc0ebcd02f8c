"""Cauchy-Schwarz divergence of lattice ITC as a differentiable torch op.

D(h, W) = log S_W + log S_X - 2 log S_XW (eq. (1) in the single-width reading)
for per-pixel weights h (Section 5) and codebooks W. Forward and backward run
in the HIP kernels (batched precompute + divergence, and the adjoint kernels);
PyTorch only supplies memory, the stream and the autograd graph.
"""
from __future__ import annotations

import torch

from . import itc

_PLANS = {}


def _plan(B, H, W, M, sigma, radius, device):
    key = (B, H, W, M, float(sigma), int(radius), str(device))
    p = _PLANS.get(key)
    if p is None:
        p = itc.BatchPlan.for_stack(B, H, W, M, sigma, iters=0, dtype=torch.float32, radius=radius, device=device)
        _PLANS[key] = p
    return p


class ITCDivergence(torch.autograd.Function):
    """D for weights (B, H, W) or (H, W) float32 and codebooks (B, M, 2) or (M, 2) float32."""

    @staticmethod
    def forward(ctx, weights: torch.Tensor, w: torch.Tensor, sigma: float, radius: int = 0):
        single = weights.dim() == 2
        h = (weights.unsqueeze(0) if single else weights).to(torch.float32).contiguous()
        cb = (w.unsqueeze(0) if single else w).to(torch.float32).contiguous()
        B, H, W = h.shape
        M = cb.shape[1]
        plan = _plan(B, H, W, M, sigma, radius, h.device)
        maps = plan.new_maps()
        w0 = cb.reshape(B * M, 2)
        w_out = torch.empty_like(w0)
        s_x = torch.empty(B, dtype=torch.float64, device=h.device)
        d = torch.empty(B, dtype=torch.float64, device=h.device)
        plan.precompute(weights=h, maps=maps)
        plan.fit(w0, w_out, s_x=s_x, d_out=d, maps=maps)
        ctx.plan, ctx.maps, ctx.single = plan, maps, single
        ctx.save_for_backward(w0, s_x)
        ctx.shape = (B, H, W, M)
        return d[0] if single else d

    @staticmethod
    def backward(ctx, grad_d: torch.Tensor):
        w0, s_x = ctx.saved_tensors
        B, H, W, M = ctx.shape
        gd = grad_d.reshape(B).to(torch.float64).contiguous()
        need_h, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gw = torch.empty_like(w0) if need_w else None
        gh = torch.empty((B, H, W), dtype=torch.float32, device=w0.device) if need_h else None
        ctx.plan.backward(w0, s_x, gd, grad_w=gw, grad_weights=gh, maps=ctx.maps)
        if gw is not None:
            gw = gw.view(B, M, 2)
            if ctx.single:
                gw = gw[0]
        if gh is not None and ctx.single:
            gh = gh[0]
        return gh, gw, None, None


def divergence(weights: torch.Tensor, w: torch.Tensor, sigma: float, radius: int = 0) -> torch.Tensor:
    """Differentiable D (see ITCDivergence)."""
    return ITCDivergence.apply(weights, w, sigma, radius)
