"""Differentiable smoothed clearance score as a torch.autograd.Function.

Forward and adjoint both run in libaf.so (af_smooth_eval); this module only
allocates the outputs and hands the pointers over.  s(p, q) sums, over the
tool's samples o, log sigma((T(p + R(q) o) - c) / tau_s) with the map's TSDF
T read trilinearly; gradients flow to the points p [n, 3] and the
quaternions q [n, 4]."""
from __future__ import annotations

import torch


class SmoothScore(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p, q, af_ctx, samples, c, tau_s):
        p, q = p.contiguous(), q.contiguous()
        s = torch.empty(p.shape[0], device=p.device, dtype=torch.float32)
        af_ctx.smooth_eval(p, q, samples, c, tau_s, s=s)
        ctx.save_for_backward(p, q, samples)
        ctx.af_ctx, ctx.c, ctx.tau_s = af_ctx, c, tau_s
        return s

    @staticmethod
    def backward(ctx, grad_s):
        p, q, samples = ctx.saved_tensors
        dq = torch.empty_like(q)
        dp = torch.empty_like(p)
        ctx.af_ctx.smooth_eval(p, q, samples, ctx.c, ctx.tau_s,
                               grad_s=grad_s.contiguous().to(torch.float32), dq=dq, dp=dp)
        return dp, dq, None, None, None, None


def smooth_score(af_ctx, p, q, samples, c: float = 0.01, tau_s: float = 0.005):
    """s[n] for the pairs (p[n, 3], q[n, 4]), differentiable in p and q."""
    return SmoothScore.apply(p, q, af_ctx, samples, c, tau_s)
