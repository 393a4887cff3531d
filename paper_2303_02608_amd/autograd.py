"""torch.autograd.Function around the hand-written adjoint of the regression.

``wlr_alpha(y, b, feat, items, r, tr, ...)`` returns alpha (Sec. 2.1, eq. 3:
the locally fitted value f(x^c)) at the listed regressions; gradients flow to
the log brightness ``y`` and to the per-dimension bandwidths ``b`` (eq. 5)
through ``esim_wlr_backward``.  Both directions run in libesim; this module
only marshals tensors.  Items are int64 (frame << 44) | pixel and must be
distinct.
"""
from __future__ import annotations

import torch

from . import binding as B


class WLRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, b, feat, items, r, tr, C, h, ridge):
        bl = [float(v) for v in b.detach().cpu().tolist()]
        plan = B.Plan([y.detach().contiguous()], [feat], [B.Params(r, tr, C, h=h, b=bl, ridge=ridge)])
        n = items.numel()
        alpha = torch.empty(n, dtype=torch.float32, device=y.device)
        count = torch.tensor([n, 0], dtype=torch.int32, device=y.device)
        if n:
            B.regress(plan, -1, items, count, n, alpha)
        ctx.plan = plan
        ctx.save_for_backward(items)
        ctx.b_meta = (b.dtype, b.device)
        return alpha

    @staticmethod
    def backward(ctx, g_alpha):
        (items,) = ctx.saved_tensors
        plan = ctx.plan
        y = plan.ys[0]
        g_y = torch.zeros_like(y)
        g_b = torch.zeros(plan.D, dtype=torch.float64, device=y.device)
        n = items.numel()
        if n:
            nbytes = B.backward_scratch_bytes(plan, n)
            scratch = torch.empty(nbytes, dtype=torch.uint8, device=y.device)
            B.backward(plan, items, g_alpha.contiguous().float(), g_y, g_b, scratch)
        dt, dev = ctx.b_meta
        return g_y, g_b.to(dtype=dt, device=dev), None, None, None, None, None, None, None


def wlr_alpha(y, b, feat, items, r, tr, C=0.15, h=1.0, ridge=1e-6):
    return WLRFunction.apply(y, b, feat, items, r, tr, C, h, ridge)


def frame_items(t, pixels):
    """Items (t << 44) | pixel for int tensors t and pixels."""
    return (t.to(torch.int64) << 44) | pixels.to(torch.int64)
