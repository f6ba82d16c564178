"""The Neo-Hookean residual as a differentiable PyTorch function.

Forward runs the fused residual kernel; backward runs the hand-written adjoint kernel
(the transpose of the pointwise Jacobian map, scattered through E^T B^T), returning the
cotangent of the displacement and of the per-element Lame parameters.  In "recompute"
mode the backward rebuilds the linearisation from the saved displacement instead of
reading the stored one, trading flops for memory.  A "stored" backward checks that the
operator still holds the linearisation its forward stored (another forward, a solve or
a multigrid setup on the same operator replaces it); if not, it recomputes the
linearisation from the saved displacement instead.
"""
from __future__ import annotations

import torch

from .binding import Operator


class NeoHookeanResidual(torch.autograd.Function):
    """``r = NeoHookeanResidual.apply(u, mu_e, lam_e, op, mode, precision)``.

    ``u``: float64 [n_nodes][3] on the device; ``mu_e``, ``lam_e``: float64 [n_elem];
    ``op``: the fine :class:`Operator` (its geometry set up); ``mode``: "stored" or
    "recompute" (how the backward obtains the linearisation); ``precision``: "f64" or
    "f32" arithmetic of the backward (the forward residual is FP64; the gradients are
    returned as float64)."""

    @staticmethod
    def forward(ctx, u, mu_e, lam_e, op: Operator, mode: str = "recompute", precision: str = "f64"):
        mu_e = mu_e.detach().contiguous()
        lam_e = lam_e.detach().contiguous()
        op.set_material(0.0, 0.0, mu_e, lam_e)
        ud = u.detach().contiguous()
        r = op.residual(ud, store_state=(mode == "stored"))
        if mode == "stored" and precision == "f32":
            op.state_cast_f32()
        ctx.op, ctx.mode, ctx.precision = op, mode, precision
        ctx.state_version = op.state_version() if mode == "stored" else None
        ctx.save_for_backward(ud, mu_e, lam_e)
        return r

    @staticmethod
    def backward(ctx, r_bar):
        u, mu_e, lam_e = ctx.saved_tensors
        op = ctx.op
        op.set_material(0.0, 0.0, mu_e, lam_e)
        wt = torch.float64 if ctx.precision == "f64" else torch.float32
        mode = ctx.mode
        if mode == "stored" and op.state_version() != ctx.state_version:
            mode = "recompute"  # the stored linearisation is no longer this forward's
        ub, mub, lamb = op.residual_vjp(u, r_bar.contiguous().to(wt), mode=mode, precision=ctx.precision)
        return ub.to(torch.float64), mub, lamb, None, None, None
