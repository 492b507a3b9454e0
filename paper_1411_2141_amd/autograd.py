"""``torch.autograd.Function`` around the library's unrolled registration.

``msd = MeshRegUnrolled.apply(reg, u0, alpha, te, n_iter, ckpt_every)`` runs
``n_iter`` iterations from ``u0`` on every pair of ``reg`` and returns the
per-pair MSD of the final warp.  The forward pass writes a checkpoint every
``ckpt_every`` iterations (``mesh_reg_forward_ckpt``); its backward calls the
library's adjoint on them (``mesh_reg_backward_ckpt``), which recomputes the
iterates between checkpoints and reuses each pair's Cholesky factor, and returns
the gradients with respect to ``u0`` (``[sum n][2]`` FP64), ``alpha``
(``[n_pairs]`` FP64) and ``te`` (``[sum H*W]`` FP32, pair-major).

``alpha`` and ``te`` are pushed into the library before the forward pass
(``mesh_reg_set_alpha`` re-factorises a pair whose alpha changed;
``mesh_reg_set_template`` re-computes the spline coefficients) and pushed
again before the backward pass, so each backward differentiates at the values
its own forward used, also when several applications share one ``MeshReg``
(with ``alpha=None`` the pairs' alphas at the forward are restored; with
``te=None`` the backward refuses to run if the template was replaced since).
"""
from __future__ import annotations

import torch

from .registration import MeshReg


def push_parameters(reg: MeshReg, alpha: torch.Tensor | None, te: torch.Tensor | None) -> None:
    if alpha is not None:
        for p, a in enumerate(alpha.detach().to("cpu", torch.float64).tolist()):
            reg.set_alpha(p, a)              # a no-op when the pair already has this alpha
    if te is not None:
        flat = te.detach().to(device=reg.device, dtype=torch.float32).contiguous().view(-1)
        for p in range(reg.n_pairs):
            reg.set_template(p, reg.pixel_slice(flat, p).contiguous())


class MeshRegUnrolled(torch.autograd.Function):
    @staticmethod
    def forward(ctx, reg: MeshReg, u0, alpha, te, n_iter: int, ckpt_every: int = 10):
        push_parameters(reg, alpha, te)
        u = u0.detach().to(torch.float64).contiguous().clone()
        msd, ckpt = reg.forward_ckpt(u, n_iter, ckpt_every)
        ctx.reg = reg
        ctx.n_iter = int(n_iter)
        ctx.ckpt_every = int(ckpt_every)
        ctx.alpha_meta = (alpha.device, alpha.dtype) if alpha is not None else None
        ctx.te_meta = (te.device, te.dtype, te.shape) if te is not None else None
        # the values this forward ran at, pushed again before its backward
        ctx.alpha_val = (alpha.detach().clone() if alpha is not None
                         else torch.tensor(reg.alphas(), dtype=torch.float64))
        ctx.te_val = te.detach().clone() if te is not None else None
        ctx.te_version = reg.template_version
        ctx.save_for_backward(ckpt)
        return msd

    @staticmethod
    def backward(ctx, grad_msd):
        (ckpt,) = ctx.saved_tensors
        g = grad_msd.detach().to(device=ckpt.device, dtype=torch.float64).contiguous()
        if ctx.te_val is None and ctx.reg.template_version != ctx.te_version:
            raise RuntimeError("the template was replaced between this forward and its backward; "
                               "pass te to the apply to differentiate at a template of its own")
        push_parameters(ctx.reg, ctx.alpha_val, ctx.te_val)
        _, g_u0, g_alpha, g_te = ctx.reg.backward_ckpt(ckpt, ctx.n_iter, ctx.ckpt_every, g_msd=g)
        ga = gt = None
        if ctx.alpha_meta is not None:
            ga = g_alpha.to(device=ctx.alpha_meta[0], dtype=ctx.alpha_meta[1])
        if ctx.te_meta is not None:
            gt = g_te.to(device=ctx.te_meta[0], dtype=ctx.te_meta[1]).view(ctx.te_meta[2])
        return None, g_u0, ga, gt, None, None


def unrolled_msd(reg: MeshReg, u0, alpha=None, te=None, n_iter: int = 10, ckpt_every: int = 10):
    """Convenience wrapper of ``MeshRegUnrolled.apply``."""
    return MeshRegUnrolled.apply(reg, u0, alpha, te, n_iter, ckpt_every)
