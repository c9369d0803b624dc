"""torch.autograd binding of the hand-written backward (tnrd_backward).

TNRDFunction.apply(f, filters, rbf_w, lam, model_meta) returns u_T and is
differentiable with respect to filters, rbf_w and lam (Sec. 3.2: gradients of
the training loss for every stage's filters, influence-function weights and
reaction weight).  Both passes run in libtnrd's HIP kernels; torch only
provides memory, the stream and the graph bookkeeping.

The forward keeps the checkpoint states the backward needs (all T + 1 states,
or every s-th with opts.recompute_every = s, the others being recomputed
inside tnrd_backward).  f is treated as data: no gradient flows to it.
"""
from __future__ import annotations

import torch

from . import tnrd


class TNRDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, filters, rbf_w, lam, meta):
        dm = tnrd.DeviceModel(filters.detach(), rbf_w.detach(), lam.detach(), meta["mu0"],
                              meta["step"], meta["sigma"], meta.get("L_model", 0))
        opts = meta.get("opts") or tnrd.default_opts()
        L = meta.get("L", 1)
        u, states = tnrd.forward(f.detach(), dm, L=L, want_states=True, opts=opts)
        ctx.meta = meta
        ctx.save_for_backward(f, filters, rbf_w, lam, states)
        return u.view_as(f) if f.dim() == 2 else u

    @staticmethod
    def backward(ctx, grad_u):
        f, filters, rbf_w, lam, states = ctx.saved_tensors
        meta = ctx.meta
        dm = tnrd.DeviceModel(filters.detach(), rbf_w.detach(), lam.detach(), meta["mu0"],
                              meta["step"], meta["sigma"], meta.get("L_model", 0))
        opts = meta.get("opts") or tnrd.default_opts()
        g = grad_u.contiguous()
        if g.dim() == 2:
            g = g[None]
        dK, dW, dl = tnrd.backward(f.detach(), dm, states, g, L=meta.get("L", 1), opts=opts)
        return None, dK, dW, dl, None


def tnrd_apply(f, filters, rbf_w, lam, mu0=-310.0, step=10.0, sigma=10.0, L=1, opts=None):
    """u_T = TNRD(f) with autograd support for filters, rbf_w and lam."""
    meta = {"mu0": float(mu0), "step": float(step), "sigma": float(sigma), "L": int(L),
            "opts": opts}
    return TNRDFunction.apply(f, filters, rbf_w, lam, meta)
