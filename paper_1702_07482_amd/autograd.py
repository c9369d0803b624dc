"""torch.autograd binding of the hand-written backward (tnrd_backward).

TNRDFunction.apply(f, filters, rbf_w, lam, model_meta) returns u_T and is
differentiable with respect to filters, rbf_w and lam (Sec. 3.2: gradients of
the training loss for every stage's filters, influence-function weights and
reaction weight).  Both passes run in libtnrd's HIP kernels; torch only
provides memory, the stream and the graph bookkeeping.

The forward keeps the checkpoint states the backward needs (all T + 1 states,
or every s-th with opts.recompute_every = s, the others being recomputed
inside tnrd_backward).  When f requires a gradient, dl/df comes from the same
backward call in full (u_0 = f plus every reaction step's explicit f).  The
reaction is the model's: "prox" (eq. diffusionprocessfinal) or "projected"
(eq. diffusion_backP, threshold proj_c).
"""
from __future__ import annotations

import torch

from . import tnrd


class TNRDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, filters, rbf_w, lam, meta):
        dm = _model(filters, rbf_w, lam, meta)
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
        dm = _model(filters, rbf_w, lam, meta)
        opts = meta.get("opts") or tnrd.default_opts()
        g = grad_u.contiguous()
        if g.dim() == 2:
            g = g[None]
        want_f = ctx.needs_input_grad[0]
        fd = f.detach() if f.dim() == 3 else f.detach()[None]
        out = tnrd.backward(fd, dm, states, g, L=meta.get("L", 1), opts=opts, want_f=want_f)
        dK, dW, dl = out[:3]
        df = out[3].view_as(f) if want_f else None
        return df, dK, dW, dl, None


def _model(filters, rbf_w, lam, meta):
    return tnrd.DeviceModel(filters.detach(), rbf_w.detach(), lam.detach(), meta["mu0"],
                            meta["step"], meta["sigma"], meta.get("L_model", 0),
                            tnrd.REACTIONS[meta.get("reaction", "prox")],
                            float(meta.get("proj_c", 1.0)))


def tnrd_apply(f, filters, rbf_w, lam, mu0=-310.0, step=10.0, sigma=10.0, L=1, opts=None,
               reaction="prox", proj_c=1.0):
    """u_T = TNRD(f) with autograd support for f, filters, rbf_w and lam."""
    meta = {"mu0": float(mu0), "step": float(step), "sigma": float(sigma), "L": int(L),
            "opts": opts, "reaction": reaction, "proj_c": float(proj_c)}
    return TNRDFunction.apply(f, filters, rbf_w, lam, meta)
