"""``torch.autograd`` binding of Hybrid LSLU with a fixed lambda: x_k as a
differentiable function of b and lambda.

The forward pass is ``lslu_solve`` (Algorithm 5, ``LSLU_REG_FIXED``); the
backward pass is the library's reverse pass ``lslu_vjp``, which holds the
pivots of the forward solve fixed (the recurrence is then a smooth map of b)
and reuses the bases that solve left on the device.  This module only
marshals arguments: every step runs in the library's kernels.  Because the
reverse pass reads the forward solve's device state, no other solve may run
on the same context between the forward and the backward call (checked).
"""

from __future__ import annotations

import torch

from . import capi


class HybridLsluFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, b, lam, ctx, op, K, x0):
        st, x, info = capi.lslu_solve(ctx, op, b.detach(), K, reg="fixed",
                                      lam=float(lam), x0=x0)
        if info["k_done"] < 1:
            raise capi.LsluError(st, "no iterate was formed (zero right-hand side)")
        fctx.lslu = (ctx, op, info["k_done"], capi.solve_serial(ctx))
        return x

    @staticmethod
    def backward(fctx, xbar):
        ctx, op, k, serial = fctx.lslu
        if capi.solve_serial(ctx) != serial:
            raise RuntimeError("another solve ran on this context after the forward "
                               "pass; its reverse pass needs the forward solve's bases")
        bbar, lam_bar = capi.lslu_vjp(ctx, op, k, xbar.contiguous())
        glam = None
        if fctx.needs_input_grad[1]:
            glam = torch.tensor(lam_bar, dtype=torch.float64)
        return bbar, glam, None, None, None, None


def hybrid_lslu(ctx, op, b, lam, maxiter, x0=None):
    """x_{k_done} of Hybrid LSLU with the fixed parameter ``lam`` (a float or
    a 0-dim float64 tensor; pass one with ``requires_grad=True`` to get its
    gradient).  ``b`` (and ``x0``) are device tensors in the working
    precision of ``op``."""
    if not torch.is_tensor(lam):
        lam = torch.tensor(float(lam), dtype=torch.float64)
    return HybridLsluFunction.apply(b, lam, ctx, op, int(maxiter), x0)
