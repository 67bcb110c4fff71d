"""The residual as a differentiable torch function (argument marshalling only).

Residual(ctx, v_old)(v, vhat) returns (R_V, R_Vhat) of Sec. 4.1 (eq. s32a-c,
time term of eq. C242) with q the weak gradient of (v, vhat), computed by
mehdg_assemble.  Reverse mode calls the library's hand-written VJP
(mehdg_vjp), forward mode its JVP (mehdg_jvp); both read the pointwise
Jacobian coefficients stored by the forward call.  If the context has been
used at another state since, the products first re-linearise at the saved
inputs.  The context must have alpha_ps = 0: the pseudo-time term is part of
the Newton Jacobian but not a derivative of the residual.
"""
from __future__ import annotations

import torch

from . import mehdg


class Residual:
    """(v, vhat) -> (R_v, R_vhat) on one library context."""

    def __init__(self, ctx: "mehdg.Context", v_old: torch.Tensor):
        if float(ctx.params.get("alpha_ps", 0.0)) != 0.0:
            raise ValueError("the context must have alpha_ps = 0 to differentiate the residual")
        self.ctx = ctx
        self.v_old = v_old.contiguous()
        self.generation = 0

    def __call__(self, v, vhat):
        return _ResidualFn.apply(v, vhat, self)

    def linearise(self, v, vhat):
        """Residual at (v, vhat); stores the coefficients the products read."""
        S = self.ctx.shapes()
        e = lambda k: torch.empty(S[k], dtype=torch.float64, device=v.device)
        R_q, R_v, R_vh, ent = e("R_q"), e("R_v"), e("R_vhat"), e("entropy")
        self.ctx.assemble(v.detach().contiguous(), vhat.detach().contiguous(), None, self.v_old,
                          R_q, R_v, R_vh, ent, want_blocks=2)
        self.generation += 1
        return R_v, R_vh


class _ResidualFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, v, vhat, op):
        R_v, R_vh = op.linearise(v, vhat)
        fctx.op = op
        fctx.generation = op.generation
        fctx.save_for_backward(v, vhat)
        fctx.save_for_forward(v, vhat)
        return R_v, R_vh

    @staticmethod
    def _at_state(fctx, v, vhat):
        op = fctx.op
        if op.generation != fctx.generation:
            op.linearise(v, vhat)
            fctx.generation = op.generation
        return op

    @staticmethod
    def backward(fctx, g_Rv, g_Rvh):
        v, vhat = fctx.saved_tensors
        op = _ResidualFn._at_state(fctx, v, vhat)
        g_Rv = torch.zeros_like(v) if g_Rv is None else g_Rv.contiguous()
        g_Rvh = torch.zeros_like(vhat) if g_Rvh is None else g_Rvh.contiguous()
        g_v, g_vh = torch.empty_like(v), torch.empty_like(vhat)
        op.ctx.vjp(g_Rv, g_Rvh, g_v, g_vh)
        return g_v, g_vh, None

    @staticmethod
    def jvp(fctx, dv, dvh, _op):
        v, vhat = fctx.saved_tensors
        op = _ResidualFn._at_state(fctx, v, vhat)
        S = op.ctx.shapes()
        dv = torch.zeros_like(v) if dv is None else dv.contiguous()
        dvh = torch.zeros_like(vhat) if dvh is None else dvh.contiguous()
        JR_q = torch.empty(S["R_q"], dtype=torch.float64, device=v.device)
        JR_v, JR_vh = torch.empty_like(v), torch.empty_like(vhat)
        op.ctx.jvp(dv, dvh, None, JR_q, JR_v, JR_vh)
        return JR_v, JR_vh
