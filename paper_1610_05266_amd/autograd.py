"""torch.autograd wrappers of P2M (eq. p2m with the App. B shape functions)
and M2P (eq. m2p with linear FE mesh functions).  Forward and backward both
call the HIP library through the C ABI; the weights are rebuilt on every
forward, as the particle shape functions change whenever particles move.
"""
from __future__ import annotations

import torch

from . import ops
from ._lib import P2M_WEIGHTS_F32


class P2MFunction(torch.autograd.Function):
    """mesh_vals = P2M(pos, vals): gradients w.r.t. vals and pos.

    recompute=False keeps the weights handle from forward to backward;
    recompute=True keeps nothing but the inputs and rebuilds the weights in
    backward (the same deterministic build, so the same bits) -- the form
    for the largest sizes."""

    @staticmethod
    def forward(ctx, pos, vals, mesh, h, flags, recompute):
        if recompute and int(flags) & ~P2M_WEIGHTS_F32:
            # the recompute entry points build the default (bounded, quadratic) weights
            raise ValueError("recompute=True takes no build flags (P2M_LINEAR, P2M_PERIODIC, P2M_STRICT)")
        p, v = pos.detach().contiguous(), vals.detach().contiguous()
        if recompute:
            out = ops.p2m_project_fused(mesh, h, p, v, check_diag=True)
            ctx.w = None
        else:
            flags = int(flags) | (0 if vals.dtype == torch.float64 else P2M_WEIGHTS_F32)
            w = ops.p2m_build_weights(mesh, h, p, flags, check_diag=True)
            out = ops.p2m_project(w, v)
            ctx.w = w
        ctx.mesh, ctx.h = mesh, h
        ctx.vals_dtype = vals.dtype
        ctx.save_for_backward(pos, vals)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        pos, vals = ctx.saved_tensors
        need_pos, need_vals = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        p, v, g = pos.detach().contiguous(), vals.detach().contiguous(), grad_out.contiguous()
        if ctx.w is None:
            gp = torch.zeros_like(p) if need_pos else None
            gv, gp = ops.p2m_backward_fused(ctx.mesh, ctx.h, p, v, g, want_vals=need_vals, grad_pos=gp)
        else:
            gv, gw = ops.p2m_project_backward(ctx.w, g, v, want_vals=need_vals, want_w=need_pos)
            gp = ops.p2m_build_weights_backward(ctx.w, p, gw) if need_pos else None
        if gv is not None and gv.dtype != ctx.vals_dtype:
            gv = gv.to(ctx.vals_dtype)
        return gp, gv, None, None, None, None


class M2PFunction(torch.autograd.Function):
    """vals = M2P(mesh_vals, pos): gradients w.r.t. mesh_vals and pos."""

    @staticmethod
    def forward(ctx, mesh_vals, pos, mesh, bf16_out):
        out = ops.m2p_interpolate(mesh, mesh_vals.detach().contiguous(), pos.detach().contiguous(),
                                  bf16_out=bool(bf16_out))
        ctx.mesh = mesh
        ctx.save_for_backward(mesh_vals, pos)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        mesh_vals, pos = ctx.saved_tensors
        need_mesh, need_pos = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        g = grad_out.contiguous()
        if g.dtype == torch.bfloat16:
            g = g.float()
        if g.dtype != mesh_vals.dtype:
            g = g.to(mesh_vals.dtype)
        gp = torch.zeros_like(pos) if need_pos else None
        gm, gp = ops.m2p_interpolate_backward(ctx.mesh, mesh_vals.detach().contiguous(), pos.detach().contiguous(),
                                              g, want_mesh=need_mesh, grad_pos=gp)
        return gm, gp, None, None


def p2m(pos, vals, mesh, h, flags=0, recompute=False):
    return P2MFunction.apply(pos, vals, ops.Mesh.of(mesh), float(h), int(flags), bool(recompute))


def m2p(mesh_vals, pos, mesh, bf16_out=False):
    return M2PFunction.apply(mesh_vals, pos, ops.Mesh.of(mesh), bool(bf16_out))
