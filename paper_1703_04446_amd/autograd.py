"""Lagrangian transport as a differentiable torch operation.

``LagrangianTransport.apply(v, T, plan)`` returns u1 = T(y(v, x_c, 1, 0))
(eq. rhoEndIR, characteristics by RK4 as in Algorithm 1).  The backward pass
is the library's hand-written J^T kernel (``lag_vjp``), which recomputes the
characteristics instead of storing them (the memory of the derivative does
not grow with the number of RK4 steps, as the paper stresses in Sec. 3.2).

Gradients:
  dL/dv = (d_v u1)^T g      (lag_vjp with weights g = dL/du1)
  dL/dT = P(phi)^T g        P = linear interpolation at the end points; its
                            transpose is the push-forward (lag_pushforward)
                            applied to g along the same end points (Sec. 3.1:
                            F is the transpose of linear interpolation).
Only the end-point displacements phi (dim x n_points floats) are kept for the
template gradient; nothing per RK4 step is stored.
"""

from __future__ import annotations

import torch

from . import _lib as L


class LagrangianTransport(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, T, plan):
        if plan.prob.model != L.LAG_TRANSPORT:
            raise ValueError("LagrangianTransport needs a transport-model plan")
        v = v.contiguous()
        T = T.contiguous()
        phi = torch.empty(plan.prob.dim * plan.n_points, device=v.device, dtype=torch.float32)
        u = torch.empty(plan.n_points, device=v.device, dtype=torch.float32)
        L.lag_trace(plan, v, -1, phi)
        L.lag_transport(plan, T, phi, u)
        ctx.plan = plan
        ctx.save_for_backward(v, T, phi)
        return u

    @staticmethod
    def backward(ctx, gu):
        v, T, phi = ctx.saved_tensors
        plan = ctx.plan
        gu = gu.contiguous().to(torch.float32)
        gv = gT = None
        if ctx.needs_input_grad[0]:
            gv = torch.empty_like(v)
            L.lag_vjp(plan, v, T, gu, gv)
        if ctx.needs_input_grad[1]:
            gT = torch.empty_like(T)
            L.lag_pushforward(plan, gu, phi, gT)
        return gv, gT, None


def lagrangian_transport(v, T, plan):
    """Functional form of :class:`LagrangianTransport`."""
    return LagrangianTransport.apply(v, T, plan)
