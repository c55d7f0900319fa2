"""Differentiable QP layer: a torch.autograd.Function around ipm_solve /
qp_backward (argument marshalling only; both directions run in libqpk).

One handle holds one solve: backward must run before the next forward on
the same handle (it raises otherwise); use one QP per concurrent solve.

The forward pass solves the QP for the given linear term c, row bounds lA,
uA and (for H = P^T W P) voxel weights w; the backward pass differentiates
the solution x* through the perturbed optimality conditions at the returned
point with one PCG solve on the same doubly augmented matrix as the last
Newton step (see qp_backward in include/qpk.h).
"""
from __future__ import annotations

import torch

from .qpk import QP, default_ipm_options, default_pcg_options


class QPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, qp: QP, c, lA, uA, w, opts=None):
        qp.update_data(c=c.detach().contiguous() if c is not None else None,
                       lA=lA.detach().contiguous() if lA is not None else None,
                       uA=uA.detach().contiguous() if uA is not None else None,
                       w=w.detach().contiguous() if w is not None else None)
        out = qp.solve(opts if opts is not None else default_ipm_options())
        if out["info"].result != 0:
            raise RuntimeError("interior point solve did not converge")
        ctx.qp = qp
        ctx.generation = qp.generation
        ctx.has = (c is not None, lA is not None, uA is not None, w is not None)
        return out["x"]

    @staticmethod
    def backward(ctx, grad_x):
        qp = ctx.qp
        if qp.generation != ctx.generation:
            # the handle now holds another solve (a later forward, or a call
            # that changed its data or iterate): its adjoint would belong to that
            raise RuntimeError("QPFunction.backward: the QP handle was solved or modified "
                               "after this forward; run backward before the next forward "
                               "on the same handle, or use one handle per solve")
        want = [k for k, h in zip(("c", "lA", "uA", "w"), ctx.has) if h]
        g, _ = qp.backward(grad_x.contiguous(), want=tuple(want),
                           opts=default_pcg_options(tol=1e-10, maxit=20000))
        return (None, g.get("c") if ctx.has[0] else None, g.get("lA") if ctx.has[1] else None,
                g.get("uA") if ctx.has[2] else None, g.get("w") if ctx.has[3] else None, None)


def qp_layer(qp: QP, c=None, lA=None, uA=None, w=None, opts=None):
    """x*(c, lA, uA, w) as a differentiable torch function."""
    return QPFunction.apply(qp, c, lA, uA, w, opts)
