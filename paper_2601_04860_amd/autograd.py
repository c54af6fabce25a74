"""torch.autograd binding of the differentiable fusion.

The forward is ``divas_fuse_views`` on a session created with
``differentiable = 1`` (mask channel = logits, soft depth test); the backward
is ``divas_fuse_backward``, the hand-written deterministic adjoint kernels.  The
gradients flow to the per-view logits and the three depth maps, so a 3D
consistency loss on the fused scores can refine the 2D masks.  This module only
marshals tensors; both passes run in libdivas.
"""
from __future__ import annotations

import torch

from . import Session, ViewSet


class FusedScores(torch.autograd.Function):
    """P = fuse(logits, d_min, d_ref, d_max) for every active voxel of ``session``.

    Inputs after (session, cams): S logit maps, S d_min, S d_ref, S d_max maps
    (float32, H x W, on the session's device).  ``cams`` is a list of
    (camera dict, d_cam) pairs.
    """

    @staticmethod
    def forward(ctx, session: Session, cams, *maps):
        S = len(cams)
        if len(maps) != 4 * S:
            raise ValueError("expected 4 maps per view")
        lg, dn, dm, dx = (maps[k * S:(k + 1) * S] for k in range(4))
        vs = ViewSet()
        for i, (cam, dcam) in enumerate(cams):
            vs.add(cam, dcam, lg[i].contiguous(), dn[i].contiguous(), dm[i].contiguous(), dx[i].contiguous())
        res = session.fuse_views(vs)
        ctx.session = session
        ctx.generation = session.generation()
        ctx.views = vs
        ctx.shapes = [tuple(m.shape) for m in lg]
        ctx.needs = ctx.needs_input_grad[2:]
        n = session.info()["n_active"]
        return res["P"][:n].clone()

    @staticmethod
    def backward(ctx, gP):
        # the adjoint kernels read the session's resident state: a later fusion
        # or update of the session would give the gradient of another forward
        if ctx.session.generation() != ctx.generation:
            raise RuntimeError("the session was fused or updated again after this forward; "
                               "its gradient is no longer available")
        S = len(ctx.shapes)
        dev = gP.device
        grads = {}
        flat = []
        for k, key in enumerate(("logit", "dmin", "dref", "dmax")):
            want = any(ctx.needs[k * S:(k + 1) * S])
            lst = [torch.empty(sh, dtype=torch.float32, device=dev) if want else None for sh in ctx.shapes]
            grads[key] = lst if want else None
            flat += lst
        n = ctx.session.info()["n_active"]
        g = torch.zeros(max(n, 1), dtype=torch.float32, device=dev)
        g[:n] = gP.to(torch.float32)
        ctx.session.fuse_backward(g, grads)
        return (None, None, *flat)


def fused_scores(session, cams, logits, d_min, d_ref, d_max):
    return FusedScores.apply(session, cams, *logits, *d_min, *d_ref, *d_max)
