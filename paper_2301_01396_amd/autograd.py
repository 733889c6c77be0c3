"""torch.autograd bindings of the XPBD rollout and the FP64 goal.

``XPBDRollout.apply`` runs the forward rollout through the C ABI and, in
backward, the library's exact adjoint (recomputing each frame from the
checkpoint the forward kept).  ``GoalL2.apply`` is the goal of Sec. 4.1
(W = I on the masked frames, beta = 0) reduced in FP64 on the device.
Gradients flow to x0, v0, the distance and bending compliances, the tet
Young's moduli or Lame parameters, the membrane coefficients, the per-frame
external forces, the sphere (c, R) and the body collider's vertices.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .lib import Simulator, XPBDError, XPBD_ERR_STATE


class XPBDRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim: Simulator, n_frames: int, x0, v0, dist_alpha, bend_alpha, tet_E, f_ext, sphere,
                tet_mu=None, tet_lambda=None, tri_coef=None, body_x=None):
        sph = None if sphere is None else sphere.detach().cpu().double().numpy()
        d = lambda t: None if t is None else t.detach().contiguous()
        grad = any(ctx.needs_input_grad[2:])
        xf, _, _ = sim.forward(n_frames, x0=d(x0), v0=d(v0), dist_alpha=d(dist_alpha), bend_alpha=d(bend_alpha),
                               tet_E=d(tet_E), f_ext=d(f_ext), sphere=sph, for_adjoint=grad,
                               tet_mu=d(tet_mu), tet_lambda=d(tet_lambda), tri_coef=d(tri_coef), body_x=d(body_x))
        ctx.sim = sim
        ctx.rid = sim.forward_count
        ctx.meta = [(t.dtype, t.device) if t is not None else None
                    for t in (x0, v0, dist_alpha, bend_alpha, tet_E, f_ext, sphere, tet_mu, tet_lambda, tri_coef,
                              body_x)]
        return xf

    @staticmethod
    def backward(ctx, gx):
        sim = ctx.sim
        if sim.forward_count != ctx.rid:
            raise XPBDError(XPBD_ERR_STATE, "another forward ran on this simulator before this backward")
        names = ("x0", "v0", "dist_alpha", "bend_alpha", "tet_E", "f_ext", "sphere", "tet_mu", "tet_lambda",
                 "tri_coef", "body_x")
        want = [n for n, m, need in zip(names, ctx.meta, ctx.needs_input_grad[2:]) if m is not None and need]
        g = sim.adjoint(gx.to(sim.dtype).contiguous(), None, want=want) if want else {}
        out = []
        for n, m in zip(names, ctx.meta):
            if m is None or n not in g:
                out.append(None)
            else:
                out.append(g[n].to(dtype=m[0], device=m[1]))
        return (None, None, *out)


class GoalL2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim: Simulator, x_frames, targets, frame_mask, vertex_weight=None):
        loss, dL = sim.goal_l2(x_frames.detach().contiguous(), targets.contiguous(), frame_mask, vertex_weight)
        ctx.save_for_backward(dL)
        return loss

    @staticmethod
    def backward(ctx, gl):
        (dL,) = ctx.saved_tensors
        return None, dL * gl.to(dL.dtype), None, None, None


def rollout(sim: Simulator, n_frames: int, x0, v0, dist_alpha=None, bend_alpha=None, tet_E=None, f_ext=None,
            sphere: Optional[torch.Tensor] = None, tet_mu=None, tet_lambda=None, tri_coef=None, body_x=None):
    """Differentiable rollout: returns the end-of-frame positions (F, V, 3).
    Tets take tet_E (Young's moduli, Poisson ratios fixed) or tet_mu and
    tet_lambda (Lame parameters); membrane triangles take tri_coef (n_tri, 4);
    a body collider takes its vertex positions body_x (n_body_verts, 3)."""
    return XPBDRollout.apply(sim, n_frames, x0, v0, dist_alpha, bend_alpha, tet_E, f_ext, sphere, tet_mu,
                             tet_lambda, tri_coef, body_x)


def goal_l2(sim: Simulator, x_frames, targets, frame_mask=None, vertex_weight=None):
    """Differentiable FP64 goal; vertex_weight (FP64 [V] on the device) is
    the diagonal of W, else W = I."""
    if frame_mask is None:
        frame_mask = np.ones(x_frames.shape[0], np.uint8)
    return GoalL2.apply(sim, x_frames, targets, frame_mask, vertex_weight)
