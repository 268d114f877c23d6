"""``torch.autograd.Function`` around the HIP render / backward of libddgs.so.

``DDGSRender.apply(renderer, views, mean, quat, log_scale, opacity_logit, feat,
b_iso, B_dir, pose_tangent, n_iso, L, entangled)`` returns the concatenated images of all
views (view-major, each H x W).  Gradients flow to every Gaussian tensor, the
two shared bases and ``pose_tangent`` (V x 6, (rho, omega) in mm and rad).
The pose actually rendered is Exp(delta) pose (R' = Exp(omega) R,
t' = Exp(omega) t + rho), composed by the library (``ddgs_compose_pose``, in
float64); the returned pose gradient is the left-tangent derivative at that
composed pose, which equals the derivative with respect to delta at
delta = 0.  Pose optimisers therefore re-base the pose after each step and
keep delta at zero.

The renderer keeps the state of its last render (tile lists, saved pixel
values) for the backward.  When another render ran on the same renderer
between this function's forward and backward (two forwards summed into one
loss, say), the backward first renders its own inputs again -- the render is
deterministic, so the state it restores is the one its forward saw.
"""
import numpy as np
import torch

from . import binding
from .synth import View


def compose_views(views, pose_tangent):
    if pose_tangent is None:
        return list(views)
    d = pose_tangent.detach().to("cpu", torch.float64).numpy().reshape(-1, 6)
    out = []
    for v, dv in zip(views, d):
        if not np.any(dv):
            out.append(v)
            continue
        pose = binding.ddgs_compose_pose(v.pose, dv)
        out.append(View(W=v.W, H=v.H, pitch=v.pitch, sdd=v.sdd, pose=pose, sid=v.sid, azimuth_deg=v.azimuth_deg))
    return out


class DDGSRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, views, mean, quat, log_scale, opacity_logit, feat, b_iso, B_dir, pose_tangent,
                n_iso, L, entangled=False):
        params = dict(mean=mean.detach(), quat=quat.detach(), log_scale=log_scale.detach(),
                      opacity_logit=opacity_logit.detach(), feat=feat.detach(), b_iso=b_iso.detach(),
                      B_dir=B_dir.detach())
        composed = compose_views(views, pose_tangent)
        renderer.set_model(params, n_iso, L, entangled)
        renderer.set_views(composed)
        img = renderer.render()
        ctx.renderer = renderer
        ctx.render_id = renderer.render_id
        ctx.inputs = (params, n_iso, L, entangled, composed)
        ctx.has_pose = pose_tangent is not None
        return img

    @staticmethod
    def backward(ctx, dimg):
        r = ctx.renderer
        if r.render_id != ctx.render_id:
            params, n_iso, L, entangled, composed = ctx.inputs
            r.set_model(params, n_iso, L, entangled)
            r.set_views(composed)
            r.render()
        need = ctx.needs_input_grad
        names = ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso", "dB_dir", "dpose")
        which = [nm for nm, flag in zip(names, need[2:10]) if flag]
        grads = r.backward(dimg.contiguous(), which=which) if which else {}
        out = [grads.get(nm) for nm in names]
        if not ctx.has_pose:
            out[-1] = None
        return (None, None, *out, None, None, None)


def render(renderer, views, params, n_iso, L, pose_tangent=None, entangled=False):
    """Differentiable render of ``views`` (list of synth.View) from ``params``
    (dict of tensors named mean, quat, log_scale, opacity_logit, feat, b_iso,
    B_dir)."""
    return DDGSRender.apply(renderer, views, params["mean"], params["quat"], params["log_scale"],
                            params["opacity_logit"], params["feat"], params["b_iso"], params["B_dir"],
                            pose_tangent, n_iso, L, entangled)
