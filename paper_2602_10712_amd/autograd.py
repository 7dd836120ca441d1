"""torch.autograd.Function over srp_trace / srp_trace_adjoint.

F, tau = srp_force(scene, sun_dirs, params, rho_s, rho_d, hinge_angles)
  forward : srp_scene_set_design (materials on device, hinge angles on the host) + srp_trace
  backward: srp_trace_adjoint with the incoming gradients as seeds -> d/d rho_s, d/d rho_d (float32,
            per facet) and d/d hinge_angles (float64).  The specular-sampling probabilities are
            frozen at the values of the forward call (p_spec argument, or the default rule
            evaluated on the forward's reflectances), the Philox counters and the grid frames are
            the forward's, and visibility-edge terms are excluded (see the adjoint kernel).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B


class SRPForce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho_s, rho_d, hinge_angles, scene, sun_dirs, params, p_spec, frames):
        ang = None if hinge_angles is None else hinge_angles.detach().cpu().numpy().astype(np.float64)
        B.srp_scene_set_design(scene.handle, ang, rho_s.detach().contiguous(), rho_d.detach().contiguous(),
                               None if p_spec is None else p_spec.detach().contiguous())
        F, T = scene.trace(sun_dirs, params, frames=frames)
        ctx.scene = scene
        ctx.params = params
        ctx.sun_dirs = sun_dirs
        ctx.frames = frames
        ctx.has_hinge = hinge_angles is not None
        return F, T

    @staticmethod
    def backward(ctx, gF, gT):
        gF = torch.zeros((ctx.sun_dirs.shape[0], 3), dtype=torch.float64, device="cuda") if gF is None else gF
        grs, grd, gh = ctx.scene.adjoint(ctx.sun_dirs, ctx.params, gF.contiguous(),
                                         None if gT is None else gT.contiguous(), frames=ctx.frames)
        gh_out = gh.to("cpu") if ctx.has_hinge else None
        return grs, grd, gh_out, None, None, None, None, None


def srp_force(scene, sun_dirs, params, rho_s, rho_d, hinge_angles=None, p_spec=None, frames=None):
    """Differentiable (F [D][3], tau [D][3]) float64 on the device."""
    sd = torch.as_tensor(sun_dirs, dtype=torch.float64, device="cuda").contiguous()
    fr = None if frames is None else torch.as_tensor(frames, dtype=torch.float64, device="cuda").contiguous()
    return SRPForce.apply(rho_s, rho_d, hinge_angles, scene, sd, params, p_spec, fr)
