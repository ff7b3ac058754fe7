"""torch.autograd bridge of the discrete adjoint.

``objective(sim, phi0, ...)`` runs ``n_steps`` of the colour-gradient step
from the rest state of ``phi0`` with the given contact angle (a scalar or a
per-voxel field, degrees), body-force acceleration and, for runs with Zou-He
faces, inlet and outlet densities ``rho = (rho_in, rho_out)``, and returns the
objective as a 0-d float64 tensor whose backward pass hands out the exact
discrete gradient computed by the library's adjoint (cg_lbm_adjoint: reverse
kernels with checkpoint-every-K recomputation).  The forward call already
runs the adjoint, so the backward pass only scales the stored gradient.
"""
from __future__ import annotations

import numpy as np
import torch


class CgObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, phi0, spec, theta, g, theta_field, rho):
        if theta_field is not None:
            sim.set_wetting(theta_field=theta_field.detach().double().cpu().numpy())
        elif theta is not None:
            sim.set_wetting(theta_deg=float(theta.detach()))
        if g is not None:
            gg = g.detach().double().cpu().numpy().reshape(-1)
            sim.set_body_force(gg)
        if rho is not None:
            r = rho.detach().double().cpu().numpy().reshape(-1)
            sim.set_pressure(float(r[0]), float(r[1]))
        sim.set_phase(phi0)
        res = sim.adjoint(spec["objective"], n_steps=spec["n_steps"],
                          checkpoint_every=spec.get("checkpoint_every"), axis=spec.get("axis", 2),
                          lo=spec.get("lo", 0), hi=spec.get("hi", 1 << 30), delta=spec.get("delta", 0.0),
                          field_grad=theta_field is not None)
        ctx.theta_like = theta
        ctx.g_like = g
        ctx.field_like = theta_field
        ctx.rho_like = rho
        ctx.res = res
        dev = next((t.device for t in (theta, g, theta_field, rho) if t is not None), torch.device("cpu"))
        return torch.tensor(res["J"], dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, gJ):
        res = ctx.res
        d_theta = d_g = d_field = d_rho = None
        if ctx.theta_like is not None and ctx.needs_input_grad[3]:
            d_theta = (gJ * res["dJ_dtheta"]).to(ctx.theta_like.dtype).reshape(ctx.theta_like.shape)
        if ctx.g_like is not None and ctx.needs_input_grad[4]:
            d_g = (gJ * torch.as_tensor(res["dJ_dg"][: ctx.g_like.numel()], device=gJ.device)).to(
                ctx.g_like.dtype).reshape(ctx.g_like.shape)
        if ctx.field_like is not None and ctx.needs_input_grad[5]:
            f = res["dJ_dtheta_field"].to(ctx.field_like.device)
            d_field = (gJ.to(f.device) * f).to(ctx.field_like.dtype).reshape(ctx.field_like.shape)
        if ctx.rho_like is not None and ctx.needs_input_grad[6]:
            d = torch.tensor([res["dJ_drho_in"], res["dJ_drho_out"]], dtype=torch.float64, device=gJ.device)
            d_rho = (gJ * d).to(ctx.rho_like.dtype).reshape(ctx.rho_like.shape)
        return None, None, None, d_theta, d_g, d_field, d_rho


def objective(sim, phi0, *, objective="saturation", n_steps, checkpoint_every=None, axis=2, lo=0, hi=1 << 30,
              delta=0.0, theta=None, g=None, theta_field=None, rho=None):
    """J(theta, g, theta_field, rho) as a differentiable 0-d tensor (see module doc)."""
    spec = dict(objective=objective, n_steps=n_steps, checkpoint_every=checkpoint_every, axis=axis, lo=lo,
                hi=hi, delta=delta)
    return CgObjective.apply(sim, np.asarray(phi0), spec, theta, g, theta_field, rho)
