"""Differentiable distance-field hit (autograd wrapper over the C ABI).

`df_hit(theta, grid4, rays, tmax)` returns the first root t of the trilinear
interpolant of the samples `theta` along each ray (the forward is
hyb_trace_df, +inf for a miss).  Its backward is hyb_df_backward: implicit
differentiation of g(t; theta) = 0 at the hit, d t / d theta_j =
-w_j / (grad f~ . d) for the 8 corners of the hit cell, with the hit point
recomputed from the saved t rather than a stored ray path.  Lets a distance
field be refit against triangle-hit targets to shrink its artefacts.

With `sdf` given (a grid of theta's size and format), the forward writes theta
into that handle with a deferred hyb_sdf_update instead of creating a grid per
call (nothing waits for the device; a non-finite theta gives NaN hits, and
sdf.check() raises); the backward then reads the handle, so it must run before
the next forward that updates the same handle (the usual forward, backward,
step loop).
"""
from __future__ import annotations

import torch

from . import df_backward, sdf_from_grid, sdf_update, trace_df


class DFHit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, grid4, rays, tmax, tmin=None, sdf=None):
        n = round(theta.numel() ** (1.0 / 3.0))
        values = theta.detach().contiguous().reshape(-1)
        sdf = sdf_from_grid(values, grid4) if sdf is None else sdf_update(sdf, values, deferred=True)
        t, prim, _, _ = trace_df(sdf, rays, tmax, tmin=tmin)
        ctx.sdf, ctx.tmax, ctx.n = sdf, float(tmax), n
        ctx.save_for_backward(rays, t, tmin if tmin is not None else torch.empty(0, device=t.device))
        ctx.has_tmin = tmin is not None
        ctx.theta_shape = theta.shape
        return t

    @staticmethod
    def backward(ctx, grad_t):
        rays, t, tmin = ctx.saved_tensors
        grad = torch.zeros(ctx.n ** 3, dtype=torch.float32, device=t.device)
        g = torch.nan_to_num(grad_t.contiguous().float(), nan=0.0, posinf=0.0, neginf=0.0)
        df_backward(ctx.sdf, rays, ctx.tmax, t, g, grad, tmin=tmin if ctx.has_tmin else None)
        return grad.reshape(ctx.theta_shape), None, None, None, None, None


def df_hit(theta, grid4, rays, tmax, tmin=None, sdf=None):
    """Differentiable DF hit distance of each ray (see module docstring)."""
    return DFHit.apply(theta, grid4, rays, tmax, tmin, sdf)
