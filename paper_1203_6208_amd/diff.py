"""torch.autograd wrappers of the library's reverse mode.

``UTerm`` is u = D(R) F + p(D(R)) dW (the drift product plus the Chebyshev
approximation of sqrt(D) dW on a fixed interval, arXiv:1203.6208 eq. DF and
eq. cheb1-cheb3); its backward is ``rpy_u_vjp``.  ``Forces`` is the spring
plus excluded-volume force of ``rpy_forces`` with backward ``rpy_forces_vjp``.
``bd_step`` composes them into the Euler step of eq. sde,
    R' = R + (dt/4) D F + (1/sqrt 2) p(D) dW = R + u(R, (dt/4) F, dW/sqrt 2)
(u is linear in F and dW), and ``trajectory`` runs many steps with
activation checkpointing: only every ``every``-th position is kept during
the forward pass and the segments are recomputed in the backward pass.  All
arithmetic runs in the HIP library; this module only routes tensors.
"""
from __future__ import annotations

import math

import torch
from torch.utils.checkpoint import checkpoint

from . import rpy


class UTerm(torch.autograd.Function):
    """u = D(R) F + p(D(R)) dW.  Inputs: pos [N, 3], F [N, 3], dw [N, 3]
    (no gradient for dw), the rpy.Context (created with grad=1), n_cheb and
    the interval.  The V_p of the forward recurrence are kept for the
    backward pass (n_cheb x 3N doubles) when ``keep`` is true."""

    @staticmethod
    def forward(ctx, pos, F, dw, rc, n_cheb, d_min, d_max, keep=True):
        pos, F, dw = pos.contiguous(), F.contiguous(), dw.contiguous()
        u = torch.empty_like(pos)
        vh = torch.empty((n_cheb,) + tuple(pos.shape), dtype=pos.dtype,
                         device=pos.device) if keep else None
        rpy.rpy_u_forward(rc.handle, pos, F, dw, n_cheb, d_min, d_max, u, vh)
        ctx.rc, ctx.n_cheb, ctx.d_min, ctx.d_max = rc, n_cheb, d_min, d_max
        ctx.keep = keep
        if keep:
            ctx.save_for_backward(pos, F, dw, vh)
        else:
            ctx.save_for_backward(pos, F, dw)
        return u

    @staticmethod
    def backward(ctx, g):
        if ctx.keep:
            pos, F, dw, vh = ctx.saved_tensors
        else:
            (pos, F, dw), vh = ctx.saved_tensors, None
        g = g.contiguous()
        g_pos = torch.empty_like(pos)
        g_F = torch.empty_like(pos) if ctx.needs_input_grad[1] else None
        rpy.rpy_u_vjp(ctx.rc.handle, pos, F, dw, g, ctx.n_cheb, ctx.d_min, ctx.d_max, g_pos,
                      g_F, vh)
        return g_pos, g_F, None, None, None, None, None, None


class Forces(torch.autograd.Function):
    """Spring + narrow-Gaussian excluded-volume forces F(R) ([N, 3])."""

    @staticmethod
    def forward(ctx, pos, rc, ev):
        pos = pos.contiguous()
        out = torch.empty_like(pos)
        z, d, cut = (ev["zstar"], ev["dstar"], ev["rcut"]) if ev else (0.0, 0.0, 0.0)
        rpy.rpy_forces(rc.handle, pos, z, d, cut, out)
        ctx.rc, ctx.ev = rc, (z, d, cut)
        ctx.save_for_backward(pos)
        return out

    @staticmethod
    def backward(ctx, gF):
        (pos,) = ctx.saved_tensors
        g = torch.empty_like(pos)
        rpy.rpy_forces_vjp(ctx.rc.handle, pos, *ctx.ev, gF.contiguous(), g)
        return g, None, None


def noise(n, dt, seed, step, device="cuda"):
    """dW ~ N(0, dt) for step `step` (device Philox; reproducible, so that a
    recomputed segment draws the same noise)."""
    out = torch.empty((n, 3), dtype=torch.float64, device=device)
    rpy.rpy_gaussian_noise(out, seed, step, dt)
    return out


def bd_step(pos, rc, dt, n_cheb, d_min, d_max, dw, ev=None, spring=None, keep=True):
    """One differentiable Euler step.  `spring` (optional 0-d tensor) scales
    the force before the drift product, a parameter whose sensitivity flows
    through F."""
    F = Forces.apply(pos, rc, ev)
    if spring is not None:
        F = spring * F
    return pos + UTerm.apply(pos, F * (dt / 4.0), dw / math.sqrt(2.0), rc, n_cheb, d_min, d_max,
                             keep)


def trajectory(pos0, rc, n_steps, dt, n_cheb, d_min, d_max, seed, ev=None, spring=None,
               every=10, step0=0):
    """Positions after n_steps differentiable steps with checkpoints every
    `every` steps (every <= 0: no checkpointing, every step's state kept)."""
    n = pos0.shape[0]

    def segment(p, s0, k, sp):
        for i in range(k):
            p = bd_step(p, rc, dt, n_cheb, d_min, d_max, noise(n, dt, seed, s0 + i), ev, sp)
        return p

    p = pos0
    if every <= 0:
        return segment(p, step0, n_steps, spring)
    for s in range(0, n_steps, every):
        k = min(every, n_steps - s)
        # the noise comes from the library's Philox stream keyed by (seed,
        # step), not from torch's generator: no RNG state to preserve
        p = checkpoint(segment, p, step0 + s, k, spring, use_reentrant=False,
                       preserve_rng_state=False)
    return p


def msd(pos, pos0):
    """Mean over beads of |r(t) - r(0)|^2."""
    return ((pos - pos0) ** 2).sum(dim=-1).mean()
