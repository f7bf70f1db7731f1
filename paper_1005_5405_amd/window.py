"""Gradient of a time-averaged lid shear through the HIP step adjoint.

J = (1/N) sum_{n=1..N} D(h^n), h^{n+1} = step(h^n) from h^0, with D the lid
shear of boltz_moments (Sec. 5.2).  ``lid_shear_window`` returns J as a torch
scalar whose backward pass runs the reverse sweep on the device: the forward
states are kept every ``every`` steps, each segment is recomputed from its
checkpoint, and the adjoint is carried back through boltz_lid_shear_adjoint
and boltz_step_adjoint.  The wall parameters are one FP64 tensor
theta = (lid_u, tau_left, tau_right, tau_top, tau of bottom face 0 .. nx-1),
the layout of the library's wall gradient.  The Philox samples of step n are
those of counter step0 + n, so the gradient is that of the sampled (fixed
seed) discrete map.
"""
from __future__ import annotations

import torch

from .binding import Boltz, Walls


def walls_from_theta(theta: torch.Tensor) -> Walls:
    t = theta.detach().to("cpu", torch.float64).numpy()
    return Walls(lid_u=float(t[0]), tau_left=float(t[1]), tau_right=float(t[2]), tau_bottom=1.0,
                 tau_top=float(t[3]), tau_bottom_x=t[4:].copy())


class _LidShearWindow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h0, theta, boltz: Boltz, n_steps: int, step0: int, every: int):
        if boltz.bc != 0:
            raise ValueError("lid_shear_window: the lid shear needs a cavity")
        if theta.numel() != boltz.grad_size():
            raise ValueError("lid_shear_window: theta needs 4 + nx values")
        walls = walls_from_theta(theta)
        h = h0.detach().to(torch.float32).contiguous().clone()
        tmp = boltz.empty()
        mom = torch.empty(boltz.ncells * 11, dtype=torch.float64, device="cuda")
        D = torch.zeros(n_steps, dtype=torch.float64, device="cuda")
        ckpts = {0: h.clone()}
        for n in range(n_steps):
            boltz.step(h, tmp, walls, step0 + n)
            h, tmp = tmp, h
            boltz.moments(h, mom, walls, D[n:n + 1])
            if (n + 1) % every == 0 and n + 1 < n_steps:
                ckpts[n + 1] = h.clone()
        ctx.boltz, ctx.walls, ctx.ckpts = boltz, walls, ckpts
        ctx.n_steps, ctx.step0, ctx.every = n_steps, step0, every
        ctx.h0_dtype, ctx.theta_like = h0.dtype, theta
        ctx.trace = D
        return D.mean()

    @staticmethod
    def backward(ctx, gJ):
        b, walls, N = ctx.boltz, ctx.walls, ctx.n_steps
        weight = float(gJ) / N
        lam = b.empty_adjoint(0.0)
        grad = torch.zeros(b.grad_size(), dtype=torch.float64, device="cuda")
        for s0 in sorted(ctx.ckpts, reverse=True):
            s1 = min(s0 + ctx.every, N)
            states = [ctx.ckpts[s0]]
            for n in range(s0, s1):
                nxt = b.empty()
                b.step(states[-1], nxt, walls, ctx.step0 + n)
                states.append(nxt)
            for n in range(s1, s0, -1):
                b.lid_shear_adjoint(states[n - s0], walls, weight, lam, grad)
                b.step_adjoint(states[n - 1 - s0], lam, lam, grad, walls, ctx.step0 + n - 1)
            del states
        g_theta = grad.to(device=ctx.theta_like.device, dtype=ctx.theta_like.dtype)
        return lam.to(ctx.h0_dtype), g_theta, None, None, None, None


def lid_shear_window(boltz: Boltz, h0: torch.Tensor, theta: torch.Tensor, n_steps: int, step0: int = 0,
                     every: int = 20) -> torch.Tensor:
    """J = (1/N) sum_{n=1..N} D(h^n) over N = n_steps steps from h0, differentiable
    in h0 and theta.  The context must be created with BOLTZ_WITH_ADJOINT."""
    if n_steps < 1 or every < 1:
        raise ValueError("lid_shear_window: n_steps and every must be positive")
    return _LidShearWindow.apply(h0, theta, boltz, int(n_steps), int(step0), int(every))
