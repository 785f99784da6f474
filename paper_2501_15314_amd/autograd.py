"""torch.autograd form of the one-way time step (argument marshalling only).

ib_step(sim, u, um, p, phi, centers, vels, omegas, offsets=None) advances one
step of the scheme of Sec. 3.1 with one pressure-force correction and returns
(u^{n+1}, p^{n+1}, Phi^{n+1}).  The bodies are rigid spheres whose points sit
at X_k = centers_b + X~_k (X~_k: `offsets`, [K][3], or the offsets given to
sim.set_bodies, taken as the orientation of the step) and move with
U_k = vels_b + omegas_b x X~_k, all at t^{n+1}.  Gradients flow to every
argument: u^n, u^{n-1}, p^n, Phi^n through the transposed step, centers
through dl/dX_k summed over each body's points, the offsets through dl/dX_k
itself (with zero angular velocities: the lever-arm term of omegas x X~_k is
not formed), vels and omegas through dl/dU_k.

The backward pass recomputes its step from the saved inputs before running
sim_step_adjoint (checkpointing: the handle's state may have moved on), so
an unrolled loop stores only the fields each step takes as input.  Both passes
run in the HIP library; nothing here computes on the CPU.
"""
from __future__ import annotations

import numpy as np
import torch

from .workloads import MOTION_PRESCRIBED, Body


def _place(sim, centers, vels, omegas, offsets=None):
    """Prescribed bodies whose kinematics at t^{n+1} = 0 are the given ones."""
    bodies = []
    c = centers.detach().cpu().numpy()
    v = vels.detach().cpu().numpy()
    w = omegas.detach().cpu().numpy()
    for i, b in enumerate(sim.bodies):
        bodies.append(Body(center=c[i].copy(), vel=v[i].copy(), omega=w[i].copy(), radius=b.radius,
                           density_ratio=b.density_ratio, motion=MOTION_PRESCRIBED, n_points=b.n_points,
                           osc_amp=np.zeros(3), osc_omega=0.0))
    # with t^n = -dt the step places the points at t^{n+1} = 0, where the
    # prescribed centre is `center` and the orientation is the identity
    sim.set_time(-sim.cfg.dt)
    off = sim.offsets if offsets is None else offsets.detach().cpu().numpy()
    sim.set_bodies(bodies, off)


def _forward(sim, u, um, p, phi, centers, vels, omegas, offsets=None):
    _place(sim, centers, vels, omegas, offsets)
    sim.set_fields(0, u, p, phi)
    sim.set_fields(1, um)
    st, rc = sim.step(1)
    u1, p1 = sim.get_fields()
    f1, _ = sim.get_forces()
    return u1, p1, f1 / sim.cfg.h ** 3


class IBStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, u, um, p, phi, centers, vels, omegas, offsets):
        if sim.cfg.outer_iters != 1:
            raise ValueError("the differentiable step takes one correction (outer_iters = 1)")
        if offsets is not None and offsets.requires_grad and bool(torch.any(omegas != 0)):
            raise ValueError("gradients with respect to the offsets need zero angular velocities")
        out = _forward(sim, u, um, p, phi, centers, vels, omegas, offsets)
        ctx.sim = sim
        ctx.has_off = offsets is not None
        ctx.save_for_backward(u, um, p, phi, centers, vels, omegas, offsets)
        return out

    @staticmethod
    def backward(ctx, gu, gp, gphi):
        sim = ctx.sim
        u, um, p, phi, centers, vels, omegas, offsets = ctx.saved_tensors
        _forward(sim, u, um, p, phi, centers, vels, omegas, offsets if ctx.has_off else None)
        r = sim.step_adjoint(gu, gp, gphi, want_inputs=True)
        gX = r["gX"]
        gc = torch.stack([gX[b0:b0 + b.n_points].sum(dim=0) for b0, b in
                          zip(np.cumsum([0] + [b.n_points for b in sim.bodies[:-1]]), sim.bodies)])
        dev = centers.device
        gv = torch.as_tensor(r["gU"], dtype=torch.float64, device=dev)
        gw = torch.as_tensor(r["gW"], dtype=torch.float64, device=dev)
        goff = gX.to(dev) if ctx.has_off else None
        return None, r["gu"], r["gum"], r["gp"], r["gphi"], gc.to(dev), gv, gw, goff


def ib_step(sim, u, um, p, phi, centers, vels, omegas, offsets=None):
    return IBStep.apply(sim, u, um, p, phi, centers, vels, omegas, offsets)
