"""Differentiable multiblob trajectories.

A ``torch.autograd.Function`` around the library's step and its hand-written
reverse step (``mb_step_ext`` / ``mb_step_adjoint``): the forward pass runs
the trajectory keeping (q, v) checkpoints every ``checkpoint_every`` steps;
the backward pass walks the segments from the last, recomputes each segment
forward keeping the step states (q^n, v^{n+1}), and reverses its steps.  All
step arithmetic, forward and reverse, runs in the library's kernels; this
module only orders the calls and keeps the checkpoints.

The differentiated quantity is the blob velocity of the last step,
u = J(q) v (M, 3) (the particle velocity U_p is its mean over the blobs of
p), as a function of the initial blob positions q0 (M, 3), the initial
velocity field v0, the per-blob external forces G (M, 3), the spring
stiffness k and the rest lengths r0 (npairs,).  Float64 grids only.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import Springs


def _springs_for(grid, nb, pa, pb, r0, k):
    """The grid's spring table for this template, created once and given the
    trajectory's rest lengths and stiffness (mb_springs_set_params) on
    later calls."""
    key = (int(nb), pa.tobytes(), pb.tobytes())
    cache = getattr(grid, "_traj_springs", None)
    if cache is not None and cache[0] == key:
        cache[1].set_params(r0, k)
        return cache[1]
    sp = Springs(nb, pa, pb, r0, k)
    grid._traj_springs = (key, sp)
    return sp


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q0, v0, G, k, r0, grid, nb, pa, pb, nsteps, every):
        if grid.precision != "fp64":
            raise ValueError("differentiable trajectories need a float64 grid")
        r0h = r0.detach().cpu().numpy().astype(np.float64)
        springs = _springs_for(grid, nb, pa, pb, r0h, float(k))
        ctx.r0h = r0h
        q = q0.detach().clone()
        v = v0.detach().clone()
        Gd = G.detach().contiguous()
        u = torch.empty_like(q)
        ckpt = []
        for n in range(nsteps):
            if n % every == 0:
                ckpt.append((q.clone(), v.clone()))
            grid.step_ext(springs, q, v, None, Gd, 1,
                          u_out=u if n == nsteps - 1 else None)
        ctx.grid, ctx.springs, ctx.ckpt = grid, springs, ckpt
        ctx.G, ctx.nsteps, ctx.every, ctx.nb = Gd, nsteps, every, nb
        ctx.vshape, ctx.k = v0.shape, float(k)
        return u

    @staticmethod
    def backward(ctx, du):
        grid, springs, G = ctx.grid, ctx.springs, ctx.G
        # another trajectory on this grid may have changed the shared table
        springs.set_params(ctx.r0h, ctx.k)
        nb, nsteps, every = ctx.nb, ctx.nsteps, ctx.every
        dev = G.device
        f64 = torch.float64
        M = G.shape[0]
        ubar_last = du.to(f64).contiguous()  # dloss/du of the last step
        qbar = torch.zeros((M, 3), dtype=f64, device=dev)
        vbar = torch.zeros(ctx.vshape, dtype=f64, device=dev)
        Gbar = torch.zeros((M, 3), dtype=f64, device=dev)
        kbar = torch.zeros(1, dtype=f64, device=dev)
        r0bar = torch.zeros(springs.npairs, dtype=f64, device=dev)
        for s in reversed(range(len(ctx.ckpt))):
            n0 = s * every
            n1 = min(n0 + every, nsteps)
            q = ctx.ckpt[s][0].clone()
            v = ctx.ckpt[s][1].clone()
            states = []
            for _ in range(n0, n1):
                qn = q.clone()
                grid.step_ext(springs, q, v, None, G, 1)
                states.append((qn, v.clone()))
            for j in reversed(range(n1 - n0)):
                qn, vn1 = states[j]
                last = n0 + j == nsteps - 1
                grid.step_adjoint(springs, qn, vn1, qbar, vbar, None, G,
                                  ubar_last if last else None, Gbar, kbar, r0bar)
        return qbar, vbar, Gbar, kbar[0], r0bar, None, None, None, None, None, None


def trajectory(grid, nb, pair_a, pair_b, q0, v0, G, k, r0, nsteps, checkpoint_every=10):
    """Blob velocities u (M, 3) of the last of ``nsteps`` steps, through
    ``torch.autograd``: gradients flow to q0, v0, G, k (0-d tensor) and r0
    (npairs,) by the library's adjoint kernels."""
    pa = np.ascontiguousarray(pair_a, dtype=np.int32)
    pb = np.ascontiguousarray(pair_b, dtype=np.int32)
    return _Trajectory.apply(q0, v0, G, k, r0, grid, int(nb), pa, pb, int(nsteps),
                             int(checkpoint_every))


def particle_means(u, nb):
    """Particle velocities U (P, 3): the mean of u over each particle's nb
    blobs (Sec. Multiblob particle model)."""
    return u.reshape(-1, nb, 3).mean(dim=1)


def place_template(centres, rotations, template, a):
    """Blob positions (P * nb, 3) of particles with the given centres (P, 3)
    and rotations (P, 3, 3), the unit template (nb, 3) scaled by the vertex
    radius a (0-d tensor): q = c_p + a R_p t_b, differentiable in a."""
    body = (rotations @ template.T).transpose(1, 2)
    return (centres[:, None, :] + a * body).reshape(-1, 3)
