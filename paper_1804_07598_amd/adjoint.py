"""Reverse mode through the Lennard-Jones forces (section 4.1) and through
velocity-Verlet trajectories, as torch.autograd.Functions.

The parameters are theta = (eps_AA, eps_AB, eps_BB, sig_AA, sig_AB, sig_BB)
(one-type systems use entries 0 and 3).  Forces are computed in FP32 by the
library; cotangents and gradients are FP64.  All arithmetic runs in libfpm.so
(fpm_lj_forces, fpm_lj_force_vjp, fpm_step, fpm_lj_adjoint_step); this module
only orders the calls and owns the buffers.
"""
from __future__ import annotations

import torch

from . import _lib as F
from .sim import _Sim


def _prm(theta):
    t = [float(x) for x in theta.detach().cpu().tolist()]
    return tuple(t[:3]), tuple(t[3:])


class LJForceFn(torch.autograd.Function):
    """F = LJForceFn.apply(pos, theta, sim, n_types): forces (n, 3) FP64 (the
    FP32 library forces, promoted) at positions `pos` of the particles held by
    `sim`, with gradients for pos (in pos.dtype) and theta (FP64, (6,), summed
    over the systems of a batch)."""

    @staticmethod
    def forward(ctx, pos, theta, sim: _Sim, n_types: int = 1):
        eps, sig = _prm(theta)
        p32 = pos.detach().to(torch.float32).contiguous()
        sim.set_positions(p32)
        sim.lj_forces(eps, sig, n_types)
        _, _, f = sim.get()
        ctx.sim, ctx.n_types, ctx.prm = sim, n_types, (eps, sig)
        ctx.save_for_backward(p32)
        ctx.pos_dtype = pos.dtype
        return f.to(torch.float64)

    @staticmethod
    def backward(ctx, gF):
        (p32,) = ctx.saved_tensors
        sim = ctx.sim
        eps, sig = ctx.prm
        sim.set_positions(p32)
        gx, gt = sim.force_vjp(gF.to(torch.float64).contiguous(), eps, sig, ctx.n_types)
        return gx.to(ctx.pos_dtype), gt.sum(0), None, None


def _frames(nsteps: int, every: int):
    return list(range(every, nsteps + 1, every))


class LJTrajFn(torch.autograd.Function):
    """Fk = LJTrajFn.apply(x0, v0, theta, sim, dt, nsteps, frame_every,
    ckpt_every, n_types): forces (nframes, n, 3) FP64 at steps frame_every,
    2 frame_every, ..., of an nsteps velocity-Verlet trajectory from (x0, v0)
    (unit mass).  The forward keeps the state every ckpt_every steps; the
    backward recomputes each segment from its checkpoint and walks it in
    reverse with one force VJP per step.  Gradients for x0, v0 (FP64 or their
    dtype) and theta (FP64)."""

    @staticmethod
    def forward(ctx, x0, v0, theta, sim: _Sim, dt: float, nsteps: int, frame_every: int,
                ckpt_every: int, n_types: int = 1):
        eps, sig = _prm(theta)
        prm = F.lj_params(eps, sig, n_types)
        frames = _frames(nsteps, frame_every)
        sim.set_particles(x0.detach().to(torch.float32), v0.detach().to(torch.float32))
        ckpts, out = [], []
        step = 0
        while step < nsteps:
            if step > 0:
                sim.build_verlet()  # the state from here on depends on (x, v) only
            p, v, _ = sim.get()
            ckpts.append((step, p, v))
            end = min(step + ckpt_every, nsteps)
            while step < end:
                nxt = min(end, min((k for k in frames if k > step), default=end))
                # no thermo rows: the captured step graphs are reused across calls
                F.fpm_step(sim.ctx, prm, dt, nxt - step, None)
                step = nxt
                if step in frames:
                    out.append(sim.get()[2].to(torch.float64))
        ctx.sim, ctx.dt, ctx.nsteps = sim, float(dt), int(nsteps)
        ctx.frames, ctx.ckpts, ctx.n_types, ctx.prm = frames, ckpts, n_types, (eps, sig)
        ctx.dtypes = (x0.dtype, v0.dtype)
        n = x0.shape[0]
        if not out:
            return torch.zeros((0, n, 3), dtype=torch.float64, device=sim.device)
        return torch.stack(out)

    @staticmethod
    def backward(ctx, gFk):
        sim, dt, K = ctx.sim, ctx.dt, ctx.nsteps
        eps, sig = ctx.prm
        n = sim.n
        dev = sim.device
        floss = {k: gFk[j].to(torch.float64).contiguous() for j, k in enumerate(ctx.frames)}
        xbar = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        vbar = torch.zeros_like(xbar)
        fbar = floss[K].clone() if K in floss else torch.zeros_like(xbar)
        gt = torch.zeros((sim.nsys, 6), dtype=torch.float64, device=dev)
        bounds = [c[0] for c in ctx.ckpts] + [K]
        x_first = None
        prm = F.lj_params(eps, sig, ctx.n_types)
        xs = None
        for q in range(len(ctx.ckpts) - 1, -1, -1):
            s0, p, v = ctx.ckpts[q]
            s1 = bounds[q + 1]
            m = s1 - s0
            sim.set_particles(p, v)
            # the segment's positions after each of its steps, recomputed from
            # its checkpoint, then its reverse sweep (both queued on the device
            # without host round trips)
            if xs is None or xs.shape[0] < m:
                xs = torch.empty((m, n, 3), dtype=torch.float32, device=dev)
            F.fpm_step_record(sim.ctx, prm, dt, m, xs)
            F.fpm_lj_adjoint_sweep(sim.ctx, prm, dt, m, xs, [floss.get(k) for k in range(s0, s1)],
                                   xbar, vbar, fbar, gt)
            sim._keep_pos = xs  # the positions handed in stay alive with the context
            x_first = p
        if x_first is None:  # no steps: the loss sees F_0 only
            x_first = ctx.ckpts[0][1] if ctx.ckpts else None
        if x_first is not None:
            sim.set_positions(x_first)
            sim.adjoint_step(dt, None, xbar, vbar, fbar, gt, eps, sig, ctx.n_types, last=True)
        return (xbar.to(ctx.dtypes[0]), vbar.to(ctx.dtypes[1]), gt.sum(0), None, None, None,
                None, None, None)
