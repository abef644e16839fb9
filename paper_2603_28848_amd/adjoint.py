"""Differentiation through the adjoint kernel: a torch.autograd.Function around the collision integral and
a log-space Heun rollout built on it.

The collision integral is the frozen-map estimator of one Vegas iteration with fixed counters (common
random numbers): C(f; lambda, m0) on every node of every species.  Its backward is bmc_vjp (dL/df, dL/dlambda,
dL/dm0).  The Heun step (Sec. III.C) f* = f exp(dt k1/f), f' = f exp(dt/2 (k1/f + k2/f*)) is composed from two
such calls with a fixed step size; autograd keeps the f of every stage (a checkpoint per Heun step) and the
adjoint kernel recomputes the samples in the backward pass.
"""
from __future__ import annotations

import numpy as np
import torch

from . import boltzmc as bm


def _opts(base: bm.RunOpts, epoch: int) -> bm.RunOpts:
    o = bm.default_opts(n_samples=base.n_samples, n_iter=1, first_iter=base.first_iter, seed=base.seed, epoch=epoch,
                        precision=bm.FP64, launch=bm.LAUNCH_BATCHED, freeze_maps=1, eval_stride=1)
    return o


def _apply_params(bctx: bm.Context, coupling: torch.Tensor, mass: torch.Tensor):
    for p, lam in enumerate(coupling.detach().cpu().tolist()):
        bctx.set_coupling(p, lam)
    for s, m0 in enumerate(mass.detach().cpu().tolist()):
        kind, _, A, w = bctx.masses[s]
        bctx.set_mass(s, kind, m0, A, w)


class CollisionFn(torch.autograd.Function):
    """C on every node (all species concatenated) from f (all species concatenated), the couplings of the
    processes and the mass parameters m0 of the species, at time t with the counters of `epoch`."""

    @staticmethod
    def forward(ctx, f, coupling, mass, bctx, t, base_opts, epoch):
        _apply_params(bctx, coupling, mass)
        bctx.set_f_all(f.detach().to(torch.float64).contiguous())
        bctx.set_time(float(t))
        C, _ = bctx.collision(-1, -1, _opts(base_opts, epoch))
        ctx.save_for_backward(f.detach().clone(), coupling.detach().clone(), mass.detach().clone())
        ctx.bctx, ctx.t, ctx.base, ctx.epoch = bctx, float(t), base_opts, epoch
        return torch.from_numpy(C).to(f.device)

    @staticmethod
    def backward(ctx, gC):
        f, coupling, mass = ctx.saved_tensors
        bctx = ctx.bctx
        _apply_params(bctx, coupling, mass)
        bctx.set_f_all(f.to(device="cuda:%d" % bctx.device, dtype=torch.float64).contiguous())
        bctx.set_time(ctx.t)
        gf, gl, gm = bctx.vjp(gC.detach().to(torch.float64).cpu().numpy(), -1, -1, _opts(ctx.base, ctx.epoch))
        return (torch.from_numpy(gf).to(device=f.device, dtype=f.dtype),
                torch.from_numpy(gl).to(device=coupling.device, dtype=coupling.dtype),
                torch.from_numpy(gm).to(device=mass.device, dtype=mass.dtype), None, None, None, None)


def heun_step(bctx, f, coupling, mass, t, dt, base_opts, epoch):
    k1 = CollisionFn.apply(f, coupling, mass, bctx, t, base_opts, epoch)
    fs = f * torch.exp(dt * k1 / f)
    k2 = CollisionFn.apply(fs, coupling, mass, bctx, t + dt, base_opts, epoch + 1)
    return f * torch.exp(0.5 * dt * (k1 / f + k2 / fs))


def heun_rollout(bctx, f0, coupling, mass, t0, dt, n_steps, base_opts, epoch0=0):
    """f after n_steps Heun steps of fixed size dt (epochs epoch0 + 2s, + 2s + 1)."""
    f = f0
    t = t0
    for s in range(n_steps):
        f = heun_step(bctx, f, coupling, mass, t, dt, base_opts, epoch0 + 2 * s)
        t = t + dt
    return f


def adaptive_dt(bctx, f0, eps, dt_max, base_opts, epoch0=0, t0=0.0):
    """The step of the epsilon rule (Eq. 20) from k1 at the start, to be frozen for differentiation."""
    bctx.set_f_all(np.asarray(f0, dtype=np.float64))
    bctx.set_time(t0)
    C, _ = bctx.collision(-1, -1, _opts(base_opts, epoch0))
    r = np.max(np.abs(C / np.asarray(f0)))
    return min(dt_max, eps / r) if r > 0 else dt_max
