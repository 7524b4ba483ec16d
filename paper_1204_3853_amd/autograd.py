"""torch.autograd.Functions over the hand-written discrete adjoint.

VlasovRollout advances f through `nsteps` RK4 Vlasov-Poisson steps with the
GPU library.  Its backward pass is the exact discrete adjoint of those steps
(vp_adjoint_step), not an autograd trace: the forward keeps a checkpoint
(f, a) every `every` steps; the backward replays each segment from its
checkpoint, recording the stage states of every step (vp_rk4_step_record),
and then runs the adjoint steps of the segment in reverse.

FieldEnergy is W = 1/2 sum_i E_i^2 of a state; its gradient goes through
the adjoint of the moment / Poisson / field chain (vp_field_adjoint).
"""
from __future__ import annotations

import torch

from . import vp


class VlasovRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f0, plan, dt, nsteps, every):
        f = f0.detach().contiguous().clone()
        a = vp.field_of(plan, f)
        ckpts = []
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append((f.clone(), a.clone()))
            vp.rk4_step(plan, f, a, dt)
        ctx.plan, ctx.dt, ctx.nsteps, ctx.every, ctx.ckpts = plan, dt, nsteps, every, ckpts
        return f

    @staticmethod
    def backward(ctx, grad_f):
        plan, dt, nsteps, every = ctx.plan, ctx.dt, ctx.nsteps, ctx.every
        lam = grad_f.detach().contiguous().clone()
        for m in reversed(range(len(ctx.ckpts))):
            f, a = (x.clone() for x in ctx.ckpts[m])
            n0, n1 = m * every, min(nsteps, (m + 1) * every)
            saved = []
            for _ in range(n0, n1):
                fn, an = f.clone(), a.clone()
                rec = torch.empty(plan.stage_elems, dtype=plan.dtype, device=f.device)
                vp.rk4_step_record(plan, f, a, dt, rec)
                saved.append((fn, an, rec))
            for fn, an, rec in reversed(saved):
                vp.adjoint_step(plan, fn, an, lam, dt, stages=rec, lam_n=lam)
        ctx.ckpts = None
        return lam, None, None, None, None


class FieldEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan):
        a = vp.field_of(plan, f.detach().contiguous())
        qm = plan.spec["qm"]
        E = a / qm
        ctx.plan, ctx.E, ctx.qm, ctx.shape = plan, E, qm, f.shape
        return 0.5 * (E * E).sum()

    @staticmethod
    def backward(ctx, gW):
        # dW/da = E / qm (a = qm E); then through K^T
        abar = (gW * ctx.E / ctx.qm).contiguous()
        fbar = vp.field_adjoint(ctx.plan, abar)
        return fbar.view(ctx.shape), None


def rollout(f0, plan, dt, nsteps, every=20):
    return VlasovRollout.apply(f0, plan, dt, nsteps, every)


def field_energy(f, plan):
    return FieldEnergy.apply(f, plan)
