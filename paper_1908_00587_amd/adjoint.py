"""Discrete adjoint of the time stepper: gradients of the perturbation
kinetic energy after S steps with respect to the initial state
(optimal-perturbation search), by checkpoint-and-recompute over steps.

Every vector--Jacobian product runs in the library (nsc_nonlinear_vjp,
nsc_radial_solve_vjp, nsc_energy_grad, and per step nsc_step_stages /
nsc_step_vjp, which chain them in one call); this module only sequences
them.
The time-step schedule and the number of corrector stages are held fixed
(not differentiated).  Inner product: sum over all stored entries of
Re(conj(a) b), so a complex gradient entry is dE/dRe + i dE/dIm.
"""
import ctypes

import torch

from ._lib import check


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def nonlinear_vjp(ctx, u, nbar, ubar=None):
    """ubar += (dN/du)^T nbar; returns ubar."""
    if ubar is None:
        ubar = torch.zeros_like(u)
    ctx._sync_stream()
    check(ctx._L.nsc_nonlinear_vjp(ctx._h, _p(u), _p(nbar), _p(ubar)), "nsc_nonlinear_vjp")
    return ubar


def radial_solve_vjp(ctx, ubar_out, ubar_n=None, nbar_n=None, nbar_q=None):
    """Accumulates the transposed implicit stage; returns (ubar_n, nbar_n, nbar_q)."""
    ubar_n = torch.zeros_like(ubar_out) if ubar_n is None else ubar_n
    nbar_n = torch.zeros_like(ubar_out) if nbar_n is None else nbar_n
    nbar_q = torch.zeros_like(ubar_out) if nbar_q is None else nbar_q
    ctx._sync_stream()
    check(ctx._L.nsc_radial_solve_vjp(ctx._h, _p(ubar_out), _p(ubar_n), _p(nbar_n), _p(nbar_q)),
          "nsc_radial_solve_vjp")
    return ubar_n, nbar_n, nbar_q


def energy_grad(ctx, u):
    g = torch.empty_like(u)
    ctx._sync_stream()
    check(ctx._L.nsc_energy_grad(ctx._h, _p(u), _p(g)), "nsc_energy_grad")
    return g


def step_stages(ctx, u, n_corr=1):
    """One predictor--corrector step at state u (current dt) by its stages:
    returns (the stage states X^(1..n_corr) the adjoint needs, u^{n+1})."""
    a = ctx.nonlinear(u)
    x = ctx.radial_solve(u, a, a)
    stages = []
    for _ in range(n_corr):
        stages.append(x)
        x = ctx.radial_solve(u, a, ctx.nonlinear(x))
    return stages, x


def step_vjp(ctx, u, ubar_next, n_corr=1, stages=None):
    """Adjoint of one predictor--corrector step at state u (current dt),
    walking the stages backwards; the stage states are recomputed unless
    given (as returned by step_stages)."""
    if stages is None:
        stages, _ = step_stages(ctx, u, n_corr)
    ubar = torch.zeros_like(u)
    abar = torch.zeros_like(u)
    xbar = ubar_next
    for q in range(n_corr, 0, -1):
        # X^(q+1) = S(u, a, N(X^(q)))
        bbar = torch.zeros_like(u)
        radial_solve_vjp(ctx, xbar, ubar, abar, bbar)
        xbar = nonlinear_vjp(ctx, stages[q - 1], bbar)
    # X^(1) = S(u, a, a)
    bbar = torch.zeros_like(u)
    radial_solve_vjp(ctx, xbar, ubar, abar, bbar)
    abar += bbar
    nonlinear_vjp(ctx, u, abar, ubar)
    return ubar


def step_stages_fused(ctx, u, n_corr=1, u_next=None):
    """step_stages in one library call (nsc_step_stages): returns
    (stage states [n_corr][...], u^{n+1}); u_next: optional output buffer."""
    stages = torch.empty((max(n_corr, 1),) + tuple(u.shape), dtype=u.dtype, device=u.device)
    if u_next is None:
        u_next = torch.empty_like(u)
    ctx._sync_stream()
    check(ctx._L.nsc_step_stages(ctx._h, _p(u), _p(stages), _p(u_next)), "nsc_step_stages")
    return stages, u_next


def step_vjp_fused(ctx, u, stages, ubar_next):
    """step_vjp in one library call (nsc_step_vjp) with the stage states of
    step_stages_fused; returns ubar."""
    ubar = torch.empty_like(u)
    ctx._sync_stream()
    check(ctx._L.nsc_step_vjp(ctx._h, _p(u), _p(stages), _p(ubar_next), _p(ubar)),
          "nsc_step_vjp")
    return ubar


def rollout(ctx, u0, steps, dt):
    """Forward: `steps` steps of size dt from a copy of u0."""
    u = u0.clone()
    for _ in range(steps):
        ctx.step(u, dt)
    return u


class RolloutEnergy(torch.autograd.Function):
    """E(u^S), u^{n+1} = Step(u^n), fixed dt; backward by checkpointing every
    `ckpt_every` steps and recomputing each segment once, stage by stage,
    keeping its stage states for the vector--Jacobian products (memory: two
    states per step of one segment for one corrector).

    For grids whose states are a sizeable part of the device memory:
    offload=True keeps the checkpoints in pinned host memory, and
    keep_stages=False keeps only the segment's step states and recomputes
    each step's stage states just before its VJP (one state per step of a
    segment, one more forward step per step)."""

    @staticmethod
    def forward(fctx, u0, ctx, steps, dt, ckpt_every, n_corr, offload, keep_stages):
        ctx.set_timestep(dt=dt, n_corr=n_corr)
        ckpts = []
        u = u0.detach().clone()
        for n in range(steps):
            if n % ckpt_every == 0:
                if offload:
                    h = torch.empty(u.shape, dtype=u.dtype, pin_memory=True)
                    h.copy_(u)
                    ckpts.append(h)
                else:
                    ckpts.append(u.clone())
            ctx.step(u, dt)
        e = ctx.energy(u)
        fctx.ctx = ctx
        fctx.steps, fctx.dt, fctx.ckpt_every, fctx.n_corr = steps, dt, ckpt_every, n_corr
        fctx.keep_stages = keep_stages
        fctx.ckpts = ckpts
        fctx.save_for_backward(u)
        return e

    @staticmethod
    def backward(fctx, ge):
        (uS,) = fctx.saved_tensors
        ctx = fctx.ctx
        ctx.set_timestep(dt=fctx.dt, n_corr=fctx.n_corr)
        ubar = energy_grad(ctx, uS) * ge.to(uS.dtype)
        steps, C = fctx.steps, fctx.ckpt_every
        for s in range(len(fctx.ckpts) - 1, -1, -1):
            n0 = s * C
            n1 = min(steps, n0 + C)
            # recompute the segment by stages, keeping each step's state and
            # stage states (the same kernels in the same order as ctx.step)
            states, stages = [], []
            x = fctx.ckpts[s].to(uS.device)
            for _ in range(n0, n1):
                states.append(x)
                if fctx.keep_stages:
                    st, x = step_stages_fused(ctx, x, fctx.n_corr)
                    stages.append(st)
                else:
                    x = x.clone()
                    ctx.step(x, fctx.dt)
            spare = None if fctx.keep_stages else torch.empty_like(uS)
            for k in range(n1 - n0 - 1, -1, -1):
                st = stages[k] if fctx.keep_stages else step_stages_fused(
                    ctx, states[k], fctx.n_corr, u_next=spare)[0]
                ubar = step_vjp_fused(ctx, states[k], st, ubar)
                st = None
                if fctx.keep_stages:
                    stages[k] = None
                states[k] = None
        return ubar, None, None, None, None, None, None, None


def rollout_energy(ctx, u0, steps, dt, ckpt_every=20, n_corr=1, offload=False, keep_stages=True):
    """Perturbation kinetic energy after `steps` steps; differentiable in u0
    (offload, keep_stages: memory options of the backward pass, see
    RolloutEnergy)."""
    return RolloutEnergy.apply(u0, ctx, steps, dt, ckpt_every, n_corr, offload, keep_stages)
