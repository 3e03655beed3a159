"""GPU discrete adjoint: dot-product tests of each vector--Jacobian product
(through the C ABI), the rollout gradient against the oracle's autograd
gradient, and against central finite differences."""
import math
import sys

import pytest
import torch

import oracle as O
from synthetic import direction, mode_amplitudes

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inner(a, b):
    return float((a.conj() * b).real.sum())


CASES = {
    "tiny": (0.5, 50.0, 0.0, 0.0, 1.0, 12, 4, 7, 2 * math.pi),
    "heated": (0.71, 100.0, 0.0, 1.0e4, 0.7, 16, 8, 15, 2 * math.pi),
    "ragged": (0.6, 80.0, 10.0, 0.0, 1.0, 13, 5, 9, 4.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_radial_solve_vjp_dot(case):
    _say("solve vjp dot", case)
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import radial_solve_vjp
    args = CASES[case]
    p = O.Params(*args)
    ctx = nsc.Context(*args)
    ctx.set_timestep(dt=1e-3, c=0.5)
    sh = (p.F, p.N_r, p.M_theta, p.M_z)
    dX, dA, dB, ub = [direction(*sh, seed=s).cuda() for s in (31, 32, 33, 34)]
    z = torch.zeros_like(dX)
    s0 = ctx.radial_solve(z, z, z)
    s1 = ctx.radial_solve(dX, dA, dB)
    lhs = _inner(ub, s1 - s0)
    xb, ab, bb = radial_solve_vjp(ctx, ub)
    rhs = _inner(xb, dX) + _inner(ab, dA) + _inner(bb, dB)
    torch.cuda.synchronize()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs), (lhs, rhs)


@pytest.mark.parametrize("case", list(CASES))
def test_nonlinear_vjp_dot(case):
    """N is quadratic (plus linear buoyancy), so the central difference
    (N(u+d) - N(u-d))/2 is the exact Jacobian action."""
    _say("nonlinear vjp dot", case)
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import nonlinear_vjp
    args = CASES[case]
    p = O.Params(*args)
    ctx = nsc.Context(*args)
    sh = (p.F, p.N_r, p.M_theta, p.M_z)
    u = (O.base_state(p) + 1e-2 * direction(*sh, seed=41)).cuda()
    d = (1e-1 * direction(*sh, seed=42)).cuda()
    nb = direction(*sh, seed=43).cuda()
    jd = 0.5 * (ctx.nonlinear(u + d) - ctx.nonlinear(u - d))
    lhs = _inner(nb, jd)
    rhs = _inner(nonlinear_vjp(ctx, u, nb), d)
    torch.cuda.synchronize()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs), (lhs, rhs)


def test_energy_grad_matches_oracle_autograd():
    _say("energy grad")
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import energy_grad
    args = CASES["heated"]
    p = O.Params(*args)
    u = O.base_state(p) + 1e-2 * direction(p.F, p.N_r, p.M_theta, p.M_z, 51)
    x = u.clone().requires_grad_(True)
    O.energy(p, x).backward()
    ctx = nsc.Context(*args)
    g = energy_grad(ctx, u.cuda()).cpu()
    assert float((g - x.grad).abs().max()) <= 1e-12 * float(x.grad.abs().max())


@pytest.mark.parametrize("case,steps,ckpt", [("tiny", 6, 4), ("heated", 4, 2)])
def test_rollout_gradient_matches_oracle_autograd(case, steps, ckpt):
    _say("rollout gradient", case)
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import rollout_energy
    args = CASES[case]
    p = O.Params(*args)
    u0 = O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-2, seed=1000))
    dt = 1e-3
    x = u0.clone().requires_grad_(True)
    uS, _ = O.run(p, x, steps, dt0=dt)
    O.energy(p, uS).backward()
    ctx = nsc.Context(*args)
    y = u0.cuda().requires_grad_(True)
    e = rollout_energy(ctx, y, steps, dt, ckpt_every=ckpt)
    e.backward()
    torch.cuda.synchronize()
    g = y.grad.cpu()
    assert float((g - x.grad).abs().max()) <= 1e-10 * float(x.grad.abs().max())


def test_rollout_gradient_finite_differences_adjoint_workload():
    """Adjoint workload (eta = 0.71, Re_i = 200, N_r = 64, 32 x 63 modes,
    200 steps at dt = 5e-4, checkpoint every 20): gradient vs FP64 central
    differences along 8 seeded directions."""
    _say("FD adjoint workload")
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import rollout, rollout_energy
    from paper_1908_00587_amd.workloads import WORKLOADS, amplitudes, params
    name = "tc-adjoint-n64"
    w = WORKLOADS[name]
    ctx = nsc.Context(*params(name))
    amps = amplitudes(name).cuda()
    u0 = ctx.initial_state(amps)
    pert_norm = float(torch.linalg.vector_norm(u0 - ctx.initial_state(0 * amps)))
    steps, dt = w["steps"], w["dt"]
    y = u0.clone().requires_grad_(True)
    e = rollout_energy(ctx, y, steps, dt, ckpt_every=20)
    e.backward()
    g = y.grad
    ctx.set_timestep(dt=dt)
    worst = 0.0
    for s in range(2000, 2008):
        d = direction(ctx.F, ctx.N_r, ctx.M_theta, ctx.M_z, s).cuda()
        d = d * (1e-3 * pert_norm / float(torch.linalg.vector_norm(d)))
        eps = 1.0
        ep = float(ctx.energy(rollout(ctx, u0 + eps * d, steps, dt)).cpu()[0])
        em = float(ctx.energy(rollout(ctx, u0 - eps * d, steps, dt)).cpu()[0])
        fd = (ep - em) / (2 * eps)
        an = _inner(g, d)
        worst = max(worst, abs(fd - an) / abs(fd))
        _say(f"dir {s}: fd {fd:.12e} adjoint {an:.12e} rel {abs(fd - an) / abs(fd):.2e}")
    assert worst <= 1e-6


def test_fused_step_calls_match_composition():
    """nsc_step_stages reproduces nsc_step bit for bit, and nsc_step_vjp the
    Python composition of the stage VJPs (same kernels in the same order)."""
    _say("fused step stages / vjp")
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import (step_stages, step_stages_fused, step_vjp,
                                              step_vjp_fused)
    args = CASES["heated"]
    p = O.Params(*args)
    ctx = nsc.Context(*args)
    dt = 1e-3
    ctx.set_timestep(dt=dt)
    u = O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-3, seed=31)).cuda()
    st, un = step_stages_fused(ctx, u)
    ref = u.clone()
    ctx.step(ref, dt)
    torch.cuda.synchronize()
    assert torch.equal(un, ref)
    st2, _ = step_stages(ctx, u)
    assert torch.equal(st[0], st2[0])
    ubar_next = direction(p.F, p.N_r, p.M_theta, p.M_z, 32).cuda()
    a = step_vjp_fused(ctx, u, st, ubar_next)
    b = step_vjp(ctx, u, ubar_next, 1, st2)
    torch.cuda.synchronize()
    assert float((a - b).abs().max() / b.abs().max()) < 1e-14


def test_rollout_gradient_full_size_largest_workload():
    """Largest workload (N_r = 256, 512 x 1023 modes, 1536^2 planes; mixed
    precision, the only one whose theta line sets fit the LDS there): the
    adjoint at full size on a short schedule (2 steps at a CFL-sized dt,
    checkpoint every step), gradient vs central differences along one seeded
    direction.  About 230 GiB of device memory."""
    _say("FD adjoint, largest workload")
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import rollout, rollout_energy
    from paper_1908_00587_amd.workloads import amplitudes, params
    name = "tc-conv-n256"
    ctx = nsc.Context(*params(name))
    ctx.set_precision("mixed")
    amps = amplitudes(name).cuda()
    u0 = ctx.initial_state(amps)
    base = ctx.initial_state(0 * amps)
    pert_norm = float(torch.linalg.vector_norm(u0 - base))
    del base
    steps, dt = 2, 1e-6
    u0.requires_grad_(True)
    e = rollout_energy(ctx, u0, steps, dt, ckpt_every=1)
    e.backward()
    g = u0.grad
    u0 = u0.detach()
    torch.cuda.synchronize()
    _say("  gradient done")
    d = direction(ctx.F, ctx.N_r, ctx.M_theta, ctx.M_z, 2100).cuda()
    d = d * (1e-3 * pert_norm / float(torch.linalg.vector_norm(d)))
    ctx.set_timestep(dt=dt)
    ep = float(ctx.energy(rollout(ctx, u0 + d, steps, dt)).cpu()[0])
    em = float(ctx.energy(rollout(ctx, u0 - d, steps, dt)).cpu()[0])
    fd = (ep - em) / 2.0
    an = _inner(g, d)
    _say(f"  fd {fd:.12e} adjoint {an:.12e} rel {abs(fd - an) / abs(fd):.2e}")
    assert abs(fd - an) <= 1e-4 * abs(fd)


@pytest.mark.parametrize("case", ["heated"])
def test_memory_options_give_the_same_gradient(case):
    """Checkpoints in pinned host memory and stage states recomputed per step
    (the memory options of the backward pass) run the same kernels in the
    same order: the gradient is bit for bit the default one."""
    _say("adjoint memory options", case)
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import rollout_energy
    args = CASES[case]
    p = O.Params(*args)
    u0 = (O.base_state(p) + 1e-3 * direction(p.F, p.N_r, p.M_theta, p.M_z, 31)).cuda()
    ctx = nsc.Context(*args)
    grads = []
    for offload, keep in [(False, True), (True, False)]:
        y = u0.clone().requires_grad_(True)
        rollout_energy(ctx, y, 7, 1e-3, ckpt_every=3, offload=offload, keep_stages=keep).backward()
        grads.append(y.grad.cpu())
    assert torch.equal(grads[0], grads[1])


def test_largest_workload_full_adjoint_schedule():
    """The largest workload's schedule on one GPU: 100 mixed-precision steps,
    the gradient of the final perturbation energy over the last 50 of them
    with a checkpoint every 10, with the backward pass's memory options
    (checkpoints in pinned host memory, stage states recomputed per step);
    checked against central differences along one seeded direction.  Prints
    the adjoint/forward cost ratio and the device memory in use."""
    _say("largest workload, full adjoint schedule")
    import time
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd.adjoint import rollout, rollout_energy
    from paper_1908_00587_amd.workloads import amplitudes, params
    name = "tc-conv-n256"
    ctx = nsc.Context(*params(name))
    ctx.set_precision("mixed")
    amps = amplitudes(name).cuda()
    u = ctx.initial_state(amps)
    base = ctx.initial_state(0 * amps)
    pert_norm = float(torch.linalg.vector_norm(u - base))
    del base
    dt = 2e-6  # fixed schedule; the initial state's CFL bound is 4.1e-6
    ctx.set_timestep(dt=dt)
    for _ in range(50):
        ctx.step(u, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u50 = u.clone()
    u = rollout(ctx, u50, 50, dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del u
    y = u50.clone().requires_grad_(True)
    t0 = time.perf_counter()
    e = rollout_energy(ctx, y, 50, dt, ckpt_every=10, offload=True, keep_stages=False)
    e.backward()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    free, total = torch.cuda.mem_get_info()
    _say(f"  forward {t_fwd:.2f} s, energy + gradient {t_all:.2f} s, ratio {t_all / t_fwd:.2f}; "
         f"torch peak {torch.cuda.max_memory_allocated() / 2**30:.1f} GiB, "
         f"in use now {(total - free) / 2**30:.1f} of {total / 2**30:.1f} GiB")
    g = y.grad
    del y, e
    d = direction(ctx.F, ctx.N_r, ctx.M_theta, ctx.M_z, 2101).cuda()
    d = d * (1e-3 * pert_norm / float(torch.linalg.vector_norm(d)))
    ctx.set_timestep(dt=dt)
    ep = float(ctx.energy(rollout(ctx, u50 + d, 50, dt)).cpu()[0])
    em = float(ctx.energy(rollout(ctx, u50 - d, 50, dt)).cpu()[0])
    fd = (ep - em) / 2.0
    an = _inner(g, d)
    _say(f"  fd {fd:.12e} adjoint {an:.12e} rel {abs(fd - an) / abs(fd):.2e}")
    assert abs(fd - an) <= 1e-4 * abs(fd)
