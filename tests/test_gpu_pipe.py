"""GPU parity of the pipe-flow variant (nsc_init_pipe, through the C ABI)
against the FP64 pipe oracle (oracle/pipe.py) on the same seeded inputs:
nonlinear term, implicit stage with pressure, full steps (fixed and dynamic
step size), the seeded initial state, Hagen--Poiseuille flow held steady,
mixed precision within its stated bound, the calls a pipe context refuses,
and a full-size grid on sampled radial rows and modes."""
import math
import sys

import pytest
import torch

from oracle import pipe as P
from synthetic import direction, mode_amplitudes

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

CASES = {
    "small": (300.0, 16, 8, 15, 2 * math.pi),
    "ragged": (120.0, 13, 5, 9, 5.0),      # radix 5, odd tiles
    "iso48": (800.0, 32, 16, 31, 8.0),     # 48-point transforms (fixed-length kernels)
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(args):
    import paper_1908_00587_amd as nsc
    return nsc.Context.pipe(*args)


def rel(a, b):
    a = a.detach().cpu()
    b = b.detach().cpu()
    return float((a - b).abs().max() / b.abs().max())


def pert(a, b, base):
    a = a.detach().cpu()
    b = b.detach().cpu()
    return float((a - b).abs().max() / (b - base).abs().max())


def _state(p, seed, amp=1e-2):
    return P.base_state(p) + amp * direction(*p.shape(), seed=seed)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pipe_nonlinear(case, prec):
    _say("pipe nonlinear", case, prec)
    args = CASES[case]
    p = P.PipeParams(*args)
    u = _state(p, 11)
    ref, dtc = P.nonlinear(p, u)
    ctx = _ctx(args)
    ctx.set_precision(prec)
    out, c = ctx.nonlinear(u.cuda(), cfl=True)
    torch.cuda.synchronize()
    r = rel(out, ref)
    cd = abs(float(c.cpu()[0]) - dtc) / dtc
    _say(f"  rel {r:.2e}  cfl {cd:.2e}")
    if prec == "fp64":
        assert r < TOL64 and cd < 1e-14
    else:
        assert r < 2e-6 and cd < 1e-6


@pytest.mark.parametrize("case", list(CASES))
def test_pipe_radial_solve(case):
    _say("pipe radial solve", case)
    args = CASES[case]
    p = P.PipeParams(*args)
    u = _state(p, 21)
    Nn = 10 * direction(*p.shape(), seed=22)
    Nq = 10 * direction(*p.shape(), seed=23)
    dt = 1e-3
    ref, pref = P.radial_solve(p, u, Nn, Nq, dt)
    ctx = _ctx(args)
    ctx.set_timestep(dt=dt)
    out, pres = ctx.radial_solve(u.cuda(), Nn.cuda(), Nq.cuda(), pressure=True)
    torch.cuda.synchronize()
    _say(f"  rel {rel(out, ref):.2e}  pressure {rel(pres, pref):.2e}")
    assert rel(out, ref) < TOL64
    assert rel(pres, pref) < 1e-10


@pytest.mark.parametrize("case", ["small", "iso48"])
def test_pipe_initial_state(case):
    _say("pipe initial state", case)
    args = CASES[case]
    p = P.PipeParams(*args)
    amps = mode_amplitudes(3, p.M_theta, p.M_z, 1e-3, seed=5)
    ref = P.initial_state(p, amps)
    ctx = _ctx(args)
    u = ctx.initial_state(amps.cuda())
    torch.cuda.synchronize()
    _say(f"  rel {rel(u, ref):.2e}")
    assert rel(u, ref) < TOL64
    assert rel(ctx.grid(), P.radial_grid(p)) < 1e-15


@pytest.mark.parametrize("case,steps", [("small", 6), ("iso48", 10)])
def test_pipe_step_fp64(case, steps):
    """Every GPU step from the oracle's state against the oracle's next
    state, per field, relative to the field and to the perturbation (FP64
    bar scaled by max|x| / max|x - base|, as for the cylinders)."""
    _say("pipe step", case, steps)
    args = CASES[case]
    p = P.PipeParams(*args)
    u0 = P.initial_state(p, mode_amplitudes(3, p.M_theta, p.M_z, 1e-3, seed=1000))
    base = P.base_state(p)
    dt = 1e-4
    ops = P._Ops(p)
    ctx = _ctx(args)
    ctx.set_timestep(dt=dt)
    x = u0
    worst, worst_p = 0.0, 0.0
    for _ in range(steps):
        ref = P.step(p, x, dt, ops=ops)[0]
        g = x.cuda()
        ctx.step(g, dt)
        g = g.cpu()
        for f in range(3):
            worst = max(worst, rel(g[f], ref[f]))
            bar = TOL64 * max(1.0, float(ref[f].abs().max() / (ref[f] - base[f]).abs().max()))
            worst_p = max(worst_p, pert(g[f], ref[f], base[f]) / bar)
        x = ref
    _say(f"  per-step rel {worst:.2e}, perturbation-relative over its bar {worst_p:.2f}")
    assert worst < TOL64
    assert worst_p < 1.0


def test_pipe_dynamic_dt_matches_oracle():
    _say("pipe dynamic dt")
    args = CASES["small"]
    p = P.PipeParams(*args)
    u0 = P.initial_state(p, mode_amplitudes(3, p.M_theta, p.M_z, 1e-3, seed=7))
    steps = 5
    ref, dts = P.run(p, u0, steps, dynamic=True, cfl=0.5, dt_max=1e-2)
    assert dts[0] < 1e-2
    ctx = _ctx(args)
    ctx.set_timestep(dt=dts[0], dynamic=True, cfl=0.5, dt_max=1e-2)
    u = u0.cuda()
    dt = dts[0]
    got = []
    for _ in range(steps):
        got.append(dt)
        dt = ctx.step(u, dt)
    torch.cuda.synchronize()
    assert all(abs(a - b) <= 1e-14 * b for a, b in zip(got, dts))
    assert rel(u, ref) < TOL64


def test_pipe_hagen_poiseuille_stays():
    _say("pipe Hagen-Poiseuille")
    args = CASES["iso48"]
    p = P.PipeParams(*args)
    u0 = P.base_state(p).cuda()
    ctx = _ctx(args)
    ctx.set_timestep(dt=1e-4)
    u = u0.clone()
    for _ in range(20):
        ctx.step(u, 1e-4)
    torch.cuda.synchronize()
    assert float((u - u0).abs().max()) <= 1e-12 * p.Re


def test_pipe_mixed_step_error_stated():
    """Mixed precision over 20 steps within the stated 1e-5 of the FP64
    oracle, relative to each field and to its perturbation."""
    _say("pipe mixed steps")
    args = CASES["iso48"]
    p = P.PipeParams(*args)
    u0 = P.initial_state(p, mode_amplitudes(3, p.M_theta, p.M_z, 1e-3, seed=1000))
    dt = 1e-4
    ref, _ = P.run(p, u0, 20, dt0=dt)
    base = P.base_state(p)
    ctx = _ctx(args)
    ctx.set_precision("mixed")
    ctx.set_timestep(dt=dt)
    u = u0.cuda()
    for _ in range(20):
        ctx.step(u, dt)
    torch.cuda.synchronize()
    for f in range(3):
        e, ep = rel(u[f], ref[f]), pert(u[f], ref[f], base[f])
        _say(f"  field {f}: rel {e:.2e}, perturbation-relative {ep:.2e}")
        assert e < 1e-5 and ep < 1e-5


def test_pipe_refuses_what_it_does_not_provide():
    from paper_1908_00587_amd._lib import NSC_ERR_STATE
    args = CASES["small"]
    ctx = _ctx(args)
    u = ctx.empty()
    buf = torch.zeros(4, dtype=torch.float64, device="cuda")
    L, h = ctx._L, ctx._h
    assert L.nsc_energy(h, u.data_ptr(), buf.data_ptr()) == NSC_ERR_STATE
    assert L.nsc_energy_grad(h, u.data_ptr(), u.clone().data_ptr()) == NSC_ERR_STATE
    assert L.nsc_nonlinear_vjp(h, u.data_ptr(), u.clone().data_ptr(), u.clone().data_ptr()) == NSC_ERR_STATE
    assert L.nsc_diagnostics(h, u.data_ptr(), buf.data_ptr()) == NSC_ERR_STATE


def test_pipe_full_size_sampled():
    """The pipe workload at full size (64 points, 64 x 127 modes, 192^2
    padded planes): sampled radial rows of the nonlinear term and sampled
    modes of the implicit stage against the oracle row by row and mode by
    mode, FP64 and mixed."""
    _say("pipe full size")
    from paper_1908_00587_amd.workloads import WORKLOADS, amplitudes, pipe_params
    name = "pipe-n64"
    args = pipe_params(name)
    p = P.PipeParams(*args)
    ops = P._Ops(p)
    ctx = _ctx(args)
    u = ctx.initial_state(amplitudes(name).cuda())
    uc = u.cpu()
    rows = [0, 1, 5, 31, 62, 63]
    ref = P.herm(p, P.nonlinear_planes(p, uc, rows, ops)[0])
    for prec, bar in (("fp64", TOL64), ("mixed", 2e-6)):
        ctx.set_precision(prec)
        out = ctx.nonlinear(u).cpu()
        e = float((out[:, rows] - ref).abs().max() / ref.abs().max())
        _say(f"  nonlinear {prec} rows {rows}: rel {e:.2e}")
        assert e < bar
    ctx.set_precision("fp64")
    dt = WORKLOADS[name]["dt"]
    ctx.set_timestep(dt=dt)
    Nn = (1e2 * direction(*p.shape(), seed=31))
    Nq = (1e2 * direction(*p.shape(), seed=32))
    out = ctx.radial_solve(u, Nn.cuda(), Nq.cuda()).cpu()
    worst = 0.0
    for m, kk in [(0, p.K), (0, p.K + 1), (1, 0), (7, p.K + 5), (63, 2 * p.K), (32, p.K)]:
        x, _ = P.radial_solve_mode(p, ops, m, kk, uc[:, :, m, kk], Nn[:, :, m, kk],
                                   Nq[:, :, m, kk], dt)
        worst = max(worst, float((out[:, :, m, kk] - x).abs().max() / x.abs().max()))
    _say(f"  radial solve sampled modes: rel {worst:.2e}")
    assert worst < TOL64
