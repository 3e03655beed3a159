"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs.  FP64 bar: relative max-norm deviation <= 1e-12
(a few ulp of FP64 amplified by the conditioning of the radial operators;
derivation in DESIGN.md, "Tolerances")."""
import math
import sys

import pytest
import torch

import oracle as O
from synthetic import direction, mode_amplitudes

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _nsc():
    import paper_1908_00587_amd as nsc
    return nsc


def rel(a, b):
    a = a.detach().cpu()
    b = b.detach().cpu()
    return float((a - b).abs().max() / b.abs().max())


CASES = {
    "tiny": (0.5, 50.0, 0.0, 0.0, 1.0, 12, 4, 7, 2 * math.pi),
    "min9": (0.3, 20.0, -5.0, 0.0, 1.0, 9, 1, 1, 3.0),            # smallest grid
    "ragged": (0.6, 80.0, 10.0, 0.0, 1.0, 13, 5, 9, 4.0),          # radix 5, odd tiles
    "heated": (0.71, 100.0, 0.0, 1.0e4, 0.7, 16, 8, 15, 2 * math.pi),
    "iso32": (0.5, 50.0, 0.0, 0.0, 1.0, 32, 16, 31, 2 * math.pi),
}


def _rand_state(p, seed, amp=1e-2):
    """Basic state plus a random (non-solenoidal) Hermitian field."""
    return O.base_state(p) + amp * direction(p.F, p.N_r, p.M_theta, p.M_z, seed)


@pytest.mark.parametrize("case", list(CASES))
def test_nonlinear_fp64(case):
    _say("nonlinear", case)
    args = CASES[case]
    p = O.Params(*args)
    u = _rand_state(p, 11)
    ref, dtc = O.nonlinear(p, u)
    ctx = _nsc().Context(*args)
    out, c = ctx.nonlinear(u.cuda(), cfl=True)
    torch.cuda.synchronize()
    assert rel(out, ref) < TOL64
    assert abs(float(c.cpu()[0]) - dtc) <= 1e-14 * dtc


@pytest.mark.parametrize("case", list(CASES))
def test_radial_solve_fp64(case):
    _say("radial_solve", case)
    args = CASES[case]
    p = O.Params(*args)
    u = _rand_state(p, 21)
    Nn = 10 * direction(p.F, p.N_r, p.M_theta, p.M_z, 22)
    Nq = 10 * direction(p.F, p.N_r, p.M_theta, p.M_z, 23)
    dt, c = 1e-3, 0.5
    ref, pref = O.radial_solve(p, u, Nn, Nq, dt, c)
    ctx = _nsc().Context(*args)
    ctx.set_timestep(dt=dt, c=c)
    out, pres = ctx.radial_solve(u.cuda(), Nn.cuda(), Nq.cuda(), pressure=True)
    torch.cuda.synchronize()
    assert rel(out, ref) < TOL64
    assert rel(pres, pref) < 1e-10  # pressure: Neumann Poisson conditioning (~1e7..1e8)


@pytest.mark.parametrize("case", ["tiny", "heated", "iso32"])
def test_initial_state_and_energy(case):
    _say("initial_state", case)
    args = CASES[case]
    p = O.Params(*args)
    amps = mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-3, seed=5)
    ref = O.initial_state(p, amps)
    ctx = _nsc().Context(*args)
    u = ctx.initial_state(amps.cuda())
    torch.cuda.synchronize()
    assert rel(u, ref) < TOL64
    e = float(ctx.energy(u).cpu()[0])
    eref = float(O.energy(p, ref))
    assert abs(e - eref) <= 1e-11 * eref
    assert rel(ctx.grid(), O.radial_grid(p)) < 1e-15


@pytest.mark.parametrize("case,steps", [("tiny", 10), ("heated", 10), ("iso32", 100)])
def test_step_fp64(case, steps):
    """Per-step (local) error: every GPU step taken from the oracle's state
    matches the oracle's next state to 1e-12 per field; the trajectory
    (global) error after `steps` steps stays below 1e-10 per field (rounding
    differences of the two LU orderings accumulate, see the tolerance
    derivation)."""
    _say("step", case, steps)
    args = CASES[case]
    p = O.Params(*args)
    u0 = O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-3, seed=1000))
    dt = 1e-3
    states = [u0]
    for _ in range(steps):
        states.append(O.step(p, states[-1], dt)[0])
    ctx = _nsc().Context(*args)
    ctx.set_timestep(dt=dt)
    worst = [0.0] * p.F
    for n in range(steps):
        x = states[n].cuda()
        ctx.step(x, dt)
        x = x.cpu()
        for f in range(p.F):
            worst[f] = max(worst[f], rel(x[f], states[n + 1][f]))
    _say("  local per-step max rel err per field", worst)
    assert max(worst) < TOL64
    u = u0.cuda()
    for _ in range(steps):
        ctx.step(u, dt)
    torch.cuda.synchronize()
    glob = [rel(u[f], states[-1][f]) for f in range(p.F)]
    _say("  global rel err per field", glob)
    assert max(glob) < 1e-10


def test_dynamic_dt_matches_oracle():
    _say("dynamic dt heated")
    args = CASES["heated"]
    p = O.Params(*args)
    u0 = O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-3, seed=7))
    steps = 6
    ref, dts = O.run(p, u0, steps, dynamic=True, cfl=0.5, dt_max=1e-2)
    assert dts[0] < 1e-2  # the CFL bound, not dt_max, sets the step
    ctx = _nsc().Context(*args)
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


@pytest.mark.parametrize("case", ["heated", "ragged"])
def test_step_size_changes_refactorise(case):
    """Steps whose size changes back and forth (each change refactorises the
    Helmholtz operators and re-solves the velocity responses; the pressure
    responses are kept from set-up): every step from the oracle's state
    matches the oracle's step of that size."""
    _say("step-size changes", case)
    args = CASES[case]
    p = O.Params(*args)
    u0 = O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-3, seed=11))
    ctx = _nsc().Context(*args)
    ctx.set_timestep(dt=1e-3)
    x = u0
    for dt in (1e-3, 6e-4, 1.3e-3, 6e-4, 1e-3):
        ref = O.step(p, x, dt)[0]
        g = x.cuda()
        ctx.step(g, dt)
        g = g.cpu()
        for f in range(p.F):
            assert rel(g[f], ref[f]) < TOL64, (dt, f)
        x = ref


@pytest.mark.parametrize("case", ["tiny", "ragged", "heated", "iso32"])
def test_nonlinear_mixed(case):
    """FP32 transforms/products: error relative to the largest entry of N."""
    _say("nonlinear mixed", case)
    args = CASES[case]
    p = O.Params(*args)
    u = _rand_state(p, 61)
    ref, dtc = O.nonlinear(p, u)
    ctx = _nsc().Context(*args)
    ctx.set_precision("mixed")
    out, c = ctx.nonlinear(u.cuda(), cfl=True)
    torch.cuda.synchronize()
    assert rel(out, ref) < 2e-6
    assert abs(float(c.cpu()[0]) - dtc) <= 1e-6 * dtc


@pytest.mark.parametrize("case,steps", [("heated", 20), ("iso32", 50)])
def test_step_mixed_error_stated(case, steps):
    """Mixed-precision stepping stays within 1e-5 of the FP64 oracle per field."""
    _say("step mixed", case, steps)
    args = CASES[case]
    p = O.Params(*args)
    u0 = O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-3, seed=1000))
    dt = 1e-3
    ref, _ = O.run(p, u0, steps, dt0=dt)
    ctx = _nsc().Context(*args)
    ctx.set_precision("mixed")
    ctx.set_timestep(dt=dt)
    u = u0.cuda()
    for _ in range(steps):
        ctx.step(u, dt)
    torch.cuda.synchronize()
    for f in range(p.F):
        err = rel(u[f], ref[f])
        _say(f"  field {f}: mixed rel err {err:.2e}")
        assert err < 1e-5, f
