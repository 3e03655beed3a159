"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (wavefront-scope 192- and 768-point transforms, 16-line z
tiles, affine padded LDS addressing), against the FP64 oracle on sampled
outputs it can compute one by one: radial rows of the nonlinear term (the
transforms of a row are independent of the other rows) and single Fourier
modes of the implicit stage (the radial systems of a mode are independent of
the other modes).  The heated workload also takes one full step against the
oracle's full step."""
import math
import sys

import pytest
import torch

import oracle as O
from paper_1908_00587_amd.workloads import amplitudes, params
from synthetic import direction

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(name, prec="fp64"):
    import paper_1908_00587_amd as nsc
    ctx = nsc.Context(*params(name))
    ctx.set_precision(prec)
    return ctx


def rel(a, b):
    a = a.detach().cpu()
    b = b.detach().cpu()
    return float((a - b).abs().max() / b.abs().max())


def report(got, ref, p, tag):
    """Print and return the error of each output field of a nonlinear term,
    relative to the field and, over the modes other than (0,0) (the mean-flow
    products dominate max|N|), relative to N there."""
    names = ["N_r", "N_theta", "N_z", "N_T"][: got.shape[0]]
    fl = torch.ones(p.M_theta, p.M_z, dtype=torch.bool)
    fl[0, p.K] = False
    worst = 0.0
    for f, nm in enumerate(names):
        d = (got[f] - ref[f]).abs()
        e_all = float(d.max() / ref[f].abs().max())
        e_fl = float(d[:, fl].max() / ref[f][:, fl].abs().max())
        worst = max(worst, e_fl)
        _say(f"  {tag} {nm}: rel {e_all:.2e}, over the fluctuating modes {e_fl:.2e}")
    return worst


ROWS = {"tc-heated-n64": [0, 1, 9, 31, 54, 62, 63], "tc-turb-n128": [0, 5, 64, 127]}


@pytest.mark.parametrize("name", list(ROWS))
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", 2e-6)])
def test_nonlinear_full_size_sampled_rows(name, prec, tol):
    _say("nonlinear full size", name, prec)
    p = O.Params(*params(name))
    u = O.base_state(p) + 1e-2 * direction(p.F, p.N_r, p.M_theta, p.M_z, 81)
    rows = torch.tensor(ROWS[name])
    ref, dt_rows = O.nonlinear_planes(p, u, rows)
    ref = O.herm(p, ref)
    ctx = _ctx(name, prec)
    out, c = ctx.nonlinear(u.cuda(), cfl=True)
    torch.cuda.synchronize()
    got = out.cpu()[:, rows]
    assert rel(got, ref) < tol
    # per field: in mixed precision N_theta and N_T are small beside the
    # products that make them up, so their own relative error is larger
    # (measured up to 2e-5 on the counter-rotating grid); a sanity bound
    assert report(got, ref, p, f"{name} {prec}") < (tol if prec == "fp64" else 1e-4)
    # the bound over all rows is at most the bound over the sampled rows (up
    # to the rounding of the transformed velocities: FP32 in mixed precision)
    c = float(c.cpu()[0])
    assert 0.0 < c <= dt_rows * (1 + (1e-14 if prec == "fp64" else 1e-6))


MODES = {"tc-heated-n64": [(0, 63), (0, 10), (0, 116), (1, 63), (1, 0), (17, 80), (63, 126)],
         "tc-turb-n128": [(0, 255), (0, 3), (0, 507), (2, 255), (100, 400), (255, 0)],
         "heated-n63": [(0, 63), (0, 5), (1, 63), (5, 70), (63, 0)],
         "counter-n63": [(0, 63), (0, 120), (1, 63), (40, 70), (127, 0), (127, 126)]}
# 63 radial points, where the stencil kernels take several rows per lane with
# a short last chunk and one-sided windows in the top chunks: the heated
# workload's modes (right sides four rows, 63 = 15 x 4 + 3; divergence two;
# velocity right sides one) and counter-rotating cylinders on 128 x 127 modes
# (right sides and divergence four rows; velocity right sides two, 63 =
# 31 x 2 + 1)
ARGS = {"tc-heated-n64": params("tc-heated-n64"), "tc-turb-n128": params("tc-turb-n128"),
        "heated-n63": (0.71, 100.0, 0.0, 1.0e4, 0.7, 63, 64, 127, 2 * math.pi),
        "counter-n63": (0.71, 2000.0, -1000.0, 0.0, 1.0, 63, 128, 127, 2 * math.pi)}


@pytest.mark.parametrize("name", list(MODES))
def test_radial_solve_full_size_sampled_modes(name):
    """Two step sizes on one context: the second refactorises the Helmholtz
    operators and re-solves the velocity responses at full size."""
    _say("radial_solve full size", name)
    import paper_1908_00587_amd as nsc
    p = O.Params(*ARGS[name])
    u = O.base_state(p) + 1e-2 * direction(p.F, p.N_r, p.M_theta, p.M_z, 82)
    Nn = 10 * direction(p.F, p.N_r, p.M_theta, p.M_z, 83)
    Nq = 10 * direction(p.F, p.N_r, p.M_theta, p.M_z, 84)
    c = 0.5
    ctx = nsc.Context(*ARGS[name])
    ctx.set_precision("fp64")
    m = torch.tensor([a for a, _ in MODES[name]])
    kk = torch.tensor([b for _, b in MODES[name]])
    # the m = 0 column is Hermitian-averaged with its mirror (0, -k)
    mirror = torch.where(m == 0, p.M_z - 1 - kk, kk)
    zero = (m == 0)
    for dt in (1e-4, 3e-5):
        _say("  dt", dt)
        ctx.set_timestep(dt=dt, c=c)
        out, pres = ctx.radial_solve(u.cuda(), Nn.cuda(), Nq.cuda(), pressure=True)
        torch.cuda.synchronize()
        out, pres = out.cpu(), pres.cpu()
        X, P = O.radial_solve_modes(p, m, kk, u[:, :, m, kk], Nn[:, :, m, kk], Nq[:, :, m, kk],
                                    dt, c)
        Xm, Pm = O.radial_solve_modes(p, m, mirror, u[:, :, m, mirror], Nn[:, :, m, mirror],
                                      Nq[:, :, m, mirror], dt, c)
        X = torch.where(zero, 0.5 * (X + Xm.conj()), X)
        P = torch.where(zero, 0.5 * (P + Pm.conj()), P)
        assert rel(out[:, :, m, kk], X) < TOL64
        assert rel(pres[:, m, kk], P) < 1e-10


@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("mixed", 1e-5)])
def test_step_full_size_heated(prec, tol):
    """One predictor--corrector step of the heated workload from its initial
    state, the whole field against the oracle's step."""
    name = "tc-heated-n64"
    _say("step full size", name, prec)
    p = O.Params(*params(name))
    u0 = O.initial_state(p, amplitudes(name))
    dt = 2e-4
    ref, dtc = O.step(p, u0, dt)
    ctx = _ctx(name, prec)
    ctx.set_timestep(dt=dt)
    u = u0.cuda()
    ctx.step(u, dt)
    torch.cuda.synchronize()
    for f in range(p.F):
        assert rel(u[f], ref[f]) < tol, f


CONV = "tc-conv-n256"
CONV_ROWS = [0, 131, 255]
CONV_MODES = [(0, 511), (0, 10), (0, 1000), (1, 511), (100, 300), (511, 0), (511, 1022)]


def test_conv_full_size_sampled():
    """The largest workload on one GPU (N_r = 256, 512 x 1023 modes, padded
    1536 x 1536 planes; about 130 GiB of library buffers): sampled radial
    rows of the mixed-precision nonlinear term and sampled modes of the FP64
    implicit stage against the oracle.  The FP64 nonlinear term, whose theta
    line set does not fit one workgroup's LDS at this size, is refused."""
    import paper_1908_00587_amd as nsc
    _say("conv full size: inputs")
    p = O.Params(*params(CONV))
    u = O.base_state(p)
    u += 1e-2 * direction(p.F, p.N_r, p.M_theta, p.M_z, 91)
    ctx = _ctx(CONV, "mixed")
    ug = u.cuda()
    _say("conv full size: mixed nonlinear")
    out, c = ctx.nonlinear(ug, cfl=True)
    torch.cuda.synchronize()
    got = out[:, CONV_ROWS].cpu()
    c = float(c.cpu()[0])
    del out
    _say("conv full size: oracle rows")
    ref, dt_rows = O.nonlinear_planes(p, u, torch.tensor(CONV_ROWS))
    ref = O.herm(p, ref)
    err = rel(got, ref)
    _say("  mixed nonlinear rel err", err)
    assert err < 1e-5
    assert report(got, ref, p, f"{CONV} mixed") < 1e-4
    assert 0.0 < c <= dt_rows * (1 + 1e-6)
    ctx.set_precision("fp64")
    with pytest.raises(nsc.NscError):
        ctx.nonlinear(ug)
    _say("conv full size: FP64 radial solve")
    Nn = 10 * direction(p.F, p.N_r, p.M_theta, p.M_z, 92)
    Nq = 10 * direction(p.F, p.N_r, p.M_theta, p.M_z, 93)
    dt, cc = 2e-5, 0.5
    ctx.set_timestep(dt=dt, c=cc)
    xg, pg = ctx.radial_solve(ug, Nn.cuda(), Nq.cuda(), pressure=True)
    torch.cuda.synchronize()
    m = torch.tensor([a for a, _ in CONV_MODES])
    kk = torch.tensor([b for _, b in CONV_MODES])
    gx = xg[:, :, m.cuda(), kk.cuda()].cpu()
    gp = pg[:, m.cuda(), kk.cuda()].cpu()
    del xg, pg
    mirror = torch.where(m == 0, p.M_z - 1 - kk, kk)
    X, P = O.radial_solve_modes(p, m, kk, u[:, :, m, kk], Nn[:, :, m, kk], Nq[:, :, m, kk], dt, cc)
    Xm, Pm = O.radial_solve_modes(p, m, mirror, u[:, :, m, mirror], Nn[:, :, m, mirror],
                                  Nq[:, :, m, mirror], dt, cc)
    zero = (m == 0)
    X = torch.where(zero, 0.5 * (X + Xm.conj()), X)
    P = torch.where(zero, 0.5 * (P + Pm.conj()), P)
    assert rel(gx, X) < TOL64
    assert rel(gp, P) < 1e-10
