"""Pins of the pipe-flow oracle (oracle/pipe.py) against what the
mathematics fixes: exactness of the parity-folded stencils on polynomials of
that parity, Hagen--Poiseuille flow as an exact steady state, the diffusion
of a pressure-free azimuthal mode against the Bessel-function eigenvalues of
the disk, the wall divergence removed by the influence correction, and the
mean-flow split of the nonlinear term against its plain definition."""
import math

import pytest
import torch
from scipy.special import jn_zeros

from oracle import pipe as P
from synthetic import direction, mode_amplitudes


def _params(N_r=16, M_theta=4, M_z=7, Re=100.0, L_z=2 * math.pi):
    return P.PipeParams(Re, N_r, M_theta, M_z, L_z)


@pytest.mark.parametrize("par", [1, -1])
def test_folded_stencils_exact_on_polynomials_of_their_parity(par):
    """The folded nine-point rows act on the restriction of an even (odd)
    polynomial as the unfolded rows act on the polynomial on the extended
    grid, which they differentiate exactly up to degree 8."""
    p = _params(N_r=20)
    r = P.radial_grid(p)
    D1, D2 = P.fd_matrices(p, par, r)
    for n in range(0 if par == 1 else 1, 9, 2):
        f = r ** n
        d1 = n * r ** (n - 1) if n >= 1 else torch.zeros_like(r)
        d2 = n * (n - 1) * r ** (n - 2) if n >= 2 else torch.zeros_like(r)
        assert float((D1 @ f - d1).abs().max()) <= 1e-9 * max(1.0, float(d1.abs().max())), n
        assert float((D2 @ f - d2).abs().max()) <= 1e-7 * max(1.0, float(d2.abs().max())), n


def test_folded_stencils_wrong_parity_is_not_exact():
    """Control: the even-parity rows do not differentiate r (odd) near the
    axis -- the fold sign matters."""
    p = _params(N_r=20)
    r = P.radial_grid(p)
    D1e, _ = P.fd_matrices(p, 1, r)
    assert float((D1e @ r - 1.0)[:4].abs().max()) > 1e-2


def test_grid_and_spacing():
    p = _params(N_r=12)
    r = P.radial_grid(p)
    assert abs(float(r[-1]) - 1.0) < 1e-15 and float(r[0]) > 0.0
    assert bool((r[1:] > r[:-1]).all())
    # nearest point of the extended grid for r_0 includes its mirror image
    dr = P._spacings(r)
    assert abs(float(dr[0]) - min(float(r[1] - r[0]), 2 * float(r[0]))) < 1e-16


def test_hagen_poiseuille_is_an_exact_steady_state():
    """u_z = Re (1 - r^2): L_0 u_z = -4 Re is exact for the even folded
    stencils, the driving 4 Re balances it, and the only nonlinear term,
    N_r = W W' in mode (0,0), is carried by the pressure (u_r = 0 there)."""
    p = _params(N_r=16, Re=250.0)
    u0 = P.base_state(p)
    u1, _ = P.step(p, u0, 1e-3)
    assert float((u1 - u0).abs().max()) <= 1e-12 * p.Re
    N, _ = P.nonlinear(p, u0)
    r = P.radial_grid(p)
    ref = -2.0 * p.Re ** 2 * r * (1.0 - r * r)
    assert float((N[0, :, 0, p.K].real - ref).abs().max()) <= 1e-12 * p.Re ** 2
    N[0, :, 0, p.K] = 0
    assert float(N.abs().max()) <= 1e-12 * p.Re ** 2


def test_pressure_free_mode_diffuses_with_the_disk_eigenvalues():
    """No mean flow (Re = 0), an axisymmetric azimuthal velocity in mode
    (0, k): neither the pressure nor the influence correction reaches it,
    so the implicit stage (no nonlinear term) multiplies its eigencomponents by
    (1 + (1-c) dt s) / (1 - c dt s), s the eigenvalues of L_1 (odd parity)
    with u = 0 at the wall; and s converges to -(j_{1,n}^2 + kappa^2)."""
    p = _params(N_r=24, M_theta=2, M_z=5, Re=0.0)
    ops = P._Ops(p)
    kk = p.K + 1
    kap = p.kz
    L = P.l_operator(ops, 1, kap)
    Li = L[:-1, :-1]  # interior rows and columns (wall value zero)
    s, V = torch.linalg.eig(Li)
    u = torch.zeros(p.shape(), dtype=torch.complex128)
    prof = V[:, 0]
    u[1, :-1, 0, kk] = prof
    u[1, :-1, 0, 2 * p.K - kk] = prof.conj()
    dt, c = 1e-3, 0.5
    zero = torch.zeros_like(u)
    un, _ = P.radial_solve(p, u, zero, zero, dt, c, ops=ops)  # the linear part of a step
    g = (1 + (1 - c) * dt * s[0]) / (1 - c * dt * s[0])
    err = (un[1, :-1, 0, kk] - g * prof).abs().max() / prof.abs().max()
    assert float(err) <= 1e-12
    # eigenvalues against the Bessel zeros (continuum): error falls fast with N_r
    errs = []
    for n in (16, 32):
        pp = _params(N_r=n, M_theta=2, M_z=5, Re=0.0)
        o = P._Ops(pp)
        ev = torch.linalg.eigvals(P.l_operator(o, 1, kap)[:-1, :-1]).real.sort(descending=True).values
        exact = -(torch.tensor(jn_zeros(1, 3), dtype=torch.float64) ** 2 + kap * kap)
        errs.append(float(((ev[:3] - exact) / exact).abs().max()))
    assert errs[1] <= 1e-6 and errs[1] < errs[0] / 50, errs


def _div(p, ops, u, m, kk):
    r = ops.r
    D1v = ops.d1(P.parity(m + 1)).to(torch.complex128)
    kap = (kk - p.K) * p.kz
    ur, ut, uz = u[0, :, m, kk], u[1, :, m, kk], u[2, :, m, kk]
    return D1v @ ur + ur / r + 1j * m * ut / r + 1j * kap * uz, float((D1v @ ur).abs().max())


def test_solve_removes_the_wall_divergence():
    """After the implicit stage with the 1 x 1 influence correction the
    divergence at the wall vanishes, for any right sides."""
    p = _params(N_r=20, M_theta=3, M_z=5)
    ops = P._Ops(p)
    sh = p.shape()
    X = P.base_state(p) + 1e-2 * direction(*sh, seed=71)
    Nn = direction(*sh, seed=72)
    Nq = direction(*sh, seed=73)
    out, _ = P.radial_solve(p, X, Nn, Nq, 1e-3, ops=ops)
    worst_wall, scale = 0.0, 0.0
    for m in range(p.M_theta):
        for kk in range(p.M_z):
            dv, sc = _div(p, ops, out, m, kk)
            worst_wall = max(worst_wall, float(dv[-1].abs()))
            scale = max(scale, sc)
    assert worst_wall <= 1e-11 * scale


def test_mean_split_equals_plain_definition():
    """The nonlinear term with the mean flow split off equals the plain
    definition, measured on the modes other than (0,0) at their own scale."""
    p = _params(N_r=12, M_theta=4, M_z=7, Re=300.0)
    u = P.base_state(p) + 1e-1 * direction(*p.shape(), seed=74)
    ops = P._Ops(p)
    rows = torch.arange(p.N_r)
    a, _ = P.nonlinear_planes(p, u, rows, ops)
    b = P.nonlinear_planes_direct(p, u, rows, ops)
    d = (a - b).clone()
    bb = b.clone()
    d[:, :, 0, p.K] = 0
    bb[:, :, 0, p.K] = 0
    assert float(d.abs().max()) <= 1e-12 * float(bb.abs().max())
    assert float((a - b)[:, :, 0, p.K].abs().max()) <= 1e-12 * float(b.abs().max())


def test_initial_state_is_projected():
    """Seeded smooth perturbation, projected by one Stokes stage: zero wall
    velocity and wall divergence, and an interior divergence that falls at
    the order of the finite differences as N_r doubles (the projection makes
    the field solenoidal up to the commutation error of the discrete
    operators); Hagen--Poiseuille underneath."""
    amps = mode_amplitudes(3, 4, 7, 1e-3, seed=5)
    rel = []
    for n in (16, 32):
        p = _params(N_r=n, M_theta=4, M_z=7, Re=100.0)
        ops = P._Ops(p)
        u = P.initial_state(p, amps)
        assert float(u[:, -1].abs().max()) <= 1e-14 * p.Re
        pert = u - P.base_state(p)
        assert float(pert.abs().max()) > 1e-6
        worst, scale = 0.0, 0.0
        for m in range(p.M_theta):
            for kk in range(p.M_z):
                dv, sc = _div(p, ops, pert, m, kk)
                assert float(dv[-1].abs()) <= 1e-12 * max(sc, 1e-300) + 1e-18
                worst = max(worst, float(dv.abs().max()))
                scale = max(scale, sc)
        rel.append(worst / scale)
    assert rel[1] < 1e-4 and rel[1] < rel[0] / 30, rel
