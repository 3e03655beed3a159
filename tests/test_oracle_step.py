"""Pins for the oracle's predictor--corrector step, dynamic time step, basic
state, initial condition and energy (sections 2.1 and 3).  CPU only."""
import math

import pytest
import torch

import oracle as O
from synthetic import mode_amplitudes

C = torch.complex128


def _discrete_couette(p, r, D1, D2):
    """Discrete steady (0,0) azimuthal flow: L_1 V = 0 inside, wall speeds."""
    L1 = D2 + D1 / r[:, None] - torch.diag(1.0 / r ** 2)
    A = L1.clone()
    A[0] = 0
    A[-1] = 0
    A[0, 0] = 1
    A[-1, -1] = 1
    b = torch.zeros(p.N_r, dtype=torch.float64)
    b[0] = p.Re_i
    b[-1] = p.Re_o
    return torch.linalg.solve(A, b)


def test_rigid_rotation_is_exactly_steady():
    p = O.Params(0.5, 50.0, 100.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    u = O.base_state(p)
    out, _ = O.run(p, u, 5, dt0=1e-3)
    assert float((out - u).abs().max()) < 1e-12 * 100.0


def test_discrete_couette_is_steady_and_close_to_analytic():
    p = O.Params(0.5, 50.0, -20.0, 0.0, 1.0, 24, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    V = _discrete_couette(p, r, D1, D2)
    ref = p.A * r + p.B / r
    assert float((V - ref).abs().max()) < 1e-7 * 50.0
    u = torch.zeros(p.shape(), dtype=C)
    u[1, :, 0, p.K] = V.to(C)
    out, _ = O.run(p, u, 10, dt0=1e-3)
    assert float((out - u).abs().max()) < 1e-12 * 50.0


def test_conduction_profile_is_steady():
    """Heated basic state: with Couette flow and the discrete conduction
    profile, T stays put (u . grad T = 0); the buoyancy drives u_z^00 only."""
    p = O.Params(0.5, 50.0, 0.0, 2.0e3, 1.0, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    L0 = D2 + D1 / r[:, None]
    A = L0.clone()
    A[0] = 0
    A[-1] = 0
    A[0, 0] = 1
    A[-1, -1] = 1
    b = torch.zeros(p.N_r, dtype=torch.float64)
    b[0], b[-1] = 0.5, -0.5
    Td = torch.linalg.solve(A, b)
    Tc = 0.5 + torch.log(r / p.r_i) / math.log(p.eta)
    assert float((Td - Tc).abs().max()) < 3e-8  # FD truncation at N_r = 16
    u = torch.zeros(p.shape(), dtype=C)
    u[1, :, 0, p.K] = _discrete_couette(p, r, D1, D2).to(C)
    u[3, :, 0, p.K] = Td.to(C)
    out, _ = O.run(p, u, 5, dt0=1e-3)
    assert float((out[3] - u[3]).abs().max()) < 1e-13
    assert float(out[2, :, 0, p.K].abs().max()) > 0.0  # buoyant axial flow develops
    assert float(out[2, [0, -1], 0, p.K].abs().max()) == 0.0


def test_initial_state_is_solenoidal_at_walls():
    p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, 24, 4, 7, 2 * math.pi)
    amps = mode_amplitudes(p.F, p.M_theta, p.M_z, 1.0e-3, seed=11)
    u = O.initial_state(p, amps)
    up = u - O.base_state(p)
    assert float(up[:, [0, -1]].abs().max()) == 0.0
    r = O.radial_grid(p)
    D1, _ = O.fd_matrices(p, r)
    m = torch.arange(p.M_theta, dtype=torch.float64)[None, :, None]
    kap = ((torch.arange(p.M_z, dtype=torch.float64) - p.K) * p.kz)[None, None, :]
    rr = r[:, None, None]
    d1 = torch.einsum('ij,jmk->imk', D1.to(C), up[0])
    div = d1 + up[0] / rr + 1j * m / rr * up[1] + 1j * kap * up[2]
    scale = float(d1.abs().max())
    assert float(div[[0, -1]].abs().max()) < 1e-11 * scale
    assert float(div.abs().max()) < 1e-3 * scale  # interior: truncation level


def test_interior_divergence_converges():
    vals = []
    for n in (16, 24, 32):
        p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, n, 4, 7, 2 * math.pi)
        amps = mode_amplitudes(p.F, p.M_theta, p.M_z, 1.0e-3, seed=11)
        up = O.initial_state(p, amps) - O.base_state(p)
        r = O.radial_grid(p)
        D1, _ = O.fd_matrices(p, r)
        m = torch.arange(p.M_theta, dtype=torch.float64)[None, :, None]
        kap = ((torch.arange(p.M_z, dtype=torch.float64) - p.K) * p.kz)[None, None, :]
        rr = r[:, None, None]
        d1 = torch.einsum('ij,jmk->imk', D1.to(C), up[0])
        div = d1 + up[0] / rr + 1j * m / rr * up[1] + 1j * kap * up[2]
        vals.append(float(div.abs().max()) / float(d1.abs().max()))
    assert vals[0] > vals[1] > vals[2]
    assert math.log(vals[0] / vals[2]) / math.log(2.0) > 5.0


def test_energy_matches_physical_quadrature():
    """E by Parseval equals 1/2 int |u'|^2 r dr dtheta dz evaluated on the
    padded grid (exact for the band-limited |u'|^2) with Clenshaw--Curtis in r."""
    p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, 12, 4, 7, 3.0)
    amps = mode_amplitudes(p.F, p.M_theta, p.M_z, 1.0e-2, seed=3)
    u = O.initial_state(p, amps)
    r = O.radial_grid(p)
    w = O.cc_weights(p, r)
    up = u - O.base_state(p, r)
    phys = O.to_physical(p, up)  # [3][N_r][N_th][N_z]
    mean_sq = (phys ** 2).sum(dim=0).mean(dim=(1, 2))
    ref = 0.5 * (2 * math.pi * p.L_z) * float((w * r * mean_sq).sum())
    e = float(O.energy(p, u))
    assert abs(e - ref) < 1e-13 * ref


def test_time_order_two():
    """Predictor + one corrector with c = 1/2: halving dt divides the error at a
    fixed time by 4 (reference from an 8x finer step).  The start state is
    first smoothed by backward-Euler stages (c = 1), which damp the stiff
    radial components that Crank--Nicolson-type stages leave undamped, and
    N_r = 24 keeps the spatial truncation level far below the time error."""
    p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, 24, 4, 7, 2 * math.pi)
    amps = mode_amplitudes(p.F, p.M_theta, p.M_z, 0.5, seed=5)
    u0, _ = O.run(p, O.initial_state(p, amps), 4, dt0=2e-3, c=1.0)
    T = 0.032
    ref, _ = O.run(p, u0, 256, dt0=T / 256)
    errs = []
    for nsteps in (8, 16, 32):
        out, _ = O.run(p, u0, nsteps, dt0=T / nsteps)
        errs.append(float((out - ref).abs().max()))
    o1 = math.log2(errs[0] / errs[1])
    o2 = math.log2(errs[1] / errs[2])
    assert 1.9 < o1 < 2.1 and 1.9 < o2 < 2.1, (errs, o1, o2)


def test_next_dt_rule():
    assert O.next_dt(1e-3, 1.0, cfl=0.5, dt_max=1e-3) == 1e-3          # capped, kept
    assert O.next_dt(1e-3, 1e-3, cfl=0.5, dt_max=1e-3) == 0.9 * 5e-4   # shrink with margin
    assert O.next_dt(5e-4, 1.1e-3, cfl=0.5, dt_max=1e-3) == 5e-4       # +10 %: keep
    assert O.next_dt(5e-4, 1.3e-3, cfl=0.5, dt_max=1e-3) == 0.9 * 6.5e-4  # +30 %: grow
    assert O.next_dt(5e-4, 1.0, cfl=0.5, dt_max=1e-3) == 1e-3
    # a slowly falling bound changes dt only once per ~20 % drop
    dt, changes = 5e-4, 0
    for n in range(100):
        b = 1.2e-3 * (1 - 0.003 * n)
        nd = O.next_dt(dt, b, cfl=0.5, dt_max=1e-3)
        changes += nd != dt
        dt = nd
        assert dt <= 0.5 * b
    assert changes <= 3


@pytest.mark.slow
def test_subcritical_perturbation_decays():
    """Re_i = 50 at eta = 0.5 lies below the first instability: the
    perturbation energy decays monotonically once the transient has passed."""
    p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, 16, 8, 15, 2 * math.pi)
    amps = mode_amplitudes(p.F, p.M_theta, p.M_z, 1.0e-3, seed=1000)
    u = O.initial_state(p, amps)
    es = []
    O.run(p, u, 40, dt0=2e-3, callback=lambda n, x, dt: es.append(float(O.energy(p, x))))
    late = es[10:]
    assert all(b < a for a, b in zip(late, late[1:]))
    assert es[-1] < 0.9 * es[10]
