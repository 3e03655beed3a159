"""Pins for the oracle's nonlinear term (rotational form u x omega,
-u . grad T, Boussinesq buoyancy; sections 2.1 and 3).  CPU only."""
import math

import torch

import oracle as O
from synthetic import direction


def test_rigid_rotation_centripetal_term_exact():
    """Rigid rotation u_theta = A r (Re_o/r_o = Re_i/r_i, so B = 0): omega_z = 2A
    exactly (D1 is exact on linear functions) and N_r = 2 A^2 r, nothing else."""
    p = O.Params(0.5, 50.0, 100.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    assert abs(p.B) < 1e-12
    r = O.radial_grid(p)
    u = O.base_state(p, r)
    N, _ = O.nonlinear(p, u)
    ref = 2 * p.A * p.A * r
    assert float((N[0, :, 0, p.K].real - ref).abs().max()) < 1e-12 * float(ref.abs().max())
    N[0, :, 0, p.K] = 0
    assert float(N.abs().max()) < 1e-10


def test_couette_centripetal_term_converges():
    """Circular Couette flow: N_r^00 = u_theta omega_z = 2 A (A r + B/r), to FD
    truncation, converging with N_r."""
    errs = []
    for n in (16, 24, 32):
        p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, n, 4, 7, 2 * math.pi)
        r = O.radial_grid(p)
        N, _ = O.nonlinear(p, O.base_state(p, r))
        ref = 2 * p.A * (p.A * r + p.B / r)
        errs.append(float((N[0, :, 0, p.K].real - ref).abs().max()))
    assert errs[0] > errs[1] > errs[2]
    assert math.log(errs[1] / errs[2]) / math.log(32 / 24) > 6.0


def test_heated_base_state_terms():
    """Conduction profile with Couette flow: u . grad T = 0 exactly
    (axisymmetric, z-independent, u_r = 0) and N_z = Gr T in mode (0,0)."""
    p = O.Params(0.5, 50.0, 0.0, 1.0e4, 0.7, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    u = O.base_state(p, r)
    N, _ = O.nonlinear(p, u)
    assert float(N[3].abs().max()) < 1e-12
    ref = p.Gr * u[3, :, 0, p.K]
    assert float((N[2, :, 0, p.K] - ref).abs().max()) < 1e-9 * p.Gr


def test_curl_of_gradient_vanishes_in_r_and_theta():
    """u = grad phi: omega_r and omega_theta vanish identically (the theta and
    z derivatives are exact, D1 commutes with i kappa); omega_z is only
    truncation-level."""
    p = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, _ = O.fd_matrices(p, r)
    g = torch.Generator().manual_seed(7)
    phi = torch.complex(torch.randn(16, 4, 7, generator=g, dtype=torch.float64),
                        torch.randn(16, 4, 7, generator=g, dtype=torch.float64))
    m = torch.arange(4, dtype=torch.float64)[None, :, None]
    kap = ((torch.arange(7, dtype=torch.float64) - p.K) * p.kz)[None, None, :]
    rr = r[:, None, None]
    u = torch.stack([torch.einsum('ij,jmk->imk', D1.to(torch.complex128), phi),
                     1j * m / rr * phi, 1j * kap * phi])
    d = O.derived_fields(p, u, D1, r)
    assert float(d[3].abs().max()) < 1e-12 * float(u.abs().max())
    assert float(d[4].abs().max()) < 1e-12 * float(u.abs().max())


def test_cfl_bound_couette():
    """dt_cfl for u = (0, V(r), 0) is min_j r_j dtheta / |V(r_j)| (u_r = u_z = 0)."""
    p = O.Params(0.5, 50.0, -20.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    _, dt = O.nonlinear(p, O.base_state(p, r))
    V = (p.A * r + p.B / r).abs()
    ok = V > 0
    ref = float((r[ok] * (2 * math.pi / p.N_theta) / V[ok]).min())
    assert abs(dt - ref) < 1e-14 * ref


def test_nonlinear_planes_consistent_with_full():
    """The per-plane evaluation (used for sampled checks on large grids) equals
    the full evaluation."""
    p = O.Params(0.5, 50.0, 0.0, 1.0e3, 1.0, 12, 4, 7, 2 * math.pi)
    g = torch.Generator().manual_seed(8)
    u = O.base_state(p) + 1e-2 * O.herm(p, torch.complex(
        torch.randn(p.shape(), generator=g, dtype=torch.float64),
        torch.randn(p.shape(), generator=g, dtype=torch.float64)))
    N, _ = O.nonlinear(p, u)
    Np, _ = O.nonlinear_planes(p, u, [0, 5, 11])
    assert float((O.herm(p, Np) - N[:, [0, 5, 11]]).abs().max()) < 1e-12 * float(N.abs().max())


def test_split_equals_direct_definition():
    """The basic-state split is exact algebra: it reproduces the plain
    transform-everything definition to rounding."""
    for Ra in (0.0, 2.0e3):
        p = O.Params(0.6, 80.0, -20.0, Ra, 0.7, 14, 5, 9, 3.0)
        u = O.base_state(p) + 1e-2 * direction(p.F, p.N_r, p.M_theta, p.M_z, 71)
        rows = torch.arange(p.N_r)
        Ns, _ = O.nonlinear_planes(p, u, rows)
        Nd = O.nonlinear_planes_direct(p, u, rows)
        assert float((Ns - Nd).abs().max()) < 1e-12 * float(Nd.abs().max())


def test_split_rounding_scales_with_the_perturbation():
    """For u = U_b +- eps d the central difference isolates the linear
    response exactly (N is quadratic); with the split its value does not
    depend on eps down to eps = 1e-8, i.e. the rounding error is relative to
    the perturbation, not to the O(Re^2) basic-state term."""
    p = O.Params(0.71, 2000.0, -1000.0, 0.0, 1.0, 16, 6, 11, 2 * math.pi)
    ub = O.base_state(p)
    d = direction(p.F, p.N_r, p.M_theta, p.M_z, 72)
    d[:, :, 0, p.K] = 0  # so that (U_b + eps d) - U_b = eps d exactly
    rows = torch.arange(p.N_r)

    def lin(eps):
        a, _ = O.nonlinear_planes(p, ub + eps * d, rows)
        b, _ = O.nonlinear_planes(p, ub - eps * d, rows)
        return (a - b) / (2 * eps)

    ref = lin(1e-2)
    got = lin(1e-8)
    assert float((got - ref).abs().max()) < 1e-13 * float(ref.abs().max())
