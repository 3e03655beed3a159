"""Further pins for the oracle's nonlinear term, temperature equation and
time-step bound (sections 2.1 and 3).  CPU only.

Each test is built so that the identity it checks holds exactly (to
rounding) for the fields chosen, and so that a wrong sign, a dropped term or
a wrong factor in the part it targets breaks it by O(1):
  * vector-calculus identities on fields whose radial profiles are
    polynomials of degree <= 8, on which the nine-point D1 is exact
    (curl grad = 0 in all three components, div curl = 0);
  * the theta and z components of grad T against a physical-space
    difference quotient of the Fourier series itself;
  * a scalar carried by solid-body rotation, where -u . grad T is
    -Omega dT/dtheta;
  * the temperature diffusivity 1/Pr through the per-step amplification of
    a pure-diffusion mode (u = 0);
  * the CFL bound for flows with a single velocity component;
  * the mean-flow split of the products at the scale of the fluctuations.
"""
import math

import numpy as np
import torch

import oracle as O
from synthetic import direction

C = torch.complex128


def _poly_profiles(r, nf, M_theta, M_z, deg, seed):
    """[nf][N_r][M_theta][M_z] complex fields whose every mode is a random
    polynomial in r of degree `deg` (coefficients complex normal)."""
    g = torch.Generator().manual_seed(seed)
    co = torch.complex(torch.randn(nf, deg + 1, M_theta, M_z, generator=g, dtype=torch.float64),
                       torch.randn(nf, deg + 1, M_theta, M_z, generator=g, dtype=torch.float64))
    x = (r - r.mean())[:, None, None]  # centred, so the monomials stay O(1)
    out = torch.zeros(nf, r.numel(), M_theta, M_z, dtype=C)
    for d in range(deg + 1):
        out = out + co[:, d][:, None] * (x ** d)[None]
    return out


def _mk(p):
    m = torch.arange(p.M_theta, dtype=torch.float64)[None, :, None]
    kap = ((torch.arange(p.M_z, dtype=torch.float64) - p.K) * p.kz)[None, None, :]
    return m, kap


def test_curl_of_polynomial_gradient_vanishes_in_every_component():
    """u = grad phi with phi = r q(r) e^{i(m theta + k z)}, deg(r q) = 8: then
    u_r = D1 phi, u_theta = i m q and u_z = i kappa phi, and every D1 that the
    curl applies acts on a polynomial of degree <= 8, so omega_r, omega_theta
    and omega_z vanish to rounding (omega_z = i m [q' + q/r - (q + r q')/r])."""
    p = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, _ = O.fd_matrices(p, r)
    q = _poly_profiles(r, 1, p.M_theta, p.M_z, 7, seed=21)[0]
    rr = r[:, None, None]
    phi = rr * q
    m, kap = _mk(p)
    u = torch.stack([torch.einsum('ij,jmk->imk', D1.to(C), phi), 1j * m * q, 1j * kap * phi])
    d = O.derived_fields(p, u, D1, r)
    scale = float(u.abs().max())
    for comp in (3, 4, 5):
        assert float(d[comp].abs().max()) < 1e-11 * scale, comp


def test_divergence_of_curl_vanishes():
    """div(curl u) = 0 for any u.  With u_r = a(r), u_theta = b(r) and
    u_z = r c(r) (deg a, deg b, deg(r c) <= 8 per mode), omega_r =
    i m c - i kappa b is a polynomial too, so every radial derivative below
    is exact and div omega = D1 omega_r + omega_r/r + (i m/r) omega_theta +
    i kappa omega_z vanishes to rounding."""
    for eta, Lz in ((0.5, 2 * math.pi), (0.71, 3.0)):
        p = O.Params(eta, 0.0, 0.0, 0.0, 1.0, 18, 5, 9, Lz)
        r = O.radial_grid(p)
        D1, _ = O.fd_matrices(p, r)
        a, b, c = _poly_profiles(r, 3, p.M_theta, p.M_z, 8, seed=22)
        c = _poly_profiles(r, 1, p.M_theta, p.M_z, 7, seed=23)[0]
        rr = r[:, None, None]
        u = torch.stack([a, b, rr * c])
        w = O.derived_fields(p, u, D1, r)
        m, kap = _mk(p)
        wr, wt, wz = w[3], w[4], w[5]
        div = (torch.einsum('ij,jmk->imk', D1.to(C), wr) + wr / rr + 1j * m / rr * wt
               + 1j * kap * wz)
        scale = float((torch.einsum('ij,jmk->imk', D1.abs().to(C), wr.abs().to(C))).abs().max())
        assert float(div.abs().max()) < 1e-12 * scale


def _series(p, fhat, j, theta, z):
    """Value of the field fhat [N_r][M_theta][M_z] at (r_j, theta, z) by the
    Fourier sum sum_k f_0k e^{i k kz z} + 2 Re sum_{m>=1,k} f_mk e^{i(m theta +
    k kz z)}, at arbitrary theta and z."""
    m = torch.arange(p.M_theta, dtype=torch.float64)[:, None]
    k = (torch.arange(p.M_z, dtype=torch.float64) - p.K)[None, :]
    cm = torch.where(m == 0, 1.0, 2.0)
    return float((cm * fhat[j] * torch.exp(1j * (m * theta + k * p.kz * z))).real.sum())


def test_grad_t_angular_and_axial_components_are_difference_quotients():
    """(grad T)_theta = (1/r) dT/dtheta and (grad T)_z = dT/dz, checked against
    fourth-order central differences of the physical field itself (the Fourier
    series evaluated off the grid), so the sign convention of the spectral
    derivative is fixed by the field, not by the formula."""
    p = O.Params(0.5, 0.0, 0.0, 1.0e3, 0.7, 12, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, _ = O.fd_matrices(p, r)
    u = torch.zeros(p.shape(), dtype=C)
    u[3] = O.herm(p, direction(1, p.N_r, p.M_theta, p.M_z, 24)[0][None])[0]
    d = O.derived_fields(p, u, D1, r)
    h = 1e-3

    def quot(f):
        return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)

    pts = [(2, 0.3, 1.1), (5, 2.0, 4.0), (9, 4.4, 0.2)]
    for j, th, z in pts:
        gt = _series(p, d[7], j, th, z)
        gz = _series(p, d[8], j, th, z)
        ref_t = quot(lambda e: _series(p, u[3], j, th + e, z)) / float(r[j])
        ref_z = quot(lambda e: _series(p, u[3], j, th, z + e))
        sc = abs(ref_t) + abs(ref_z) + 1.0
        assert abs(gt - ref_t) < 1e-7 * sc, (j, gt, ref_t)
        assert abs(gz - ref_z) < 1e-7 * sc, (j, gz, ref_z)


def test_scalar_carried_by_solid_body_rotation():
    """u = (0, Omega r, 0): -u . grad T = -Omega dT/dtheta, i.e. every
    coefficient of N_T is -i m Omega T_mk (the pattern turns with the fluid),
    through the split evaluation and through the plain definition."""
    Om = 3.0
    r_i = 1.0  # eta = 0.5
    p = O.Params(0.5, Om * r_i, Om * 2 * r_i, 1.0e3, 0.7, 14, 5, 9, 2 * math.pi)
    assert abs(p.B) < 1e-12 and abs(p.A - Om) < 1e-12
    u = O.base_state(p)
    tp = 1e-2 * direction(1, p.N_r, p.M_theta, p.M_z, 25)[0]
    tp[:, 0, p.K] = 0.0
    u[3] = u[3] + tp
    m = torch.arange(p.M_theta, dtype=torch.float64)[None, :, None]
    ref = -1j * m * Om * tp
    N, _ = O.nonlinear(p, u)
    rows = torch.arange(p.N_r)
    Nd = O.herm(p, O.nonlinear_planes_direct(p, u, rows))
    scale = float(ref.abs().max())
    for NT in (N[3], Nd[3]):
        diff = NT - ref
        diff[:, 0, p.K] = 0.0  # mode (0,0): the conduction profile's own (zero) term
        assert float(diff.abs().max()) < 1e-11 * scale


def test_temperature_diffusivity_amplification():
    """u = 0 and a temperature perturbation in the axisymmetric modes (0, +-k):
    no advection (u stays O(Ra T) with Ra = 1e-12), so every step multiplies
    the interior eigencomponents by (1 + (1-c) dt s/Pr)/(1 - c dt s/Pr),
    s in eig(L_0) (zero walls) -- the thermal diffusivity is 1/Pr in viscous
    units."""
    p = O.Params(0.5, 0.0, 0.0, 1.0e-12, 0.7, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    k = 1
    kap = k * p.kz
    g = 16.0 * (r - p.r_i) ** 2 * (p.r_o - r) ** 2
    amp = 1e-7 * (0.8 - 0.6j)
    u = O.base_state(p, r)  # zero velocity, conduction profile
    u[3, :, 0, p.K + k] = amp * g
    u[3, :, 0, p.K - k] = np.conj(amp) * g
    dt, c, steps = 2e-3, 0.5, 5
    out, _ = O.run(p, u, steps, dt0=dt)
    L = O.l_operator(p, torch.tensor([0]), torch.tensor([kap]), D1, D2, r)[0].numpy()[1:-1, 1:-1]
    s, V = np.linalg.eig(L)
    amp_f = (1 + (1 - c) * dt * s / p.Pr) / (1 - c * dt * s / p.Pr)
    x0 = u[3, 1:-1, 0, p.K + k].numpy()
    pred = V @ (amp_f ** steps * np.linalg.solve(V, x0))
    got = out[3, 1:-1, 0, p.K + k].numpy()
    assert np.abs(got - pred).max() < 1e-10 * np.abs(pred).max()
    # the same with Pr = 1 would be a different sequence: the test can see 1/Pr
    amp_1 = (1 + (1 - c) * dt * s) / (1 - c * dt * s)
    other = V @ (amp_1 ** steps * np.linalg.solve(V, x0))
    assert np.abs(other - pred).max() > 1e-4 * np.abs(pred).max()


def test_cfl_bound_axial_flow_only():
    """u = (0, 0, w) uniform: dt_cfl = (L_z / N_z) / |w|."""
    p = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, 16, 4, 7, 3.0)
    u = torch.zeros(p.shape(), dtype=C)
    w = 2.5
    u[2, :, 0, p.K] = w
    _, dt = O.nonlinear(p, u)
    ref = (p.L_z / p.N_z) / w
    assert abs(dt - ref) < 1e-14 * ref


def test_cfl_bound_radial_flow_only():
    """u = (U(r), 0, 0) with U vanishing at the walls: dt_cfl is the smallest
    time in which a particle at a grid point r_j reaches the grid point nearest
    to it, min_j min_{i != j} |r_i - r_j| / |U(r_j)| (points with U = 0 put no
    bound)."""
    for n in (16, 21):
        p = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, n, 4, 7, 2 * math.pi)
        r = O.radial_grid(p)
        U = 4.0 * (r - p.r_i) * (p.r_o - r) + 0.1 * (r - p.r_i)
        u = torch.zeros(p.shape(), dtype=C)
        u[0, :, 0, p.K] = U.to(C)
        _, dt = O.nonlinear(p, u)
        dist = (r[:, None] - r[None, :]).abs() + torch.diag(torch.full((n,), math.inf,
                                                                       dtype=torch.float64))
        near = dist.min(dim=1).values
        ok = U.abs() > 0
        ref = float((near[ok] / U.abs()[ok]).min())
        assert abs(dt - ref) < 1e-14 * ref, (n, dt, ref)


def test_split_matches_direct_at_the_fluctuation_scale():
    """The mean-flow split equals the plain definition; away from mode (0,0)
    (where the O(Re^2) mean x mean term lives) the agreement is measured
    against the size of the fluctuation terms themselves."""
    for Ra in (0.0, 2.0e3):
        p = O.Params(0.6, 80.0, -20.0, Ra, 0.7, 14, 5, 9, 3.0)
        u = O.base_state(p) + 0.1 * direction(p.F, p.N_r, p.M_theta, p.M_z, 71)
        rows = torch.arange(p.N_r)
        Ns, _ = O.nonlinear_planes(p, u, rows)
        Nd = O.nonlinear_planes_direct(p, u, rows)
        for f in range(p.F):
            a, b = Ns[f].clone(), Nd[f].clone()
            assert float((a[:, 0, p.K] - b[:, 0, p.K]).abs().max()) < \
                1e-12 * float(b[:, 0, p.K].abs().max())
            a[:, 0, p.K] = 0.0
            b[:, 0, p.K] = 0.0
            assert float((a - b).abs().max()) < 2e-13 * float(b.abs().max()), f
