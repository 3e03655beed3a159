"""Pins for the oracle's per-mode implicit radial solve (linear terms per
Fourier mode, section 2.2; predictor--corrector stage, section 2.1).  CPU only."""
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.special
import torch

import oracle as O


def _rand(shape, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return scale * torch.complex(torch.randn(shape, generator=g, dtype=torch.float64),
                                 torch.randn(shape, generator=g, dtype=torch.float64))


def test_l_operator_manufactured():
    """L_q f = f'' + f'/r - q^2 f/r^2 - kappa^2 f on f = r sin(pi (r - r_i)),
    converging at FD order."""
    errs = []
    ns = (20, 28, 40)
    for n in ns:
        p = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, n, 4, 7, 2 * math.pi)
        r = O.radial_grid(p)
        D1, D2 = O.fd_matrices(p, r)
        q, kap = 3, 2.0
        L = O.l_operator(p, torch.tensor([q]), torch.tensor([kap]), D1, D2, r)[0]
        s = torch.sin(math.pi * (r - p.r_i))
        c = torch.cos(math.pi * (r - p.r_i))
        f = r * s
        f1 = s + math.pi * r * c
        f2 = 2 * math.pi * c - math.pi ** 2 * r * s
        exact = f2 + f1 / r - q * q * f / r ** 2 - kap * kap * f
        errs.append(float((L @ f - exact).abs().max()))
    for i in range(1, 3):
        assert math.log(errs[i - 1] / errs[i]) / math.log(ns[i] / ns[i - 1]) > 6.5


def _monolithic(p, m, k, f_p, f_m, f_z, dt, c, D1, D2, r):
    """Independent statement of the coupled per-mode system: unknowns
    (X+, X-, X_z, p); momentum rows inside, zero wall velocity, pressure
    Poisson rows inside, zero divergence at both walls."""
    n = p.N_r
    D1n, D2n, rn = D1.numpy(), D2.numpy(), r.numpy()
    kap = k * p.kz
    I = np.eye(n)

    def L(q):
        return D2n + D1n / rn[:, None] - np.diag(q * q / rn ** 2) - kap * kap * I

    R = np.diag(1.0 / rn)
    M = np.zeros((4 * n, 4 * n), dtype=np.complex128)
    rhs = np.zeros(4 * n, dtype=np.complex128)
    blocks = [(I / dt - c * L(m + 1), D1n - m * R, f_p),
              (I / dt - c * L(abs(m - 1)), D1n + m * R, f_m),
              (I / dt - c * L(m), 1j * kap * I, f_z)]
    for b, (H, G, f) in enumerate(blocks):
        sl = slice(b * n, (b + 1) * n)
        M[sl, sl] = H
        M[sl, 3 * n:] = G
        rhs[sl] = f
        for j in (0, n - 1):
            M[b * n + j, :] = 0
            M[b * n + j, b * n + j] = 1
            rhs[b * n + j] = 0
    Lm = L(m)
    fdiv = 0.5 * ((D1n @ f_p + (1 + m) / rn * f_p) + (D1n @ f_m + (1 - m) / rn * f_m)) + 1j * kap * f_z
    M[3 * n:, 3 * n:] = Lm
    rhs[3 * n:] = fdiv
    for w, j in enumerate((0, n - 1)):
        row = 3 * n + j
        M[row, :] = 0
        M[row, 0:n] = 0.5 * (D1n[j] + (1 + m) / rn[j] * I[j])
        M[row, n:2 * n] = 0.5 * (D1n[j] + (1 - m) / rn[j] * I[j])
        M[row, 2 * n:3 * n] = 1j * kap * I[j]
        rhs[row] = 0
    v = np.linalg.solve(M, rhs)
    return v[:n], v[n:2 * n], v[2 * n:3 * n], v[3 * n:]


@pytest.mark.parametrize("heated", [False, True])
def test_influence_matrix_equals_monolithic_solve(heated):
    """The influence-matrix decomposition (particular + two homogeneous
    responses) reproduces the monolithic coupled velocity--pressure solve."""
    p = O.Params(0.71, 100.0, 0.0, 1.0e3 if heated else 0.0, 0.7, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    modes = [(0, 1), (0, 5), (1, 3), (1, 4), (2, 0), (3, 6), (3, 3)]
    m = torch.tensor([a for a, _ in modes])
    kk = torch.tensor([b for _, b in modes])
    B = len(modes)
    Xn = _rand((p.F, p.N_r, B), 1)
    Nn = _rand((p.F, p.N_r, B), 2, 10.0)
    Nq = _rand((p.F, p.N_r, B), 3, 10.0)
    dt, c = 1e-3, 0.5
    X, P = O.radial_solve_modes(p, m, kk, Xn, Nn, Nq, dt, c, True, D1, D2, r)
    for b, (mm, kidx) in enumerate(modes):
        k = kidx - p.K
        kap = k * p.kz
        rn = r.numpy()
        L = lambda q: (D2 + D1 / r[:, None] - torch.diag(q * q / r ** 2) - kap * kap * torch.eye(p.N_r)).numpy()
        xp = (Xn[0, :, b] + 1j * Xn[1, :, b]).numpy()
        xm = (Xn[0, :, b] - 1j * Xn[1, :, b]).numpy()
        xz = Xn[2, :, b].numpy()
        np_ = (Nn[0, :, b] + 1j * Nn[1, :, b]).numpy(); nm_ = (Nn[0, :, b] - 1j * Nn[1, :, b]).numpy()
        qp_ = (Nq[0, :, b] + 1j * Nq[1, :, b]).numpy(); qm_ = (Nq[0, :, b] - 1j * Nq[1, :, b]).numpy()
        f_p = xp / dt + (1 - c) * L(mm + 1) @ xp + c * qp_ + (1 - c) * np_
        f_m = xm / dt + (1 - c) * L(abs(mm - 1)) @ xm + c * qm_ + (1 - c) * nm_
        f_z = xz / dt + (1 - c) * L(mm) @ xz + c * Nq[2, :, b].numpy() + (1 - c) * Nn[2, :, b].numpy()
        Xp, Xm, Xz, pp = _monolithic(p, mm, k, f_p, f_m, f_z, dt, c, D1, D2, r)
        ur = 0.5 * (Xp + Xm)
        ut = (Xp - Xm) / 2j
        scale = np.abs(np.concatenate([ur, ut, Xz])).max()
        assert np.abs(X[0, :, b].numpy() - ur).max() < 1e-10 * scale
        assert np.abs(X[1, :, b].numpy() - ut).max() < 1e-10 * scale
        assert np.abs(X[2, :, b].numpy() - Xz).max() < 1e-10 * scale
        assert np.abs(P[:, b].numpy() - pp).max() < 1e-9 * np.abs(pp).max()
        # wall velocity exactly zero, wall divergence zero
        assert np.abs(X[:3, [0, -1], b].numpy()).max() == 0.0


def test_mode00_reading():
    """(0,0): u_r = 0; u_theta solves the L_1 Helmholtz problem with the wall
    speeds, u_z the L_0 problem with zero walls; the mean pressure head solves
    dp/dr = F_r in divergence form with p(r_i) = 0, so that for a smooth F_r
    it converges to the integral of F_r."""
    p = O.Params(0.5, 50.0, -10.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    Xn = _rand((3, 16, 1), 4).real.to(torch.complex128)
    Nn = _rand((3, 16, 1), 5).real.to(torch.complex128)
    Nq = _rand((3, 16, 1), 6).real.to(torch.complex128)
    dt, c = 1e-3, 0.5
    X, P = O.radial_solve_modes(p, torch.tensor([0]), torch.tensor([p.K]), Xn, Nn, Nq, dt, c, True, D1, D2, r)
    assert float(X[0].abs().max()) == 0.0
    L1 = (D2 + D1 / r[:, None] - torch.diag(1 / r ** 2)).to(torch.complex128)
    ut = X[1, :, 0]
    f = Xn[1, :, 0] / dt + (1 - c) * L1 @ Xn[1, :, 0] + c * Nq[1, :, 0] + (1 - c) * Nn[1, :, 0]
    res = ut / dt - c * L1 @ ut - f
    assert float(res[1:-1].abs().max()) < 1e-9 * float(f.abs().max())
    assert abs(complex(ut[0]) - 50.0) < 1e-13 and abs(complex(ut[-1]) + 10.0) < 1e-13
    assert abs(complex(P[0, 0])) < 1e-14
    # smooth radial force: p converges to the integral of F_r from r_i
    errs = []
    for n in (16, 24, 32):
        q = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, n, 4, 7, 2 * math.pi)
        rr = O.radial_grid(q)
        Fr = torch.cos(3 * rr).to(torch.complex128)[:, None]
        z = torch.zeros((3, n, 1), dtype=torch.complex128)
        Nn2 = z.clone()
        Nn2[0] = Fr
        _, P2 = O.radial_solve_modes(q, torch.tensor([0]), torch.tensor([q.K]), z, Nn2, Nn2, dt, c)
        exact = (torch.sin(3 * rr) - math.sin(3 * q.r_i)) / 3
        errs.append(float((P2[:, 0].real - exact).abs().max()))
    assert errs[2] < 1e-9 and errs[0] > errs[1] > errs[2]


def _bessel_roots(ri, ro, count):
    def cross(a):
        return (scipy.special.jv(1, a * ri) * scipy.special.yv(1, a * ro)
                - scipy.special.jv(1, a * ro) * scipy.special.yv(1, a * ri))
    xs = np.linspace(0.5, (count + 2) * math.pi / (ro - ri), 4000)
    vals = cross(xs)
    roots = []
    for i in range(len(xs) - 1):
        if vals[i] * vals[i + 1] < 0:
            roots.append(scipy.optimize.brentq(cross, xs[i], xs[i + 1], xtol=1e-15))
        if len(roots) == count:
            break
    return np.array(roots)


def test_l1_dirichlet_spectrum_converges_to_bessel():
    """Interior eigenvalues of L_1 with zero walls converge to -(alpha^2 +
    kappa^2), alpha the roots of J1(a r_i) Y1(a r_o) - J1(a r_o) Y1(a r_i)."""
    kap = 2.0
    errs = []
    for n in (24, 48):
        p = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, n, 4, 7, 2 * math.pi)
        r = O.radial_grid(p)
        D1, D2 = O.fd_matrices(p, r)
        L = O.l_operator(p, torch.tensor([1]), torch.tensor([kap]), D1, D2, r)[0].numpy()
        ev = np.sort(np.linalg.eigvals(L[1:-1, 1:-1]).real)[::-1][:3]
        exact = -(_bessel_roots(p.r_i, p.r_o, 3) ** 2 + kap * kap)
        errs.append(np.abs(ev - exact).max() / np.abs(exact).max())
    assert errs[1] < 2e-8
    assert math.log2(errs[0] / errs[1]) > 7.0


def test_pressure_free_mode_amplification():
    """Stokes decay of u_theta in the axisymmetric modes (0, +-k): no pressure
    and no influence correction reach u_theta, so each step multiplies the
    interior eigencomponents by (1 + (1-c) dt s)/(1 - c dt s), s in eig(L_1)."""
    p = O.Params(0.5, 0.0, 0.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    k = 2
    kap = k * p.kz
    g = 16.0 * (r - p.r_i) ** 2 * (p.r_o - r) ** 2
    amp = 1e-7 * (1.0 + 0.5j)
    u = torch.zeros(p.shape(), dtype=torch.complex128)
    u[1, :, 0, p.K + k] = amp * g
    u[1, :, 0, p.K - k] = np.conj(amp) * g
    dt, c, steps = 2e-3, 0.5, 5
    out, _ = O.run(p, u, steps, dt0=dt)
    L = O.l_operator(p, torch.tensor([1]), torch.tensor([kap]), D1, D2, r)[0].numpy()[1:-1, 1:-1]
    s, V = np.linalg.eig(L)
    amp_f = (1 + (1 - c) * dt * s) / (1 - c * dt * s)
    x0 = u[1, 1:-1, 0, p.K + k].numpy()
    pred = V @ (amp_f ** steps * np.linalg.solve(V, x0))
    got = out[1, 1:-1, 0, p.K + k].numpy()
    assert np.abs(got - pred).max() < 1e-11 * np.abs(pred).max()
