"""Plain FP64 statement of one time step of the pipe-flow variant (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Parity pinned by the
``-m "not gpu"`` tests in ``tests/test_oracle_pipe.py`` (closed forms,
library routines, invariants).

The paper ships a version of the method for flows in straight pipes that
keeps its numerical method and infrastructure (abstract; section 4,
"Impact"), with the pipe formulation of another code whose description is
not part of the paper.  Every pipe-specific formula below is therefore a
reading:

  * geometry and units: a pipe of radius 1, periodic in z with period L_z;
    time in R^2/nu, velocity in nu/R; the flow is driven by a constant mean
    pressure gradient -dP/dz = 4 Re, whose laminar (Hagen--Poiseuille)
    solution is u_z = Re (1 - r^2): Re is its centreline speed;
  * equations: du/dt = -grad P + lap u + u x omega + 4 Re e_z, div u = 0,
    u = 0 at r = 1 (rotational form, pressure = head, as for the cylinders);
  * radial grid: the N_r positive points of the 2 N_r Chebyshev--Gauss--
    Lobatto points of [-1, 1], r_j = cos(pi (N_r - 1 - j) / (2 N_r - 1)):
    clustered at the wall, r = 1 included, the axis not a grid point;
  * axis: a Fourier coefficient of azimuthal order m is the restriction of
    a function that is even in r for even m and odd for odd m (scalars and
    u_z), and of parity (-1)^(m+1) for u_r and u_theta (so for
    u_+- = u_r +- i u_theta, of order q = m +- 1, parity (-1)^q).  The
    nine-point stencils are taken on the grid extended by the mirror points
    -r_j, and the weights of mirror points are folded onto r_j with that
    parity: every radial operator of order q uses the parity (-1)^q;
  * pressure--velocity coupling: the cylinder method with one wall: a
    Neumann pressure problem, the Helmholtz solves with the wall value, and
    a 1 x 1 influence matrix so that div u = 0 at r = 1;
  * mode (0,0): u_r = 0 (r u_r is constant and vanishes on the axis),
    u_theta and u_z from their Helmholtz problems, u_z forced by 4 Re.
"""
import math

import torch

from .tc import fornberg, herm, to_physical, to_spectral, next_dt

F64 = torch.float64
C128 = torch.complex128


class PipeParams:
    """Pipe-flow problem: Re (centreline speed of the laminar flow driven by
    the imposed mean pressure gradient 4 Re), N_r radial points, M_theta
    azimuthal modes (m >= 0), M_z axial modes (odd), L_z the axial period."""

    def __init__(self, Re, N_r, M_theta, M_z, L_z):
        if N_r < 9:
            raise ValueError("N_r must be >= 9 (nine-point stencils)")
        if M_z < 1 or M_z % 2 == 0:
            raise ValueError("M_z must be odd")
        if M_theta < 1 or L_z <= 0.0:
            raise ValueError("M_theta >= 1 and L_z > 0 required")
        self.Re = float(Re)
        self.N_r, self.M_theta, self.M_z, self.L_z = int(N_r), int(M_theta), int(M_z), float(L_z)
        self.K = (self.M_z - 1) // 2
        self.N_theta = 3 * self.M_theta
        self.N_z = 3 * (self.K + 1)
        self.kz = 2.0 * math.pi / self.L_z
        self.F = 3
        self.heated = False
        self.G = 4.0 * self.Re  # imposed mean pressure gradient -dP/dz

    def shape(self):
        return (self.F, self.N_r, self.M_theta, self.M_z)


def radial_grid(p):
    """r_j = cos(pi (N_r - 1 - j) / (2 N_r - 1)), j = 0..N_r-1: the positive
    half of the Gauss--Lobatto points of [-1, 1] (r_{N_r-1} = 1)."""
    n = p.N_r
    j = torch.arange(n, dtype=F64)
    return torch.cos(math.pi * (n - 1 - j) / (2 * n - 1))


def fd_matrices(p, parity, r=None, width=9):
    """Dense D1, D2 for functions of the given parity (+1 even, -1 odd) in r.
    Row j uses the nine points of the extended grid (-r_{N-1} .. -r_0, r_0 ..
    r_{N-1}) nearest to r_j -- centred, one-sided at the wall -- with
    Fornberg's weights; the weight of a mirror point -r_k is added, times the
    parity, to column k."""
    if r is None:
        r = radial_grid(p)
    n = r.numel()
    ext = [-x for x in reversed(r.tolist())] + r.tolist()  # ascending, 2n points
    D1 = torch.zeros(n, n, dtype=F64)
    D2 = torch.zeros(n, n, dtype=F64)
    half = width // 2
    for j in range(n):
        e0 = n + j  # position of r_j in the extended grid
        s = min(max(e0 - half, 0), 2 * n - width)
        w = fornberg(ext[e0], ext[s:s + width], 2)
        for i in range(width):
            e = s + i
            col, sg = (e - n, 1.0) if e >= n else (n - 1 - e, float(parity))
            D1[j, col] += sg * w[i][1]
            D2[j, col] += sg * w[i][2]
    return D1, D2


def parity(q):
    return 1 if q % 2 == 0 else -1


class _Ops:
    """The two parities' derivative matrices and the grid."""

    def __init__(self, p):
        self.r = radial_grid(p)
        self.D1e, self.D2e = fd_matrices(p, 1, self.r)
        self.D1o, self.D2o = fd_matrices(p, -1, self.r)

    def d1(self, par):
        return self.D1e if par == 1 else self.D1o

    def d2(self, par):
        return self.D2e if par == 1 else self.D2o


def _modes(p):
    m = torch.arange(p.M_theta, dtype=F64)
    kap = (torch.arange(p.M_z, dtype=F64) - p.K) * p.kz
    return m, kap


def _d1_modes(ops, x, shift, rows):
    """D1 of a field [N_r][M_theta][M_z] whose order-m coefficients have the
    parity (-1)^(m + shift), at the radial rows ``rows``."""
    out = torch.zeros((len(rows),) + tuple(x.shape[1:]), dtype=C128)
    for m in range(x.shape[1]):
        D = ops.d1(parity(m + shift))[rows].to(C128)
        out[:, m, :] = D @ x[:, m, :]
    return out


def derived_fields(p, u, ops, rows):
    """u_r, u_theta, u_z and omega = curl u at the rows ``rows`` (the
    cylindrical curl as for the cylinders; D1 with the parity of each
    component: (-1)^(m+1) for u_r, u_theta, (-1)^m for u_z)."""
    rows = torch.as_tensor(rows)
    m, kap = _modes(p)
    rr = ops.r[rows][:, None, None]
    imr = 1j * m[None, :, None] / rr
    ik = 1j * kap[None, None, :]
    ur, ut, uz = u[0][rows], u[1][rows], u[2][rows]
    return torch.stack([ur, ut, uz,
                        imr * uz - ik * ut,
                        ik * ur - _d1_modes(ops, u[2], 0, rows),
                        _d1_modes(ops, u[1], 1, rows) + ut / rr - imr * ur])


def _spacings(r):
    """Distance to the nearest other point of the extended grid (at r_0 the
    mirror point -r_0 counts)."""
    d = r[1:] - r[:-1]
    dr = torch.empty_like(r)
    dr[0] = torch.minimum(d[0], 2.0 * r[0])
    dr[-1] = d[-1]
    dr[1:-1] = torch.minimum(d[:-1], d[1:])
    return dr


def nonlinear_planes_direct(p, u, rows, ops=None):
    """Plain definition: transform u and omega of the full state, form
    u x omega on the padded grid, transform back."""
    if ops is None:
        ops = _Ops(p)
    phys = to_physical(p, derived_fields(p, u, ops, rows))
    ur, ut, uz, wr, wt, wz = phys[:6]
    return to_spectral(p, torch.stack([ut * wz - uz * wt, uz * wr - ur * wz, ur * wt - ut * wr]))


def nonlinear_planes(p, u, rows, ops=None):
    """u x omega at the rows ``rows`` with the exact split into the mean
    (mode (0,0): U_r, V, W, functions of r only) and the rest, as for the
    cylinders: only u' x omega' goes through the padded grid; products with
    r-only profiles multiply each coefficient.  Mean vorticity
    (0, -D1 W, D1 V + V/r) with D1 of the parities of W (even) and V (odd).
    Returns (Nhat [3][len(rows)][M_theta][M_z], dt_cfl over those rows)."""
    if ops is None:
        ops = _Ops(p)
    rows = torch.as_tensor(rows)
    r = ops.r
    mean = u[:, :, 0, p.K].real
    up = u.clone()
    up[:, :, 0, p.K] = 0.0
    spec = derived_fields(p, up, ops, rows)
    phys = to_physical(p, spec)
    ur, ut, uz, wr, wt, wz = phys[:6]
    Nhat = to_spectral(p, torch.stack([ut * wz - uz * wt, uz * wr - ur * wz, ur * wt - ut * wr]))
    Ur, V, W = mean[0], mean[1], mean[2]
    Om_t = -(ops.D1e @ W)
    Om_z = ops.D1o @ V + V / r
    col = lambda x: x[rows][:, None, None].to(C128)  # noqa: E731
    cUr, cV, cW, cOt, cOz = col(Ur), col(V), col(W), col(Om_t), col(Om_z)
    pr, pt, pz, qr, qt, qz = spec[:6]
    Nhat[0] = Nhat[0] + cV * qz - cW * qt + pt * cOz - pz * cOt
    Nhat[1] = Nhat[1] + cW * qr - cUr * qz - pr * cOz
    Nhat[2] = Nhat[2] + cUr * qt - cV * qr + pr * cOt
    Nhat[0, :, 0, p.K] = Nhat[0, :, 0, p.K] + (V * Om_z - W * Om_t)[rows]
    Nhat[1, :, 0, p.K] = Nhat[1, :, 0, p.K] - (Ur * Om_z)[rows]
    Nhat[2, :, 0, p.K] = Nhat[2, :, 0, p.K] + (Ur * Om_t)[rows]
    # CFL bound on the padded grid from the full velocity
    rr = r[rows][:, None, None]
    ur = ur + Ur[rows][:, None, None]
    ut = ut + V[rows][:, None, None]
    uz = uz + W[rows][:, None, None]
    dr = _spacings(r)[rows][:, None, None]
    dth = 2.0 * math.pi / p.N_theta
    dz = p.L_z / p.N_z
    inf = torch.tensor(math.inf, dtype=F64)
    cand = torch.stack([
        torch.where(ur.abs() > 0, dr / ur.abs(), inf),
        torch.where(ut.abs() > 0, rr * dth / ut.abs(), inf),
        torch.where(uz.abs() > 0, dz / uz.abs(), inf)])
    return Nhat, float(cand.detach().min())


def nonlinear(p, u, ops=None):
    """N(u) on all rows, the m = 0 column made Hermitian, and dt_cfl(u)."""
    N, dt_cfl = nonlinear_planes(p, u, torch.arange(p.N_r), ops)
    return herm(p, N), dt_cfl


def cfl_dt(p, u):
    return nonlinear(p, u)[1]


def l_operator(ops, q, kap):
    """Dense L_q = D2 + R^-1 D1 - q^2 R^-2 - kappa^2 I with the parity (-1)^q."""
    r = ops.r
    par = parity(q)
    n = r.numel()
    return (ops.d2(par) + ops.d1(par) / r[:, None] - q * q * torch.diag(1.0 / r ** 2)
            - kap * kap * torch.eye(n, dtype=F64))


def _solve(A, b):
    """Real A [n, n] against complex b [n] or [n, c]."""
    br = torch.stack([b.real, b.imag], dim=-1) if b.dim() == 1 else torch.cat([b.real, b.imag], -1)
    x = torch.linalg.solve(A, br)
    if b.dim() == 1:
        return torch.complex(x[:, 0], x[:, 1])
    c = b.shape[-1]
    return torch.complex(x[:, :c], x[:, c:])


def _wall_row(A):
    """Helmholtz operator with the wall row replaced by the identity row."""
    A = A.clone()
    A[-1, :] = 0.0
    A[-1, -1] = 1.0
    return A


def radial_solve_mode(p, ops, m, kk, Xn, Nn, Nq, dt, c=0.5, forcing=True):
    """Implicit stage for one mode (m, kk = k + K).  Xn, Nn, Nq: [3][N_r]
    complex (u_r, u_theta, u_z).  With X+- = X_r +- i X_theta, q(+) = m + 1,
    q(-) = |m - 1|, q(z) = q(p) = m (each operator with the parity of its
    order):
      1. f_X = X^n/dt + (1-c) L_q X^n + c N^q_X + (1-c) N^n_X on all rows
         (mode (0,0): f_z += 4 Re, the driving pressure gradient, when
         ``forcing``);
      2. g = 1/2[(D1 + (1+m)/r) f+ + (D1 + (1-m)/r) f-] + i kappa f_z;
      3. P_m p0 = g with the wall row replaced by the Neumann row D1 and
         zero data there;
      4. H_X X0 = f_X - (grad p0)_X with X0 = 0 at the wall, H_X = I/dt -
         c L_q, (grad p)+- = D1 p -+ (m/r) p, (grad p)_z = i kappa p;
      5. the response to a unit Neumann datum: P_m p1 = e_wall,
         H_X X1 = -(grad p1)_X;
      6. lambda = -beta(X0) / beta(X1), beta = div X at the wall;
         X = X0 + lambda X1, p = p0 + lambda p1;
      7. mode (0,0): u_r = 0; u_theta, u_z from their Helmholtz problems
         (orders 1 and 0) with zero wall values; the pressure head from
         dp/dr = F_r = c N^q_r + (1-c) N^n_r in divergence form,
         (D2 + D1/r) p = (D1 + 1/r) F_r inside, p = 0 at the wall.
    Returns (X [3][N_r], p [N_r])."""
    r = ops.r
    n = r.numel()
    kap = (kk - p.K) * p.kz
    eye = torch.eye(n, dtype=F64)
    qs = {"+": m + 1, "-": abs(m - 1), "z": m}
    L = {x: l_operator(ops, q, kap) for x, q in qs.items()}
    Xs = {"+": Xn[0] + 1j * Xn[1], "-": Xn[0] - 1j * Xn[1], "z": Xn[2]}
    Nns = {"+": Nn[0] + 1j * Nn[1], "-": Nn[0] - 1j * Nn[1], "z": Nn[2]}
    Nqs = {"+": Nq[0] + 1j * Nq[1], "-": Nq[0] - 1j * Nq[1], "z": Nq[2]}
    f = {x: Xs[x] / dt + (1 - c) * (L[x].to(C128) @ Xs[x]) + c * Nqs[x] + (1 - c) * Nns[x]
         for x in qs}
    H = {x: _wall_row(eye / dt - c * L[x]) for x in qs}
    inv_r = 1.0 / r
    D1v = ops.d1(parity(m + 1)).to(C128)  # velocity components: parity (-1)^(m+1)
    D1s = ops.d1(parity(m)).to(C128)      # scalars (p, u_z, div): parity (-1)^m
    X = torch.zeros((3, n), dtype=C128)
    if m == 0 and kk == p.K:
        ft = (f["+"] - f["-"]) / 2j
        fz = f["z"] + (p.G if forcing else 0.0)
        ft[-1] = 0.0
        fz[-1] = 0.0
        X[1] = _solve(H["+"], ft)
        X[2] = _solve(H["z"], fz)
        Fr = c * Nq[0] + (1 - c) * Nn[0]
        Pm = ops.D2e + ops.D1e / r[:, None]
        Pm[-1, :] = 0.0
        Pm[-1, -1] = 1.0
        rhs = ops.D1o.to(C128) @ Fr + inv_r * Fr
        rhs[-1] = 0.0
        return X, _solve(Pm, rhs)

    def div(ap, am, az):
        return (0.5 * ((D1v @ ap + (1 + m) * inv_r * ap) + (D1v @ am + (1 - m) * inv_r * am))
                + 1j * kap * az)

    g = div(f["+"], f["-"], f["z"])
    g[-1] = 0.0
    P = L["z"].clone()
    P[-1, :] = ops.d1(parity(m))[-1]
    e = torch.zeros(n, dtype=C128)
    e[-1] = 1.0
    p0 = _solve(P, g)
    p1 = _solve(P, e)

    def grad(pp):
        dp = D1s @ pp
        mr = m * inv_r * pp
        return {"+": dp - mr, "-": dp + mr, "z": 1j * kap * pp}

    g0, g1 = grad(p0), grad(p1)
    X0, X1 = {}, {}
    for x in qs:
        b0 = f[x] - g0[x]
        b1 = -g1[x]
        b0[-1] = 0.0
        b1[-1] = 0.0
        X0[x] = _solve(H[x], b0)
        X1[x] = _solve(H[x], b1)
    beta0 = div(X0["+"], X0["-"], X0["z"])[-1]
    beta1 = div(X1["+"], X1["-"], X1["z"])[-1]
    lam = -beta0 / beta1.real
    Xp = X0["+"] + lam * X1["+"]
    Xm = X0["-"] + lam * X1["-"]
    X[0] = 0.5 * (Xp + Xm)
    X[1] = (Xp - Xm) / 2j
    X[2] = X0["z"] + lam * X1["z"]
    return X, p0 + lam * p1


def radial_solve(p, Xn, Nn, Nq, dt, c=0.5, forcing=True, ops=None):
    """Full-field implicit stage: [3][N_r][M_theta][M_z] -> (X, p), the
    m = 0 column made Hermitian."""
    if ops is None:
        ops = _Ops(p)
    X = torch.zeros_like(Xn, dtype=C128)
    P = torch.zeros((p.N_r, p.M_theta, p.M_z), dtype=C128)
    for m in range(p.M_theta):
        for kk in range(p.M_z):
            x, pp = radial_solve_mode(p, ops, m, kk, Xn[:, :, m, kk], Nn[:, :, m, kk],
                                      Nq[:, :, m, kk], dt, c, forcing)
            X[:, :, m, kk] = x
            P[:, m, kk] = pp
    return herm(p, X), herm(p, P)


def step(p, u, dt, c=0.5, n_corr=1, ops=None):
    """N^n = N(u^n); X^(1) = Solve(u^n, N^n, N^n); n_corr correctors
    X^(q+1) = Solve(u^n, N^n, N(X^(q))).  Returns (u^{n+1}, dt_cfl(u^n))."""
    if ops is None:
        ops = _Ops(p)
    Nn, dt_cfl = nonlinear(p, u, ops)
    X, _ = radial_solve(p, u, Nn, Nn, dt, c, ops=ops)
    for _ in range(n_corr):
        Nq, _ = nonlinear(p, X, ops)
        X, _ = radial_solve(p, u, Nn, Nq, dt, c, ops=ops)
    return X, dt_cfl


def run(p, u0, steps, dt0=None, dynamic=False, cfl=0.5, dt_max=1e-3, c=0.5, n_corr=1):
    """Integrate ``steps`` steps (dynamic control as for the cylinders)."""
    ops = _Ops(p)
    u = u0
    if dt0 is None:
        dt0 = min(dt_max, cfl * nonlinear(p, u0, ops)[1])
    dt = dt0
    dts = []
    for _ in range(steps):
        u, dtc = step(p, u, dt, c, n_corr, ops)
        dts.append(dt)
        if dynamic:
            dt = next_dt(dt, dtc, cfl, dt_max)
    return u, dts


def base_state(p, r=None):
    """Hagen--Poiseuille flow u_z = Re (1 - r^2) in mode (0,0)."""
    if r is None:
        r = radial_grid(p)
    u = torch.zeros(p.shape(), dtype=C128)
    u[2, :, 0, p.K] = (p.Re * (1.0 - r * r)).to(C128)
    return u


def initial_state(p, amps, dt_proj=1e-3):
    """Divergence-free initial condition exciting the modes of ``amps``
    ([3][M_theta][M_z]; amps[0], amps[1] the u_r and u_theta amplitudes,
    amps[2] the u_z amplitude), added to Hagen--Poiseuille flow.  The
    perturbation is regular at the axis: u_+- = (a_r +- i a_theta) g_{m+-1}(r),
    u_z = a_z g_m(r), with g_q(r) = r^q (1 - r^2)^2 scaled to a peak of one
    (the behaviour r^q of an order-q field at the axis; zero value and slope
    at the wall), then projected by one backward-Euler Stokes stage (c = 1,
    N = 0, no driving, zero wall values)."""
    ops = _Ops(p)
    r = ops.r

    def g(q):
        peak = (q / (q + 4.0)) ** (q / 2.0) * (4.0 / (q + 4.0)) ** 2 if q > 0 else 1.0
        return (r ** q) * (1.0 - r * r) ** 2 / peak

    amps = herm(p, amps.to(C128))
    ut = torch.zeros(p.shape(), dtype=C128)
    for m in range(p.M_theta):
        up = (amps[0, m] + 1j * amps[1, m])[None, :] * g(m + 1)[:, None].to(C128)
        um = (amps[0, m] - 1j * amps[1, m])[None, :] * g(abs(m - 1))[:, None].to(C128)
        ut[0, :, m, :] = 0.5 * (up + um)
        ut[1, :, m, :] = (up - um) / 2j
        ut[2, :, m, :] = amps[2, m][None, :] * g(m)[:, None].to(C128)
    ut = herm(p, ut)
    zero = torch.zeros_like(ut)
    proj, _ = radial_solve(p, ut, zero, zero, dt_proj, c=1.0, forcing=False, ops=ops)
    return base_state(p, r) + proj
