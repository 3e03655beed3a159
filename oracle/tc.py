"""Plain FP64 statement of one Taylor--Couette DNS time step (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Parity pinned by the
``-m "not gpu"`` tests in ``tests/test_oracle_*.py`` (closed forms, invariants,
brute force and library routines); the nsCouette formulation itself is
"parity unpinned" because the paper prints none of its equations.

Conventions (all readings; the paper fixes only the ansatz, section 2.1):
  * gap d = 1, time in viscous units d^2/nu (section 3 quotes times in d^2/nu),
    r_i = eta/(1-eta), r_o = 1/(1-eta); Re_i, Re_o are the azimuthal wall
    speeds; Gr = Ra/Pr; buoyancy +Gr*T e_z; T(r_i) = +1/2, T(r_o) = -1/2.
  * spectral arrays [F][N_r][M_theta][M_z] complex128, fields (u_r, u_theta,
    u_z[, T]); k = -K..K stored at index k+K; m = 0..M_theta-1 with the m = 0
    column Hermitian; f = sum_k f_0k e^{ikz'} + 2 Re sum_{m>=1,k} f_mk e^{i(m
    theta + k z')}, z' = 2 pi z / L_z.
  * padded physical grid N_theta = 3 M_theta, N_z = 3 (K+1) (3/2 rule).
"""
import math

import torch

F64 = torch.float64
C128 = torch.complex128


# --------------------------------------------------------------------------
# Parameters and geometry (section 2.1 "Functionality"; section 3 for the
# basic state)
# --------------------------------------------------------------------------
class Params:
    """Problem statement: two concentric, independently rotating cylinders,
    optionally differentially heated (Motivation, section 1; section 2.1).

    eta = r_i/r_o, Re_i/Re_o the wall speeds, Ra/Pr the heating, N_r radial
    points, M_theta azimuthal modes (m >= 0), M_z axial modes (odd), L_z the
    axial period.
    """

    def __init__(self, eta, Re_i, Re_o, Ra, Pr, N_r, M_theta, M_z, L_z):
        if not (0.0 < eta < 1.0):
            raise ValueError("eta must lie in (0, 1)")
        if N_r < 9:
            raise ValueError("N_r must be >= 9 (nine-point stencils)")
        if M_z < 1 or M_z % 2 == 0:
            raise ValueError("M_z must be odd")
        if M_theta < 1 or L_z <= 0.0:
            raise ValueError("M_theta >= 1 and L_z > 0 required")
        if Ra != 0.0 and Pr <= 0.0:
            raise ValueError("Pr > 0 required when Ra != 0")
        self.eta, self.Re_i, self.Re_o = float(eta), float(Re_i), float(Re_o)
        self.Ra, self.Pr = float(Ra), float(Pr)
        self.N_r, self.M_theta, self.M_z, self.L_z = int(N_r), int(M_theta), int(M_z), float(L_z)
        self.r_i = self.eta / (1.0 - self.eta)
        self.r_o = 1.0 / (1.0 - self.eta)
        self.K = (self.M_z - 1) // 2
        self.N_theta = 3 * self.M_theta
        self.N_z = 3 * (self.K + 1)
        self.kz = 2.0 * math.pi / self.L_z
        self.heated = self.Ra != 0.0
        self.F = 4 if self.heated else 3
        self.Gr = self.Ra / self.Pr if self.heated else 0.0
        # circular Couette flow u_theta = A r + B / r through the wall speeds
        self.A = (self.Re_o * self.r_o - self.Re_i * self.r_i) / (self.r_o ** 2 - self.r_i ** 2)
        self.B = self.r_i * (self.Re_i - self.A * self.r_i)

    def shape(self):
        return (self.F, self.N_r, self.M_theta, self.M_z)


def radial_grid(p):
    """Chebyshev--Gauss--Lobatto points including both walls, r_0 = r_i."""
    n = p.N_r
    j = torch.arange(n, dtype=F64)
    x = torch.cos(math.pi * (n - 1 - j) / (n - 1))
    return 0.5 * (p.r_i + p.r_o) + 0.5 * x


def fornberg(z, xs, dmax):
    """Finite-difference weights at z from the nodes xs for derivative orders
    0..dmax, by Fornberg's recursion (Math. Comp. 51 (1988) 699-706): the
    weights of the interpolating polynomial's derivatives, built up one node
    at a time.  Returns a list w[node][order]."""
    n = len(xs)
    w = [[0.0] * (dmax + 1) for _ in range(n)]
    w[0][0] = 1.0
    prod_prev = 1.0
    dz_prev = xs[0] - z
    for i in range(1, n):
        top = min(i, dmax)
        prod = 1.0
        dz_old = dz_prev
        dz_prev = xs[i] - z
        for j in range(i):
            dx = xs[i] - xs[j]
            prod *= dx
            if j == i - 1:
                # new node i: weights from the previous last node
                for d in range(top, 0, -1):
                    w[i][d] = prod_prev * (d * w[i - 1][d - 1] - dz_old * w[i - 1][d]) / prod
                w[i][0] = -prod_prev * dz_old * w[i - 1][0] / prod
            # update the old nodes j < i
            for d in range(top, 0, -1):
                w[j][d] = (dz_prev * w[j][d] - d * w[j][d - 1]) / dx
            w[j][0] = dz_prev * w[j][0] / dx
        prod_prev = prod
    return w


def fd_matrices(p, r=None, width=9):
    """Dense first/second radial derivative matrices: row j uses the nine
    nodes starting at s_j = min(max(j-4, 0), N_r-9) (section 2.1: stencil
    length nine by default); centred inside, one-sided near the walls."""
    if r is None:
        r = radial_grid(p)
    n = r.numel()
    rl = r.tolist()
    D1 = torch.zeros(n, n, dtype=F64)
    D2 = torch.zeros(n, n, dtype=F64)
    half = width // 2
    for j in range(n):
        s = min(max(j - half, 0), n - width)
        w = fornberg(rl[j], rl[s:s + width], 2)
        for i in range(width):
            D1[j, s + i] = w[i][1]
            D2[j, s + i] = w[i][2]
    return D1, D2


def cc_weights(p, r=None):
    """Clenshaw--Curtis weights for the integral over [r_i, r_o] on the CGL
    grid: the interpolatory rule, i.e. exact on Chebyshev polynomials T_n,
    n < N_r (moments 2/(1-n^2) for even n, 0 for odd n), mapped by dr = dx/2."""
    n = p.N_r
    j = torch.arange(n, dtype=F64)
    theta = math.pi * (n - 1 - j) / (n - 1)  # x_j = cos(theta_j)
    ns = torch.arange(n, dtype=F64)
    V = torch.cos(ns[:, None] * theta[None, :])
    mu = torch.zeros(n, dtype=F64)
    for k in range(0, n, 2):
        mu[k] = 2.0 / (1.0 - k * k)
    w = torch.linalg.solve(V, mu)
    return 0.5 * w


# --------------------------------------------------------------------------
# Fourier transforms in theta and z (section 2.1, pseudospectral
# Fourier--Galerkin ansatz; 3/2-rule dealiasing)
# --------------------------------------------------------------------------
def _phase(n_len, idx_out, idx_in, sign):
    """exp(sign * 2 pi i * (a*b mod N) / N) with the product reduced exactly."""
    a = torch.as_tensor(idx_out, dtype=torch.int64)[:, None]
    b = torch.as_tensor(idx_in, dtype=torch.int64)[None, :]
    t = torch.remainder(a * b, n_len).to(F64) * (2.0 * math.pi / n_len)
    return torch.complex(torch.cos(t), sign * torch.sin(t))


def _mats(p):
    m = torch.arange(p.M_theta)
    k = torch.arange(p.M_z) - p.K
    a = torch.arange(p.N_theta)
    b = torch.arange(p.N_z)
    Eth = _phase(p.N_theta, a, m, +1.0)          # [N_theta, M_theta]
    Ez = _phase(p.N_z, b, k, +1.0)               # [N_z, M_z]
    cm = torch.full((p.M_theta,), 2.0, dtype=F64)
    cm[0] = 1.0
    return Eth, Ez, cm


def to_physical(p, fhat):
    """Inverse transform: [..., M_theta, M_z] -> real [..., N_theta, N_z],
    f(theta_a, z_b) = Re sum_{m,k} c_m fhat_mk exp(i(m theta_a + k kz z_b))
    with c_0 = 1, c_{m>0} = 2 (the real part also projects a non-Hermitian
    m = 0 column onto its Hermitian part)."""
    Eth, Ez, cm = _mats(p)
    g = fhat * cm[:, None]
    return torch.real(Eth @ g @ Ez.transpose(0, 1))


def to_spectral(p, f):
    """Forward transform of a real field, retained modes only:
    fhat_mk = (N_theta N_z)^-1 sum_{a,b} f_ab exp(-i(m theta_a + k kz z_b))."""
    Eth, Ez, _ = _mats(p)
    fc = f.to(C128)
    return (Eth.conj().transpose(0, 1) @ fc @ Ez.conj()) / (p.N_theta * p.N_z)


def herm(p, x):
    """Project the m = 0 column onto Hermitian symmetry:
    x(0,k) <- (x(0,k) + conj x(0,-k)) / 2 (self-adjoint projection)."""
    col = x[..., 0, :]
    sym = 0.5 * (col + torch.flip(col, dims=(-1,)).conj())
    out = x.clone()
    out[..., 0, :] = sym
    return out


# --------------------------------------------------------------------------
# Nonlinear term: spectral curl / gradient, products in physical space
# (u x omega, -u . grad T), Boussinesq buoyancy (section 2.1)
# --------------------------------------------------------------------------
def _modes(p):
    m = torch.arange(p.M_theta, dtype=F64)
    kap = (torch.arange(p.M_z, dtype=F64) - p.K) * p.kz
    return m, kap


def derived_fields(p, u, D1=None, r=None, rows=None):
    """Return the physical-space input fields' spectra at the radial rows
    ``rows`` (default all): u_r, u_theta, u_z, omega = curl u and, if heated,
    grad T, all in cylindrical components:
      omega_r = (i m / r) u_z - i kappa u_theta
      omega_t = i kappa u_r - D1 u_z
      omega_z = D1 u_theta + u_theta / r - (i m / r) u_r
      grad T = (D1 T, (i m / r) T, i kappa T)."""
    if r is None:
        r = radial_grid(p)
    if D1 is None:
        D1, _ = fd_matrices(p, r)
    if rows is None:
        rows = torch.arange(p.N_r)
    rows = torch.as_tensor(rows)
    m, kap = _modes(p)
    rr = r[rows][:, None, None]
    imr = 1j * m[None, :, None] / rr
    ik = 1j * kap[None, None, :]

    def d1(x):
        return torch.einsum('ij,jmk->imk', D1[rows].to(C128), x)

    ur, ut, uz = u[0][rows], u[1][rows], u[2][rows]
    out = [ur, ut, uz,
           imr * uz - ik * ut,
           ik * ur - d1(u[2]),
           d1(u[1]) + ut / rr - imr * ur]
    if p.heated:
        T = u[3][rows]
        out += [d1(u[3]), imr * T, ik * T]
    return torch.stack(out)


def _spacings(p, r):
    d = r[1:] - r[:-1]
    dr = torch.empty_like(r)
    dr[0] = d[0]
    dr[-1] = d[-1]
    dr[1:-1] = torch.minimum(d[:-1], d[1:])
    return dr


def nonlinear_planes_direct(p, u, rows, D1=None, r=None):
    """Plain definition of the nonlinear term at the radial rows ``rows``:
    transform u, omega and grad T of the full state, form u x omega and
    -u . grad T on the padded grid, transform back; N_z += Gr T."""
    if r is None:
        r = radial_grid(p)
    if D1 is None:
        D1, _ = fd_matrices(p, r)
    rows = torch.as_tensor(rows)
    spec = derived_fields(p, u, D1, r, rows)
    phys = to_physical(p, spec)  # [n][R][N_theta][N_z]
    ur, ut, uz, wr, wt, wz = phys[:6]
    outs = [ut * wz - uz * wt, uz * wr - ur * wz, ur * wt - ut * wr]
    if p.heated:
        gr, gt, gz = phys[6:9]
        outs.append(-(ur * gr + ut * gt + uz * gz))
    Nhat = to_spectral(p, torch.stack(outs))
    if p.heated:
        Nhat[2] = Nhat[2] + p.Gr * u[3][rows]
    return Nhat


def nonlinear_planes(p, u, rows, D1=None, r=None):
    """Nonlinear term at the radial rows ``rows``, evaluated with the exact
    split of the state into its mean (mode (0,0): a function of r only,
    taken as the real part that the physical field carries) and the rest:
    with mean velocity (U, V, W)(r), mean vorticity (0, -D1 W, D1 V + V/r),
    mean temperature gradient (D1 T_m, 0, 0) and the primed remainder,
      u x omega  = mean x mean + mean x omega' + u' x mean-vorticity + u' x omega',
      -u . grad T = -(mean . grad T_m) - mean . grad T' - u' . grad T_m - u' . grad T'.
    Products with r-only fields multiply every Fourier coefficient by a
    radial profile (no new modes, nothing to dealias); only u' x omega' and
    u' . grad T' go through the padded grid.  Equal to the plain definition
    (nonlinear_planes_direct) in exact arithmetic, with rounding errors that
    scale with the non-mean part of the flow.

    Returns (Nhat [F][len(rows)][M_theta][M_z], dt_cfl over those rows)."""
    if r is None:
        r = radial_grid(p)
    if D1 is None:
        D1, _ = fd_matrices(p, r)
    rows = torch.as_tensor(rows)
    mean = u[:, :, 0, p.K].real  # [F][N_r]
    up = u.clone()
    up[:, :, 0, p.K] = 0.0
    spec = derived_fields(p, up, D1, r, rows)
    phys = to_physical(p, spec)  # [n][R][N_theta][N_z]
    ur, ut, uz, wr, wt, wz = phys[:6]
    outs = [ut * wz - uz * wt, uz * wr - ur * wz, ur * wt - ut * wr]
    if p.heated:
        gr, gt, gz = phys[6:9]
        outs.append(-(ur * gr + ut * gt + uz * gz))
    Nhat = to_spectral(p, torch.stack(outs))
    # mean profiles at the rows (R-vectors) and their discrete derivatives
    Ur, V, W = mean[0], mean[1], mean[2]
    Om_t = -(D1 @ W)
    Om_z = D1 @ V + V / r
    col = lambda x: x[rows][:, None, None].to(C128)  # noqa: E731
    cUr, cV, cW, cOt, cOz = col(Ur), col(V), col(W), col(Om_t), col(Om_z)
    pr, pt, pz, qr, qt, qz = spec[:6]  # u' and omega' spectra
    Nhat[0] = Nhat[0] + cV * qz - cW * qt + pt * cOz - pz * cOt
    Nhat[1] = Nhat[1] + cW * qr - cUr * qz - pr * cOz
    Nhat[2] = Nhat[2] + cUr * qt - cV * qr + pr * cOt
    Nhat[0, :, 0, p.K] = Nhat[0, :, 0, p.K] + (V * Om_z - W * Om_t)[rows]
    Nhat[1, :, 0, p.K] = Nhat[1, :, 0, p.K] - (Ur * Om_z)[rows]
    Nhat[2, :, 0, p.K] = Nhat[2, :, 0, p.K] + (Ur * Om_t)[rows]
    if p.heated:
        G = D1 @ mean[3]
        cG = col(G)
        g1, g2, g3 = spec[6:9]  # grad T' spectra
        Nhat[3] = Nhat[3] - (cUr * g1 + cV * g2 + cW * g3 + pr * cG)
        Nhat[3, :, 0, p.K] = Nhat[3, :, 0, p.K] - (Ur * G)[rows]
        Nhat[2] = Nhat[2] + p.Gr * u[3][rows]
    # CFL time-step bound on the padded grid, from the full velocity
    rr = r[rows][:, None, None]
    ur = ur + Ur[rows][:, None, None]
    ut = ut + V[rows][:, None, None]
    uz = uz + W[rows][:, None, None]
    dr = _spacings(p, r)[rows][:, None, None]
    dth = 2.0 * math.pi / p.N_theta
    dz = p.L_z / p.N_z
    inf = torch.tensor(math.inf, dtype=F64)
    cand = torch.stack([
        torch.where(ur.abs() > 0, dr / ur.abs(), inf),
        torch.where(ut.abs() > 0, rr * dth / ut.abs(), inf),
        torch.where(uz.abs() > 0, dz / uz.abs(), inf)])
    return Nhat, float(cand.detach().min())


def nonlinear(p, u, D1=None, r=None):
    """Full nonlinear term N(u) (all rows) with the m = 0 column made
    Hermitian, and the CFL bound dt_cfl evaluated from u."""
    N, dt_cfl = nonlinear_planes(p, u, torch.arange(p.N_r), D1, r)
    return herm(p, N), dt_cfl


def cfl_dt(p, u):
    return nonlinear(p, u)[1]


# --------------------------------------------------------------------------
# Radial operators and the per-mode implicit solve (section 2.2: the linear
# terms are independent per Fourier mode)
# --------------------------------------------------------------------------
def l_operator(p, q, kap, D1, D2, r):
    """Batched dense L_q = D2 + R^-1 D1 - q^2 R^-2 - kappa^2 I; q and kap are
    1-D tensors of equal length B -> [B, N_r, N_r]."""
    n = r.numel()
    base = D2 + D1 / r[:, None]
    eye = torch.eye(n, dtype=F64)
    q2 = (q.to(F64) ** 2)[:, None, None]
    k2 = (kap.to(F64) ** 2)[:, None, None]
    return base[None] - q2 * torch.diag(1.0 / r ** 2)[None] - k2 * eye[None]


def _rsolve(A, b):
    """Solve real A [B,n,n] against complex right sides b [B,n,c]."""
    br = torch.cat([b.real, b.imag], dim=-1)
    x = torch.linalg.solve(A, br)
    c = b.shape[-1]
    return torch.complex(x[..., :c], x[..., c:])


def _dirichlet(H):
    H = H.clone()
    n = H.shape[-1]
    H[:, 0, :] = 0.0
    H[:, -1, :] = 0.0
    H[:, 0, 0] = 1.0
    H[:, -1, n - 1] = 1.0
    return H


def radial_solve_modes(p, m, kk, Xn, Nn, Nq, dt, c=0.5, walls=True,
                       D1=None, D2=None, r=None):
    """Implicit part of one predictor or corrector stage for the modes
    (m[b], kk[b]) (kk = k+K), b = 0..B-1.  Xn, Nn, Nq: [F][N_r][B] complex.

    Per mode, with X+- = X_r +- i X_theta and q(+) = m+1, q(-) = |m-1|,
    q(z) = q(T) = q(p) = m:
      1. f_X = X^n/dt + (1-c) L_q X^n + c N^q + (1-c) N^n on all rows
         (T: L_m / Pr);
      2. g = 1/2[(D1 + (1+m)/r) f+ + (D1 + (1-m)/r) f-] + i kappa f_z;
      3. P_m p0 = g with Neumann rows (D1) at both walls and zero data there;
      4. H_X X0 = f_X - (grad p0)_X inside, wall rows = wall values, with
         H_X = I/dt - c L_q, (grad p)+- = D1 p -+ (m/r) p, (grad p)_z = i kappa p;
      5. homogeneous responses p_j (Neumann data e_j), X_j = H^-1(-grad p_j);
      6. influence matrix: lambda = -A^-1 beta(X0), A = [beta(X1) beta(X2)],
         beta = wall values of div X; X = X0 + sum lambda_j X_j, p likewise;
      7. mode (0,0): u_r = 0, u_theta with L_1 and u_z with L_0 under the wall
         speeds; p^00 from dp/dr = F_r = c N^q_r + (1-c) N^n_r in divergence
         form, (D2 + D1/r) p = (D1 + 1/r) F_r inside, p(r_i) = 0, D1 p = F_r
         at r_o;
      8. T: (I/dt - (c/Pr) L_m) T = f_T with T = +-1/2 at the walls in (0,0).
    Returns (X [F][N_r][B], p [N_r][B])."""
    if r is None:
        r = radial_grid(p)
    if D1 is None:
        D1, D2 = fd_matrices(p, r)
    n = p.N_r
    m = torch.as_tensor(m, dtype=torch.int64)
    kk = torch.as_tensor(kk, dtype=torch.int64)
    B = m.numel()
    mf = m.to(F64)
    kap = (kk - p.K).to(F64) * p.kz
    eye = torch.eye(n, dtype=F64)
    D1c = D1.to(C128)

    def tomode(x):  # [N_r][B] -> [B][N_r]
        return x.transpose(0, 1)

    def apply(Lop, x):  # Lop [B,n,n], x [B,n] complex
        return torch.einsum('bij,bj->bi', Lop.to(C128), x)

    def d1(x):
        return torch.einsum('ij,bj->bi', D1c, x)

    inv_r = (1.0 / r)[None, :]
    Xp = tomode(Xn[0] + 1j * Xn[1]); Xm = tomode(Xn[0] - 1j * Xn[1]); Xz = tomode(Xn[2])
    Np_n = tomode(Nn[0] + 1j * Nn[1]); Nm_n = tomode(Nn[0] - 1j * Nn[1]); Nz_n = tomode(Nn[2])
    Np_q = tomode(Nq[0] + 1j * Nq[1]); Nm_q = tomode(Nq[0] - 1j * Nq[1]); Nz_q = tomode(Nq[2])

    Lp = l_operator(p, m + 1, kap, D1, D2, r)
    Lm = l_operator(p, (m - 1).abs(), kap, D1, D2, r)
    Lz = l_operator(p, m, kap, D1, D2, r)

    f_p = Xp / dt + (1 - c) * apply(Lp, Xp) + c * Np_q + (1 - c) * Np_n
    f_m = Xm / dt + (1 - c) * apply(Lm, Xm) + c * Nm_q + (1 - c) * Nm_n
    f_z = Xz / dt + (1 - c) * apply(Lz, Xz) + c * Nz_q + (1 - c) * Nz_n

    def div(ap, am, az, mv, kv):
        return (0.5 * ((d1(ap) + (1 + mv)[:, None] * inv_r * ap)
                       + (d1(am) + (1 - mv)[:, None] * inv_r * am))
                + 1j * kv[:, None] * az)

    Hp = _dirichlet(eye[None] / dt - c * Lp)
    Hm = _dirichlet(eye[None] / dt - c * Lm)
    Hz = _dirichlet(eye[None] / dt - c * Lz)

    Xout = torch.zeros((p.F, n, B), dtype=C128)
    Pout = torch.zeros((n, B), dtype=C128)

    zero = (m == 0) & (kk == p.K)
    gen = ~zero
    if gen.any():
        gi = gen.nonzero().flatten()
        mg = mf[gi]
        kg = kap[gi]
        g = div(f_p[gi], f_m[gi], f_z[gi], mg, kg)
        g[:, 0] = 0.0
        g[:, -1] = 0.0
        P = Lz[gi].clone()
        P[:, 0, :] = D1[0]
        P[:, -1, :] = D1[-1]
        e = torch.zeros((gi.numel(), n, 2), dtype=C128)
        e[:, 0, 0] = 1.0
        e[:, -1, 1] = 1.0
        sol = _rsolve(P, torch.cat([g[:, :, None], e], dim=-1))
        pr = [sol[..., 0], sol[..., 1], sol[..., 2]]  # p0, p1, p2

        def grad_p(pp):
            dp = d1(pp)
            mr = mg[:, None] * inv_r * pp
            return dp - mr, dp + mr, 1j * kg[:, None] * pp

        def masked(v):
            v = v.clone()
            v[:, 0] = 0.0
            v[:, -1] = 0.0
            return v

        rhs_p, rhs_m, rhs_z = [], [], []
        for j, pp in enumerate(pr):
            gp, gm, gz = grad_p(pp)
            if j == 0:
                rhs_p.append(masked(f_p[gi] - gp))
                rhs_m.append(masked(f_m[gi] - gm))
                rhs_z.append(masked(f_z[gi] - gz))
            else:
                rhs_p.append(masked(-gp))
                rhs_m.append(masked(-gm))
                rhs_z.append(masked(-gz))
        Sp = _rsolve(Hp[gi], torch.stack(rhs_p, dim=-1))
        Sm = _rsolve(Hm[gi], torch.stack(rhs_m, dim=-1))
        Sz = _rsolve(Hz[gi], torch.stack(rhs_z, dim=-1))
        # wall divergence of each candidate: beta[b, wall, j]
        beta = torch.stack([div(Sp[..., j], Sm[..., j], Sz[..., j], mg, kg)[:, [0, -1]]
                            for j in range(3)], dim=-1)
        A = beta[..., 1:].real  # [B,2,2]: A[:, wall, j] = beta_wall(X_j)
        det = A[:, 0, 0] * A[:, 1, 1] - A[:, 0, 1] * A[:, 1, 0]
        b0 = beta[..., 0]
        lam1 = -(A[:, 1, 1] * b0[:, 0] - A[:, 0, 1] * b0[:, 1]) / det
        lam2 = -(-A[:, 1, 0] * b0[:, 0] + A[:, 0, 0] * b0[:, 1]) / det
        l1 = lam1[:, None]
        l2 = lam2[:, None]
        Xp_new = Sp[..., 0] + l1 * Sp[..., 1] + l2 * Sp[..., 2]
        Xm_new = Sm[..., 0] + l1 * Sm[..., 1] + l2 * Sm[..., 2]
        Xz_new = Sz[..., 0] + l1 * Sz[..., 1] + l2 * Sz[..., 2]
        P_new = pr[0] + l1 * pr[1] + l2 * pr[2]
        Xout[0][:, gi] = (0.5 * (Xp_new + Xm_new)).transpose(0, 1)
        Xout[1][:, gi] = ((Xp_new - Xm_new) / 2j).transpose(0, 1)
        Xout[2][:, gi] = Xz_new.transpose(0, 1)
        Pout[:, gi] = P_new.transpose(0, 1)
    if zero.any():
        zi = zero.nonzero().flatten()
        f_t = (f_p[zi] - f_m[zi]) / 2j
        rt = f_t.clone()
        rz = f_z[zi].clone()
        rt[:, 0] = p.Re_i if walls else 0.0
        rt[:, -1] = p.Re_o if walls else 0.0
        rz[:, 0] = 0.0
        rz[:, -1] = 0.0
        ut = _rsolve(Hp[zi], rt[:, :, None])[..., 0]
        uz = _rsolve(Hz[zi], rz[:, :, None])[..., 0]
        Xout[0][:, zi] = 0.0
        Xout[1][:, zi] = ut.transpose(0, 1)
        Xout[2][:, zi] = uz.transpose(0, 1)
        # pressure head of the mean flow, dp/dr = F_r = c N^q_r + (1-c) N^n_r,
        # in divergence form: (D2 + D1/r) p = (D1 + 1/r) F_r inside,
        # p(r_i) = 0, D1 p = F_r at r_o
        fr = (c * Nq[0][:, zi] + (1 - c) * Nn[0][:, zi]).transpose(0, 1)
        Pm = D2 + D1 / r[:, None]
        Pm[0, :] = 0.0
        Pm[0, 0] = 1.0
        Pm[-1, :] = D1[-1]
        rhs = d1(fr) + inv_r * fr
        rhs[:, 0] = 0.0
        rhs[:, -1] = fr[:, -1]
        Pz = _rsolve(Pm[None].expand(zi.numel(), n, n), rhs[:, :, None])[..., 0]
        Pout[:, zi] = Pz.transpose(0, 1)
    if p.heated:
        LT = Lz / p.Pr
        Tn = tomode(Xn[3])
        f_T = Tn / dt + (1 - c) * apply(LT, Tn) + c * tomode(Nq[3]) + (1 - c) * tomode(Nn[3])
        HT = _dirichlet(eye[None] / dt - c * LT)
        rT = f_T.clone()
        rT[:, 0] = 0.0
        rT[:, -1] = 0.0
        if walls and zero.any():
            zi = zero.nonzero().flatten()
            rT[zi, 0] = 0.5
            rT[zi, -1] = -0.5
        Xout[3] = _rsolve(HT, rT[:, :, None])[..., 0].transpose(0, 1)
    return Xout, Pout


def radial_solve(p, Xn, Nn, Nq, dt, c=0.5, walls=True, chunk=None):
    """Full-field implicit stage: Xn, Nn, Nq [F][N_r][M_theta][M_z] ->
    (X, p) with the m = 0 column made Hermitian."""
    r = radial_grid(p)
    D1, D2 = fd_matrices(p, r)
    F, n, Mt, Mz = Xn.shape
    tot = Mt * Mz
    m_all = torch.arange(Mt).repeat_interleave(Mz)
    k_all = torch.arange(Mz).repeat(Mt)
    X = torch.zeros((F, n, tot), dtype=C128)
    P = torch.zeros((n, tot), dtype=C128)
    if chunk is None:
        chunk = max(1, min(tot, 2 ** 22 // (n * n)))
    Xf = Xn.reshape(F, n, tot)
    Nnf = Nn.reshape(F, n, tot)
    Nqf = Nq.reshape(F, n, tot)
    for s in range(0, tot, chunk):
        e = min(tot, s + chunk)
        xo, po = radial_solve_modes(p, m_all[s:e], k_all[s:e], Xf[:, :, s:e],
                                    Nnf[:, :, s:e], Nqf[:, :, s:e], dt, c, walls,
                                    D1, D2, r)
        X[:, :, s:e] = xo
        P[:, s:e] = po
    X = X.reshape(F, n, Mt, Mz)
    P = P.reshape(n, Mt, Mz)
    return herm(p, X), herm(p, P)


# --------------------------------------------------------------------------
# Predictor--corrector step and dynamic time step (section 2.1)
# --------------------------------------------------------------------------
def step(p, u, dt, c=0.5, n_corr=1):
    """One step: N^n = N(u^n); X^(1) = Solve(u^n, N^n, N^n); then n_corr
    corrector stages X^(q+1) = Solve(u^n, N^n, N(X^(q))).  Returns
    (u^{n+1}, dt_cfl(u^n))."""
    Nn, dt_cfl = nonlinear(p, u)
    X, _ = radial_solve(p, u, Nn, Nn, dt, c)
    for _ in range(n_corr):
        Nq, _ = nonlinear(p, X)
        X, _ = radial_solve(p, u, Nn, Nq, dt, c)
    return X, dt_cfl


def next_dt(dt, dt_cfl, cfl=0.5, dt_max=1e-3):
    """Dynamic time-step control with hysteresis: the bound is
    b = cfl * dt_cfl.  If b < dt the step shrinks to 0.9 b; if
    min(dt_max, b) > 1.2 dt it grows to min(dt_max, 0.9 b); otherwise dt is
    kept (so the radial operators are refactorised only on real changes)."""
    b = cfl * dt_cfl
    if b < dt:
        return 0.9 * b
    if min(dt_max, b) > 1.2 * dt:
        return min(dt_max, 0.9 * b)
    return dt


def run(p, u0, steps, dt0=None, dynamic=False, cfl=0.5, dt_max=1e-3, c=0.5,
        n_corr=1, callback=None):
    """Integrate ``steps`` steps.  With dynamic control the step n+1 uses
    next_dt(dt_n, dt_cfl(u^n)); dt0 defaults to min(dt_max, cfl*dt_cfl(u^0)).
    Returns (u, list of the dt used by each step)."""
    u = u0
    if dt0 is None:
        dt0 = min(dt_max, cfl * cfl_dt(p, u0))
    dt = dt0
    dts = []
    for n in range(steps):
        u, dtc = step(p, u, dt, c, n_corr)
        dts.append(dt)
        if callback is not None:
            callback(n, u, dt)
        if dynamic:
            dt = next_dt(dt, dtc, cfl, dt_max)
    return u, dts


# --------------------------------------------------------------------------
# Basic state, initial condition, energy (sections 2.1 and 3)
# --------------------------------------------------------------------------
def base_state(p, r=None):
    """Circular Couette flow u_theta = A r + B/r and, if heated, the
    conduction profile T = 1/2 + ln(r/r_i)/ln(eta), both in mode (0,0)."""
    if r is None:
        r = radial_grid(p)
    u = torch.zeros(p.shape(), dtype=C128)
    u[1, :, 0, p.K] = (p.A * r + p.B / r).to(C128)
    if p.heated:
        u[3, :, 0, p.K] = (0.5 + torch.log(r / p.r_i) / math.log(p.eta)).to(C128)
    return u


def initial_state(p, amps, dt_proj=1e-3):
    """Divergence-free initial condition exciting the modes given by ``amps``
    ([F][M_theta][M_z] complex mode amplitudes; section 2.1 "divergence-free
    initial conditions can be used to excite selected Fourier modes").

    Perturbation u~ = amps * g(r), g = 16 (r-r_i)^2 (r_o-r)^2, made
    divergence-free by one backward-Euler Stokes stage (c = 1, N = 0, zero
    wall data, dt = dt_proj), then added to the basic state.  A temperature
    perturbation amps[3] * g(r) is added without projection."""
    r = radial_grid(p)
    g = 16.0 * (r - p.r_i) ** 2 * (p.r_o - r) ** 2
    amps = herm(p, amps.to(C128))
    ut = amps[:, None, :, :] * g[None, :, None, None].to(C128)
    zero = torch.zeros_like(ut)
    proj, _ = radial_solve(p, ut, zero, zero, dt_proj, c=1.0, walls=False)
    u = base_state(p, r) + proj
    if p.heated:
        u[3] = u[3] * 0.0 + base_state(p, r)[3] + ut[3]
    return u


def energy(p, u, r=None, w=None):
    """Perturbation kinetic energy about Couette flow,
    E = 1/2 int |u - U_b|^2 dV = pi L_z sum_j w_j r_j sum_{m,k} c_m |u'_mk(r_j)|^2
    (Parseval in theta, z; Clenshaw--Curtis in r)."""
    if r is None:
        r = radial_grid(p)
    if w is None:
        w = cc_weights(p, r)
    up = u[:3] - base_state(p, r)[:3]
    cm = torch.full((p.M_theta,), 2.0, dtype=F64)
    cm[0] = 1.0
    s = (up.real ** 2 + up.imag ** 2).sum(dim=0)  # [N_r][M_theta][M_z]
    s = (s * cm[None, :, None]).sum(dim=(1, 2))
    return math.pi * p.L_z * (w * r * s).sum()


def weighted_norm(p, x, r=None, w=None):
    """||x||_W^2 = sum_j w_j r_j sum_{m,k} c_m |x_mk(r_j)|^2 for one field."""
    if r is None:
        r = radial_grid(p)
    if w is None:
        w = cc_weights(p, r)
    cm = torch.full((p.M_theta,), 2.0, dtype=F64)
    cm[0] = 1.0
    s = ((x.real ** 2 + x.imag ** 2) * cm[None, :, None]).sum(dim=(1, 2))
    return torch.sqrt((w * r * s).sum())


# --------------------------------------------------------------------------
# Restart with a change of resolution (section 2.1: at every restart the
# spatial resolution may change through interpolation and mode padding;
# section 2.4: the checkpoint-restart works on the spectral coefficients).
# Reading (the paper names no interpolant): every Fourier mode's radial
# profile is carried to the new grid by the polynomial through all points of
# the old grid; modes present at both resolutions keep their coefficients,
# new modes start at zero, modes beyond the new truncation are dropped.
# --------------------------------------------------------------------------
def lagrange_matrix(x_src, x_dst):
    """W[i][j] = l_j(x_dst[i]) with the Lagrange basis of the nodes x_src,
    l_j(x) = prod_{l != j} (x - x_l) / (x_j - x_l), evaluated as written; a
    new point equal to an old node takes that node's value (W row = e_j)."""
    x_src = torch.as_tensor(x_src, dtype=F64)
    x_dst = torch.as_tensor(x_dst, dtype=F64)
    n0 = x_src.numel()
    W = torch.zeros(x_dst.numel(), n0, dtype=F64)
    for i in range(x_dst.numel()):
        x = x_dst[i]
        hit = (x_src == x).nonzero()
        if hit.numel():
            W[i, int(hit[0])] = 1.0
            continue
        for j in range(n0):
            others = torch.cat([x_src[:j], x_src[j + 1:]])
            W[i, j] = torch.prod((x - others) / (x_src[j] - others))
    return W


def remap_state(p, u_src, N_r_src):
    """State u_src [F][N_r_src][M_theta_src][M_z_src] (same geometry eta,
    L_z) at the resolution of p: modes (m, k) with m < min(M_theta) and
    |k| <= min(K) copied (k stored at k + K on each side), the others zero;
    then each mode's profile interpolated from the old radial grid to the
    new one with lagrange_matrix."""
    F, n0, mt0, mz0 = u_src.shape
    assert n0 == N_r_src and F == p.F
    K0 = (mz0 - 1) // 2
    mt = min(mt0, p.M_theta)
    kc = min(K0, p.K)
    padded = torch.zeros(F, n0, p.M_theta, p.M_z, dtype=C128)
    for k in range(-kc, kc + 1):
        padded[:, :, :mt, p.K + k] = u_src[:, :, :mt, K0 + k]
    src = Params(p.eta, p.Re_i, p.Re_o, p.Ra, p.Pr, n0, p.M_theta, p.M_z, p.L_z)
    W = lagrange_matrix(radial_grid(src), radial_grid(p)).to(C128)
    return torch.einsum("ij,fjmk->fimk", W, padded)


# --------------------------------------------------------------------------
# Heated-flow diagnostics (section 3: the Nusselt number at the inner
# cylinder -- the heat transfer there over that of the basic state at the
# same temperature difference -- and a velocity probe time series).
# Readings: the heat transfer is the radial derivative of the theta-z mean
# temperature (mode (0,0)) with the nine-point stencil at the wall; the basic
# state's is dT_c/dr = 1/(r ln eta).  The torque (not defined in the paper)
# is the angular-momentum flux G(r) = -2 pi L_z r^3 d(<u_theta>/r)/dr at a
# wall, which Couette flow carries unchanged through the gap (4 pi L_z B).
# --------------------------------------------------------------------------
def diagnostics(p, u, D1=None, r=None):
    """(Nu_i, Nu_o, G_i, G_o): Nusselt numbers at both walls (0 without
    temperature) and the torques at both walls."""
    if r is None:
        r = radial_grid(p)
    if D1 is None:
        D1, _ = fd_matrices(p, r)
    V = u[1, :, 0, p.K].real
    dV = D1 @ V
    G = -2.0 * math.pi * p.L_z * r ** 3 * (dV / r - V / r ** 2)
    if p.heated:
        T = u[3, :, 0, p.K].real
        Nu = (D1 @ T) * r * math.log(p.eta)
        nu_i, nu_o = float(Nu[0]), float(Nu[-1])
    else:
        nu_i = nu_o = 0.0
    return nu_i, nu_o, float(G[0]), float(G[-1])


def probe(p, u, rows, theta, z):
    """Every field at the physical points (r_rows[n], theta[n], z[n]): the
    Fourier sum sum_k u_0k e^{ik kz z} + 2 Re sum_{m>=1,k} u_mk e^{i(m theta
    + k kz z)}, written out term by term.  Returns [n][F]."""
    out = torch.zeros(len(rows), p.F, dtype=F64)
    m = torch.arange(p.M_theta, dtype=F64)[:, None]
    k = (torch.arange(p.M_z, dtype=F64) - p.K)[None, :]
    c = torch.where(m == 0, 1.0, 2.0)
    for n, (j, th, zz) in enumerate(zip(rows, theta, z)):
        ph = torch.exp(1j * (m * th + k * p.kz * zz))
        for f in range(p.F):
            out[n, f] = (c * u[f, j] * ph).real.sum()
    return out
