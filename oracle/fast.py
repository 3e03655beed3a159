"""Faster FP64 CPU evaluation of the oracle's time step (CPU reference figure).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the CPU tests and
the benchmark's CPU reference figure use it; the library never does.

The same method and formulas as ``oracle.tc`` -- the nonlinear term with
the mean split of ``nonlinear_planes``, the implicit stage of
``radial_solve_modes`` (sections 2.1 and 2.2: Fourier--Galerkin in theta
and z with 3/2-rule dealiasing, nine-point finite differences in r,
pressure by an influence-matrix method, predictor--corrector) -- evaluated
the way a CPU code would, so that the figure says what a tuned host
implementation of this discretisation costs:

  * transforms by FFT (pocketfft through ``scipy.fft``, over every host
    thread the process may use) instead of DFT matrices;
  * the radial operators applied as the shared derivative matrices plus a
    diagonal per mode, and the radial systems inverted once per step size
    (LU with partial pivoting, batched over the modes), so that a stage only
    multiplies (a batched product of 64-point systems runs several times
    faster on the host than batched triangular solves); the pressure
    operators and their wall responses depend on the mode alone and are
    inverted once, the velocity responses and the 2x2 influence matrices
    once per step size.

Results agree with ``oracle.tc`` up to rounding order (tests in
``tests/test_oracle_fast.py``).
"""
import math
import os

import numpy as np
import scipy.fft as sfft
import torch

from . import tc

F64 = torch.float64
C128 = torch.complex128


def host_threads():
    """The CPUs this process may run on."""
    return len(os.sched_getaffinity(0))


class Stepper:
    """Time steps of one problem (tc.Params) on the host."""

    def __init__(self, p, workers=None):
        self.p = p
        self.workers = workers or host_threads()
        r = tc.radial_grid(p)
        D1, D2 = tc.fd_matrices(p, r)
        self.r, self.D1, self.D2 = r, D1, D2
        n = p.N_r
        self.B = p.M_theta * p.M_z
        # flat mode index b = m * M_z + (k + K)
        self.m = torch.arange(p.M_theta).repeat_interleave(p.M_z)
        self.kk = torch.arange(p.M_z).repeat(p.M_theta)
        self.kap = (self.kk - p.K).to(F64) * p.kz
        self.zero = int(p.K)  # mode (0, 0)
        gen = torch.ones(self.B, dtype=torch.bool)
        gen[self.zero] = False
        self.gi = gen.nonzero().flatten()
        self.base = D2 + D1 / r[:, None]  # L_q = base - q^2/r^2 - kappa^2
        self.inv_r2 = 1.0 / r ** 2
        self.eye = torch.eye(n, dtype=F64)
        mg, kg = self.m[self.gi], self.kap[self.gi]
        # pressure: L_m with Neumann rows; responses to unit wall data
        P = self._dense(mg, kg)
        P[:, 0, :] = D1[0]
        P[:, -1, :] = D1[-1]
        self.P = torch.linalg.inv(P)
        self.p1 = self.P[:, :, 0].to(C128)  # responses to unit Neumann data
        self.p2 = self.P[:, :, -1].to(C128)
        self.dt = None

    # ------------------------------------------------------------------
    # radial operators
    # ------------------------------------------------------------------
    def _dense(self, q, kap):
        """L_q for the modes of q, kap: [B, N_r, N_r]."""
        q2 = (q.to(F64) ** 2)[:, None, None]
        k2 = (kap ** 2)[:, None, None]
        return self.base[None] - q2 * torch.diag(self.inv_r2)[None] - k2 * self.eye[None]

    def _apply_l(self, q, kap, x, scale=1.0):
        """scale * L_q x for x [B, N_r] complex (shared matrix + diagonal)."""
        bx = x @ self.base.T.to(C128)
        d = (q.to(F64) ** 2)[:, None] * self.inv_r2[None, :] + (kap ** 2)[:, None]
        return scale * (bx - d * x)

    @staticmethod
    def _dirichlet(H):
        n = H.shape[-1]
        H[:, 0, :] = 0.0
        H[:, -1, :] = 0.0
        H[:, 0, 0] = 1.0
        H[:, -1, n - 1] = 1.0
        return H

    @staticmethod
    def _lu_solve_c(ainv, b):
        """Solve with the inverses ainv [B, n, n] against complex right
        sides b [B, n]."""
        x = torch.bmm(ainv, torch.stack([b.real, b.imag], dim=-1))
        return torch.complex(x[..., 0], x[..., 1])

    def _d1(self, x):
        return x @ self.D1.T.to(C128)

    def _div(self, ap, am, az, mv, kv):
        inv_r = (1.0 / self.r)[None, :]
        return (0.5 * ((self._d1(ap) + (1 + mv)[:, None] * inv_r * ap)
                       + (self._d1(am) + (1 - mv)[:, None] * inv_r * am))
                + 1j * kv[:, None] * az)

    def _grad(self, pp, mv, kv):
        dp = self._d1(pp)
        mr = mv[:, None] * (1.0 / self.r)[None, :] * pp
        return dp - mr, dp + mr, 1j * kv[:, None] * pp

    @staticmethod
    def _masked(v):
        v = v.clone()
        v[:, 0] = 0.0
        v[:, -1] = 0.0
        return v

    def set_dt(self, dt, c=0.5):
        """Invert the Helmholtz operators of step size dt and solve the
        velocity responses and influence matrices of the pressure responses."""
        if self.dt == (dt, c):
            return
        p = self.p
        g = self.gi
        mg, kg = self.m[g].to(F64), self.kap[g]
        I = self.eye[None]
        inv = torch.linalg.inv
        self.Hp = inv(self._dirichlet(I / dt - c * self._dense(self.m[g] + 1, kg)))
        self.Hm = inv(self._dirichlet(I / dt - c * self._dense((self.m[g] - 1).abs(), kg)))
        self.Hz = inv(self._dirichlet(I / dt - c * self._dense(self.m[g], kg)))
        if p.heated:
            self.HT = inv(self._dirichlet(I / dt - (c / p.Pr) * self._dense(self.m, self.kap)))
        resp = []
        for pj in (self.p1, self.p2):
            gp, gm, gz = self._grad(pj, mg, kg)
            resp.append((self._lu_solve_c(self.Hp, self._masked(-gp)),
                         self._lu_solve_c(self.Hm, self._masked(-gm)),
                         self._lu_solve_c(self.Hz, self._masked(-gz))))
        self.resp = resp
        beta = torch.stack([self._div(*resp[j], mg, kg)[:, [0, -1]] for j in range(2)], dim=-1)
        self.A = beta.real  # [B, wall, j]
        self.dt = (dt, c)

    # ------------------------------------------------------------------
    # implicit stage (radial_solve_modes over all modes)
    # ------------------------------------------------------------------
    def radial_solve(self, Xn, Nn, Nq, dt, c=0.5):
        p = self.p
        self.set_dt(dt, c)
        F, n = p.F, p.N_r
        B = self.B
        flat = lambda x: x.reshape(F, n, B)  # noqa: E731
        Xf, Nnf, Nqf = flat(Xn), flat(Nn), flat(Nq)
        g = self.gi
        mg, kg = self.m[g].to(F64), self.kap[g]

        def tomode(x):
            return x[:, g].transpose(0, 1)

        Xp = tomode(Xf[0] + 1j * Xf[1])
        Xm = tomode(Xf[0] - 1j * Xf[1])
        Xz = tomode(Xf[2])
        f_p = Xp / dt + self._apply_l(self.m[g] + 1, kg, Xp, 1 - c) \
            + c * tomode(Nqf[0] + 1j * Nqf[1]) + (1 - c) * tomode(Nnf[0] + 1j * Nnf[1])
        f_m = Xm / dt + self._apply_l((self.m[g] - 1).abs(), kg, Xm, 1 - c) \
            + c * tomode(Nqf[0] - 1j * Nqf[1]) + (1 - c) * tomode(Nnf[0] - 1j * Nnf[1])
        f_z = Xz / dt + self._apply_l(self.m[g], kg, Xz, 1 - c) \
            + c * tomode(Nqf[2]) + (1 - c) * tomode(Nnf[2])
        div = self._div(f_p, f_m, f_z, mg, kg)
        div[:, 0] = 0.0
        div[:, -1] = 0.0
        p0 = self._lu_solve_c(self.P, div)
        gp, gm, gz = self._grad(p0, mg, kg)
        Sp = self._lu_solve_c(self.Hp, self._masked(f_p - gp))
        Sm = self._lu_solve_c(self.Hm, self._masked(f_m - gm))
        Sz = self._lu_solve_c(self.Hz, self._masked(f_z - gz))
        b0 = self._div(Sp, Sm, Sz, mg, kg)[:, [0, -1]]
        A = self.A
        det = A[:, 0, 0] * A[:, 1, 1] - A[:, 0, 1] * A[:, 1, 0]
        l1 = (-(A[:, 1, 1] * b0[:, 0] - A[:, 0, 1] * b0[:, 1]) / det)[:, None]
        l2 = (-(-A[:, 1, 0] * b0[:, 0] + A[:, 0, 0] * b0[:, 1]) / det)[:, None]
        (p1p, p1m, p1z), (p2p, p2m, p2z) = self.resp
        Xp_new = Sp + l1 * p1p + l2 * p2p
        Xm_new = Sm + l1 * p1m + l2 * p2m
        Xz_new = Sz + l1 * p1z + l2 * p2z
        X = torch.zeros((F, n, B), dtype=C128)
        X[0][:, g] = (0.5 * (Xp_new + Xm_new)).transpose(0, 1)
        X[1][:, g] = ((Xp_new - Xm_new) / 2j).transpose(0, 1)
        X[2][:, g] = Xz_new.transpose(0, 1)
        # mode (0, 0): one dense solve of the plain statement
        z = self.zero
        xo, _ = tc.radial_solve_modes(p, [0], [p.K], Xf[:, :, z:z + 1], Nnf[:, :, z:z + 1],
                                      Nqf[:, :, z:z + 1], dt, c, True, self.D1, self.D2, self.r)
        X[:3, :, z] = xo[:3, :, 0]
        if p.heated:
            Tn = Xf[3].transpose(0, 1)
            f_T = Tn / dt + self._apply_l(self.m, self.kap, Tn, (1 - c) / p.Pr) \
                + c * Nqf[3].transpose(0, 1) + (1 - c) * Nnf[3].transpose(0, 1)
            rT = self._masked(f_T)
            rT[z, 0] = 0.5
            rT[z, -1] = -0.5
            X[3] = self._lu_solve_c(self.HT, rT).transpose(0, 1)
        return tc.herm(p, X.reshape(F, n, p.M_theta, p.M_z))

    # ------------------------------------------------------------------
    # transforms and nonlinear term (nonlinear_planes over all rows)
    # ------------------------------------------------------------------
    def to_physical(self, spec):
        """[..., M_theta, M_z] -> real [..., N_theta, N_z], as tc.to_physical."""
        p = self.p
        x = spec.numpy()
        g = np.zeros(x.shape[:-1] + (p.N_z,), dtype=np.complex128)
        g[..., :p.K + 1] = x[..., p.K:]
        g[..., p.N_z - p.K:] = x[..., :p.K]
        g = sfft.ifft(g, axis=-1, norm="forward", workers=self.workers)
        h = np.zeros(x.shape[:-2] + (p.N_theta // 2 + 1, p.N_z), dtype=np.complex128)
        h[..., :p.M_theta, :] = g
        return torch.from_numpy(sfft.irfft(h, n=p.N_theta, axis=-2, norm="forward",
                                           workers=self.workers))

    def to_spectral(self, f):
        """Real [..., N_theta, N_z] -> retained modes, as tc.to_spectral."""
        p = self.p
        a = sfft.rfft(f.numpy(), axis=-2, norm="forward", workers=self.workers)[..., :p.M_theta, :]
        a = sfft.fft(a, axis=-1, norm="forward", workers=self.workers)
        return torch.from_numpy(np.concatenate([a[..., p.N_z - p.K:], a[..., :p.K + 1]], axis=-1))

    def nonlinear(self, u):
        p = self.p
        r, D1 = self.r, self.D1
        mean = u[:, :, 0, p.K].real
        up = u.clone()
        up[:, :, 0, p.K] = 0.0
        spec = tc.derived_fields(p, up, D1, r)
        phys = self.to_physical(spec)
        ur, ut, uz, wr, wt, wz = phys[:6]
        outs = [ut * wz - uz * wt, uz * wr - ur * wz, ur * wt - ut * wr]
        if p.heated:
            gr, gt, gz = phys[6:9]
            outs.append(-(ur * gr + ut * gt + uz * gz))
        N = self.to_spectral(torch.stack(outs))
        Ur, V, W = mean[0], mean[1], mean[2]
        Om_t = -(D1 @ W)
        Om_z = D1 @ V + V / r
        col = lambda x: x[:, None, None].to(C128)  # noqa: E731
        cUr, cV, cW, cOt, cOz = col(Ur), col(V), col(W), col(Om_t), col(Om_z)
        pr, pt, pz, qr, qt, qz = spec[:6]
        N[0] = N[0] + cV * qz - cW * qt + pt * cOz - pz * cOt
        N[1] = N[1] + cW * qr - cUr * qz - pr * cOz
        N[2] = N[2] + cUr * qt - cV * qr + pr * cOt
        N[0, :, 0, p.K] += V * Om_z - W * Om_t
        N[1, :, 0, p.K] -= Ur * Om_z
        N[2, :, 0, p.K] += Ur * Om_t
        if p.heated:
            G = D1 @ mean[3]
            cG = col(G)
            g1, g2, g3 = spec[6:9]
            N[3] = N[3] - (cUr * g1 + cV * g2 + cW * g3 + pr * cG)
            N[3, :, 0, p.K] -= Ur * G
            N[2] = N[2] + p.Gr * u[3]
        # CFL bound on the padded grid from the full velocity
        rr = r[:, None, None]
        aur = (ur + Ur[:, None, None]).abs()
        aut = (ut + V[:, None, None]).abs()
        auz = (uz + W[:, None, None]).abs()
        dr = tc._spacings(p, r)[:, None, None]
        inf = torch.tensor(math.inf, dtype=F64)
        cand = torch.stack([
            torch.where(aur > 0, dr / aur, inf),
            torch.where(aut > 0, rr * (2.0 * math.pi / p.N_theta) / aut, inf),
            torch.where(auz > 0, (p.L_z / p.N_z) / auz, inf)])
        return tc.herm(p, N), float(cand.min())

    # ------------------------------------------------------------------
    # predictor--corrector step (tc.step with one corrector stage)
    # ------------------------------------------------------------------
    def step(self, u, dt, c=0.5):
        Nn, dt_cfl = self.nonlinear(u)
        X = self.radial_solve(u, Nn, Nn, dt, c)
        Nq, _ = self.nonlinear(X)
        X = self.radial_solve(u, Nn, Nq, dt, c)
        return X, dt_cfl
