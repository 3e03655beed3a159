"""The radial operators can be factorised without pivoting (CPU check of the
choice the HIP library makes; the oracle itself solves with pivoted LU).

Gaussian elimination without row exchanges is backward stable when the
growth factor rho = max over the elimination steps of |a_ij^(k)| / max |a_ij|
stays O(1) (Wilkinson's bound: the backward error is at most about
n * rho * eps * |A|).  This test eliminates every operator family the
library factorises -- the Helmholtz operators I/dt - beta L_q with identity
(Dirichlet) wall rows, the pressure Poisson operators L_q with D1 (Neumann)
wall rows, and the mean pressure-head operator -- over radius ratios
0.1..0.9, 9..256 radial points, azimuthal orders, axial wavenumbers and step
sizes spanning the configured workloads and beyond, and checks that rho
stays below 1.1 and that the unpivoted solutions agree with pivoted LU to
the conditioning limit.  Operators come from the oracle's nine-point D1, D2
on the Chebyshev--Gauss--Lobatto grid.
"""
import math

import numpy as np
import pytest

import oracle as O

QS = (0, 1, 2, 5, 40, 300)
KAPS = (0.0, 1.3, 20.0, 300.0)
DTS = (1e-5, 1e-3, 1e-1)
BETAS = (0.5, 0.5 / 0.7)  # velocity c, temperature c/Pr


def _operators(eta, n):
    p = O.Params(eta, 0.0, 0.0, 0.0, 1.0, n, 4, 7, 2 * math.pi)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    D1, D2, r = D1.numpy(), D2.numpy(), r.numpy()
    base = D2 + D1 / r[:, None]
    mats = []
    for q in QS:
        for kap in KAPS:
            L = base - np.diag(q * q / r ** 2) - kap * kap * np.eye(n)
            for dt in DTS:
                for beta in BETAS:
                    H = np.eye(n) / dt - beta * L
                    H[[0, -1]] = 0.0
                    H[0, 0] = H[-1, -1] = 1.0
                    mats.append(H)
            if q == 0 and kap == 0.0:  # pure Neumann is singular: the mean head
                P = base.copy()
                P[0] = 0.0
                P[0, 0] = 1.0
                P[-1] = D1[-1]
            else:
                P = L.copy()
                P[0] = D1[0]
                P[-1] = D1[-1]
            mats.append(P)
    return np.array(mats)


def _eliminate(A):
    """Batched LU without pivoting of band matrices whose rows reach at most
    8 columns either side of the diagonal (nine-point windows, one-sided at
    the walls): returns (packed L\\U, growth factor per matrix)."""
    A = A.copy()
    B, n, _ = A.shape
    amax = np.abs(A).reshape(B, -1).max(axis=1)
    grow = amax.copy()
    for k in range(n - 1):
        hi = min(n, k + 9)
        lk = A[:, k + 1:hi, k] / A[:, k:k + 1, k]
        A[:, k + 1:hi, k:hi] -= lk[:, :, None] * A[:, k:k + 1, k:hi]
        A[:, k + 1:hi, k] = lk
        grow = np.maximum(grow, np.abs(A[:, k + 1:hi, k + 1:hi]).reshape(B, -1).max(axis=1))
    return A, grow / amax


def _solve_packed(LU, b):
    B, n, _ = LU.shape
    y = b.copy()
    for i in range(1, n):
        y[:, i] -= np.einsum('bj,bj->b', LU[:, i, :i], y[:, :i])
    x = y
    for i in range(n - 1, -1, -1):
        x[:, i] = (x[:, i] - np.einsum('bj,bj->b', LU[:, i, i + 1:], x[:, i + 1:])) / LU[:, i, i]
    return x


def test_elimination_stays_in_the_band():
    """Without row exchanges no fill appears outside the nine-point envelope
    (8 sub- and super-diagonals), which is what lets the factors live in it."""
    A = _operators(0.5, 24)
    LU, _ = _eliminate(A)
    full = A.copy()
    for k in range(24 - 1):
        lk = full[:, k + 1:, k] / full[:, k:k + 1, k]
        full[:, k + 1:, k:] -= lk[:, :, None] * full[:, k:k + 1, k:]
        full[:, k + 1:, k] = lk
    assert np.allclose(full, LU, rtol=1e-12, atol=1e-12 * np.abs(A).max())


@pytest.mark.parametrize("n", [9, 17, 33, 64, 128, 256])
@pytest.mark.parametrize("eta", [0.1, 0.3, 0.5, 0.71, 0.9])
def test_growth_factor_and_agreement_with_pivoted_lu(eta, n):
    A = _operators(eta, n)
    LU, rho = _eliminate(A)
    assert float(rho.max()) < 1.1, float(rho.max())
    rng = np.random.default_rng(1000 + n)
    b = rng.standard_normal((A.shape[0], n))
    x = _solve_packed(LU, b)
    ref = np.linalg.solve(A, b[:, :, None])[:, :, 0]
    inv = np.linalg.inv(A)
    cond = np.abs(A).sum(axis=1).max(axis=1) * np.abs(inv).sum(axis=1).max(axis=1)  # inf-norm
    err = np.abs(x - ref).max(axis=1) / np.abs(ref).max(axis=1)
    bound = 4.0 * n * np.finfo(np.float64).eps * cond
    assert bool((err <= np.maximum(bound, 1e-14)).all()), float((err / bound).max())
