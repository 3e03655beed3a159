"""Pins for the oracle's radial grid, finite-difference weights and radial
quadrature (nine-point FD in r, section 2.1).  CPU only."""
import math

import pytest
import torch

import oracle as O


def _p(n, eta=0.5):
    return O.Params(eta, 0.0, 0.0, 0.0, 1.0, n, 4, 7, 1.0)


def test_grid_endpoints_and_clustering():
    p = _p(33)
    r = O.radial_grid(p)
    assert abs(float(r[0]) - p.r_i) < 1e-14 and abs(float(r[-1]) - p.r_o) < 1e-14
    d = r[1:] - r[:-1]
    assert bool((d > 0).all())
    # Chebyshev clustering: wall spacing ~ (pi/(N-1))^2/4, mid spacing ~ pi/(2(N-1))
    assert float(d[0]) < 0.1 * float(d[16])


@pytest.mark.parametrize("n", [9, 12, 32, 64])
def test_fd_exact_on_polynomials(n):
    """D1, D2 are exact on polynomials of degree <= 8 (nine-point windows)."""
    p = _p(n)
    r = O.radial_grid(p)
    D1, D2 = O.fd_matrices(p, r)
    for deg in range(9):
        f = r ** deg
        d1 = deg * r ** (deg - 1) if deg >= 1 else torch.zeros_like(r)
        d2 = deg * (deg - 1) * r ** (deg - 2) if deg >= 2 else torch.zeros_like(r)
        # condition-aware scale: sum_i |w_i| |f_i|
        s1 = (D1.abs() @ f.abs()) + 1.0
        s2 = (D2.abs() @ f.abs()) + 1.0
        assert float(((D1 @ f - d1).abs() / s1).max()) < 1e-13
        assert float(((D2 @ f - d2).abs() / s2).max()) < 1e-13


def test_fd_textbook_uniform_weights():
    """On a uniform grid the centred nine-point weights are the textbook ones:
    D1: (4/5, -1/5, 4/105, -1/280), D2: (-205/72, 8/5, -1/5, 8/315, -1/560)."""
    xs = [float(i) for i in range(-4, 5)]
    w = O.fornberg(0.0, xs, 2)
    d1 = [w[i][1] for i in range(9)]
    d2 = [w[i][2] for i in range(9)]
    ref1 = [1 / 280, -4 / 105, 1 / 5, -4 / 5, 0.0, 4 / 5, -1 / 5, 4 / 105, -1 / 280]
    ref2 = [-1 / 560, 8 / 315, -1 / 5, 8 / 5, -205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560]
    for a, b in zip(d1, ref1):
        assert abs(a - b) < 1e-15
    for a, b in zip(d2, ref2):
        assert abs(a - b) < 1e-14
    # interpolation weights at a node are the Kronecker delta
    assert all(abs(w[i][0] - (1.0 if i == 4 else 0.0)) < 1e-15 for i in range(9))


@pytest.mark.parametrize("eta", [0.5, 0.1])
def test_fd_convergence_order(eta):
    """Smooth non-polynomial functions converge at >= 7th order as N_r grows
    (pre-asymptotic range, before rounding dominates)."""
    def f(r):
        return torch.sin(5 * r)

    def f1(r):
        return 5 * torch.cos(5 * r)

    def f2(r):
        return -25 * torch.sin(5 * r)

    errs = []
    ns = [24, 32, 48]
    for n in ns:
        p = _p(n, eta)
        r = O.radial_grid(p)
        D1, D2 = O.fd_matrices(p, r)
        errs.append((float((D1 @ f(r) - f1(r)).abs().max()),
                     float((D2 @ f(r) - f2(r)).abs().max())))
    for i in range(1, len(ns)):
        for c in range(2):
            order = math.log(errs[i - 1][c] / errs[i][c]) / math.log(ns[i] / ns[i - 1])
            assert order > 7.0, (ns[i], c, order)


@pytest.mark.parametrize("n", [9, 16, 33, 64])
def test_cc_weights_exact(n):
    """Clenshaw--Curtis on [r_i, r_o] integrates polynomials of degree < N_r
    exactly and sums to the gap width 1."""
    p = _p(n)
    r = O.radial_grid(p)
    w = O.cc_weights(p, r)
    assert abs(float(w.sum()) - 1.0) < 1e-14
    assert bool((w > 0).all())
    for deg in range(n):
        exact = (p.r_o ** (deg + 1) - p.r_i ** (deg + 1)) / (deg + 1)
        assert abs(float((w * r ** deg).sum()) - exact) < 1e-12 * max(1.0, exact)


def test_cc_weights_spectral_accuracy():
    p = _p(24)
    r = O.radial_grid(p)
    w = O.cc_weights(p, r)
    exact = math.exp(p.r_o) - math.exp(p.r_i)
    assert abs(float((w * torch.exp(r)).sum()) - exact) < 1e-13 * exact
