"""Pins for the oracle's Fourier transforms and 3/2-rule dealiasing
(pseudospectral Fourier--Galerkin in theta and z, section 2.1).  CPU only."""
import math

import numpy as np
import pytest
import torch

import oracle as O


def _p(Mt=4, Mz=7):
    return O.Params(0.5, 0.0, 0.0, 0.0, 1.0, 9, Mt, Mz, 2.0)


def _rand_spec(p, gen, lead=()):
    x = torch.complex(torch.randn(*lead, p.M_theta, p.M_z, generator=gen, dtype=torch.float64),
                      torch.randn(*lead, p.M_theta, p.M_z, generator=gen, dtype=torch.float64))
    return O.herm(p, x)


@pytest.mark.parametrize("Mt,Mz", [(4, 7), (16, 31), (5, 9)])
def test_round_trip(Mt, Mz):
    p = _p(Mt, Mz)
    g = torch.Generator().manual_seed(1)
    x = _rand_spec(p, g, (3,))
    y = O.to_spectral(p, O.to_physical(p, x))
    assert float((y - x).abs().max()) < 1e-14 * float(x.abs().max())


def test_inverse_matches_numpy_fft():
    """Inverse transform = numpy's unnormalised 2-D inverse FFT of the
    Hermitian-extended, zero-padded spectrum."""
    p = _p(4, 7)
    g = torch.Generator().manual_seed(2)
    x = _rand_spec(p, g)
    full = np.zeros((p.N_theta, p.N_z), dtype=np.complex128)
    xn = x.numpy()
    for m in range(p.M_theta):
        for kk in range(p.M_z):
            k = kk - p.K
            full[m % p.N_theta, k % p.N_z] += xn[m, kk]
            if m > 0:
                full[(-m) % p.N_theta, (-k) % p.N_z] += np.conj(xn[m, kk])
    ref = np.fft.ifft2(full) * (p.N_theta * p.N_z)
    assert np.abs(ref.imag).max() < 1e-13
    got = O.to_physical(p, x).numpy()
    assert np.abs(got - ref.real).max() < 1e-13


def test_forward_matches_numpy_fft():
    p = _p(4, 7)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((p.N_theta, p.N_z))
    ref = np.fft.fft2(f) / (p.N_theta * p.N_z)
    got = O.to_spectral(p, torch.from_numpy(f)).numpy()
    for m in range(p.M_theta):
        for kk in range(p.M_z):
            k = kk - p.K
            assert abs(got[m, kk] - ref[m, k % p.N_z]) < 1e-15


def test_parseval():
    """Mean of f^2 over the padded grid equals sum c_m |f_mk|^2."""
    p = _p(6, 11)
    g = torch.Generator().manual_seed(4)
    x = _rand_spec(p, g)
    f = O.to_physical(p, x)
    cm = torch.full((p.M_theta,), 2.0, dtype=torch.float64)
    cm[0] = 1.0
    lhs = float((f ** 2).mean())
    rhs = float(((x.abs() ** 2) * cm[:, None]).sum())
    assert abs(lhs - rhs) < 1e-13 * rhs


def test_dealiased_product_equals_galerkin_convolution():
    """Brute force: the pseudospectral product of two band-limited real fields,
    truncated to the retained modes, equals the exact convolution sum over
    the two-sided spectra restricted to |m| < M_theta, |k| <= K."""
    p = _p(4, 7)
    g = torch.Generator().manual_seed(5)
    a = _rand_spec(p, g)
    b = _rand_spec(p, g)
    ps = O.to_spectral(p, O.to_physical(p, a) * O.to_physical(p, b)).numpy()

    def two_sided(x):
        d = {}
        xn = x.numpy()
        for m in range(p.M_theta):
            for kk in range(p.M_z):
                k = kk - p.K
                d[(m, k)] = d.get((m, k), 0) + xn[m, kk]
                if m > 0:
                    d[(-m, -k)] = d.get((-m, -k), 0) + np.conj(xn[m, kk])
        return d

    A = two_sided(a)
    B = two_sided(b)
    for m in range(p.M_theta):
        for kk in range(p.M_z):
            k = kk - p.K
            s = 0j
            for (m1, k1), v1 in A.items():
                v2 = B.get((m - m1, k - k1))
                if v2 is not None:
                    s += v1 * v2
            assert abs(ps[m, kk] - s) < 1e-13, (m, k)


def test_herm_projection_is_self_adjoint_and_idempotent():
    p = _p(4, 7)
    g = torch.Generator().manual_seed(6)
    x = torch.complex(torch.randn(4, 7, generator=g, dtype=torch.float64),
                      torch.randn(4, 7, generator=g, dtype=torch.float64))
    y = torch.complex(torch.randn(4, 7, generator=g, dtype=torch.float64),
                      torch.randn(4, 7, generator=g, dtype=torch.float64))
    hx = O.herm(p, x)
    assert float((O.herm(p, hx) - hx).abs().max()) < 1e-15
    lhs = float((hx.conj() * y).real.sum())
    rhs = float((x.conj() * O.herm(p, y)).real.sum())
    assert abs(lhs - rhs) < 1e-13
    assert abs(float(hx[0, p.K].imag)) < 1e-16
    assert math.isclose(float(hx[0, p.K + 1].real), float(hx[0, p.K - 1].real))
