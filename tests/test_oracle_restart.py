"""Pins of the oracle's restart with a change of resolution (section 2.1:
interpolation and mode padding at a restart) against what the mathematics
fixes: the identity at equal resolution, exact reproduction of polynomial
radial profiles of degree < N_r (evaluated independently as Chebyshev series
with numpy), the Couette profile A r + B/r to rounding, wall values kept,
mode padding followed by truncation as the identity, the energy (Parseval)
unchanged by padding, and the Hermitian m = 0 column preserved."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from synthetic import direction


def _p(N_r, M_theta, M_z, Ra=0.0):
    return O.Params(0.71, 100.0, -20.0, Ra, 0.7, N_r, M_theta, M_z, 2 * math.pi)


def test_identity_at_equal_resolution():
    p = _p(13, 5, 9, Ra=1e3)
    u = direction(p.F, p.N_r, p.M_theta, p.M_z, 3)
    assert torch.equal(O.remap_state(p, u, p.N_r), u)


@pytest.mark.parametrize("n0,n1", [(9, 17), (17, 9), (16, 33), (33, 20)])
def test_polynomial_profiles_reproduced(n0, n1):
    """Profiles that are polynomials of degree n0 - 1 in r (random Chebyshev
    coefficients on [r_i, r_o]) land on the new grid exactly, to rounding;
    a transposed or shifted interpolation matrix fails this."""
    src, dst = _p(n0, 2, 3), _p(n1, 2, 3)
    rng = np.random.default_rng(5)
    coef = rng.standard_normal((src.F, n0, 2, 3)) + 1j * rng.standard_normal((src.F, n0, 2, 3))
    coef[:, :, 0, 1] = coef[:, :, 0, 1].real  # (0,0) real; (0,+-1) conjugate pair
    coef[:, :, 0, 0] = np.conj(coef[:, :, 0, 2])

    def values(p):
        r = O.radial_grid(p).numpy()
        x = (2 * r - (p.r_i + p.r_o)) / (p.r_o - p.r_i)
        out = np.zeros((p.F, p.N_r, 2, 3), dtype=complex)
        for f in range(p.F):
            for m in range(2):
                for k in range(3):
                    out[f, :, m, k] = np.polynomial.chebyshev.chebval(x, coef[f, :, m, k])
        return torch.from_numpy(out)

    got = O.remap_state(dst, values(src), n0)
    want = values(dst)
    assert float((got - want).abs().max() / want.abs().max()) < 1e-12


def test_couette_profile_and_walls():
    src, dst = _p(33, 3, 5), _p(48, 4, 7)
    u = O.base_state(src)
    got = O.remap_state(dst, u, src.N_r)
    want = O.base_state(dst)
    assert float((got - want).abs().max() / want.abs().max()) < 1e-12
    # both grids contain the walls: their values are copied, not interpolated
    v = direction(src.F, src.N_r, src.M_theta, src.M_z, 4)
    w = O.remap_state(dst, v, src.N_r)
    assert torch.equal(w[:, 0, :3, 1:6], v[:, 0, :, :])
    assert torch.equal(w[:, -1, :3, 1:6], v[:, -1, :, :])


def test_padding_then_truncation_is_identity():
    small, big = _p(12, 3, 5, Ra=1e3), _p(12, 6, 11, Ra=1e3)
    u = direction(small.F, small.N_r, small.M_theta, small.M_z, 6)
    up = O.remap_state(big, u, 12)
    # new modes are zero, kept ones at their (m, k)
    assert torch.equal(up[:, :, 3:], torch.zeros_like(up[:, :, 3:]))
    assert torch.equal(up[:, :, :, :3], torch.zeros_like(up[:, :, :, :3]))
    assert torch.equal(up[:, :, :3, 3:8], u)
    assert torch.equal(O.remap_state(small, up, 12), u)


def test_energy_unchanged_by_padding():
    small, big = _p(14, 3, 5), _p(14, 5, 9)
    u = O.base_state(small) + 1e-2 * direction(small.F, small.N_r, small.M_theta, small.M_z, 7)
    e0 = float(O.energy(small, u))
    e1 = float(O.energy(big, O.remap_state(big, u, small.N_r)))
    assert abs(e1 - e0) <= 1e-14 * e0


def test_hermitian_column_preserved():
    src, dst = _p(11, 2, 5), _p(19, 3, 9)
    u = direction(src.F, src.N_r, src.M_theta, src.M_z, 8)
    w = O.remap_state(dst, u, src.N_r)
    K = dst.K
    for k in range(1, K + 1):
        assert torch.allclose(w[:, :, 0, K - k], w[:, :, 0, K + k].conj(), rtol=0, atol=1e-15)
