"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Holds random draws and the input recipe only -- none of the
method's arithmetic (no grid, no operators, no transforms).

Recipe (initial conditions of the Taylor--Couette workloads): complex
Gaussian mode amplitudes xi with independent real and imaginary parts of
variance 1/2, scaled by amp * exp(-sqrt(m^2 + k^2) / 4); mode (0,0) is zero
and the m = 0 column is made Hermitian, xi(0,-k) = conj xi(0,k), so that the
amplitudes describe a real field.  Draws come from numpy's PCG64 generator.
"""
import math

import numpy as np
import torch

__all__ = ["complex_normal", "mode_amplitudes", "direction"]


def complex_normal(shape, seed):
    """Complex normal array with Re, Im ~ N(0, 1/2), numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return torch.from_numpy((re + 1j * im) * math.sqrt(0.5))


def _hermitian_m0(x, K):
    x = x.clone()
    for k in range(1, K + 1):
        x[..., 0, K - k] = x[..., 0, K + k].conj()
    x[..., 0, K] = 0.0
    return x


def mode_amplitudes(F, M_theta, M_z, amp, seed):
    """[F][M_theta][M_z] complex128 mode amplitudes (see module docstring)."""
    K = (M_z - 1) // 2
    xi = complex_normal((F, M_theta, M_z), seed)
    m = torch.arange(M_theta, dtype=torch.float64)[:, None]
    k = (torch.arange(M_z, dtype=torch.float64) - K)[None, :]
    env = amp * torch.exp(-torch.sqrt(m * m + k * k) / 4.0)
    return _hermitian_m0(xi * env[None], K)


def direction(F, N_r, M_theta, M_z, seed):
    """A seeded random direction [F][N_r][M_theta][M_z] (complex normal,
    m = 0 column Hermitian) for finite-difference checks."""
    K = (M_z - 1) // 2
    xi = complex_normal((F, N_r, M_theta, M_z), seed)
    out = xi.clone()
    for k in range(1, K + 1):
        out[..., 0, K - k] = out[..., 0, K + k].conj()
    out[..., 0, K] = out[..., 0, K].real.to(out.dtype)
    return out
