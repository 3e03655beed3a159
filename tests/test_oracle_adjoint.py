"""Pins for the oracle's gradient (PyTorch autograd through the FP64 oracle):
central finite differences along seeded directions, and the exact
quadratic energy gradient.  CPU only."""
import math

import torch

import oracle as O
from synthetic import direction, mode_amplitudes


def test_energy_gradient_closed_form():
    """dE/du = 2 pi L_z w_j r_j c_m (u - U_b) for the velocity."""
    p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, 12, 4, 7, 3.0)
    u = O.base_state(p) + 1e-2 * direction(p.F, p.N_r, p.M_theta, p.M_z, 3)
    x = u.clone().requires_grad_(True)
    O.energy(p, x).backward()
    r = O.radial_grid(p)
    w = O.cc_weights(p, r)
    cm = torch.full((p.M_theta,), 2.0, dtype=torch.float64)
    cm[0] = 1.0
    ref = 2 * math.pi * p.L_z * (w * r)[None, :, None, None] * cm[None, None, :, None] \
        * (u - O.base_state(p))
    assert float((x.grad - ref).abs().max()) <= 1e-14 * float(ref.abs().max())


def test_rollout_gradient_central_differences():
    """Autograd gradient of E(u^S) agrees with FP64 central differences along
    seeded directions (O(eps^2) truncation, eps relative 1e-3)."""
    p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, 12, 4, 7, 2 * math.pi)
    u0 = O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, 1e-2, seed=1000))
    steps, dt = 5, 1e-3
    x = u0.clone().requires_grad_(True)
    uS, _ = O.run(p, x, steps, dt0=dt)
    O.energy(p, uS).backward()
    pert = float(torch.linalg.vector_norm(u0 - O.base_state(p)))
    with torch.no_grad():
        for s in range(2000, 2004):
            d = direction(p.F, p.N_r, p.M_theta, p.M_z, s)
            d = d * (1e-3 * pert / float(torch.linalg.vector_norm(d)))
            ep = float(O.energy(p, O.run(p, u0 + d, steps, dt0=dt)[0]))
            em = float(O.energy(p, O.run(p, u0 - d, steps, dt0=dt)[0]))
            fd = (ep - em) / 2
            an = float((x.grad.conj() * d).real.sum())
            assert abs(fd - an) <= 1e-7 * abs(fd), (s, fd, an)
