"""Pins of the oracle's heated-flow diagnostics (section 3: Nusselt number at
the inner cylinder, velocity probe series) against closed forms: the basic
state conducts heat with Nu = 1 at both walls, Couette flow carries the same
torque 4 pi L_z B through both walls, and the probe sum reproduces the
oracle's transform to the padded physical grid at its grid points."""
import math

import pytest
import torch

import oracle as O
from synthetic import direction


@pytest.mark.parametrize("n", [32, 64])
def test_basic_state_nusselt_and_torque(n):
    p = O.Params(0.71, 50.0, -10.0, 2130.0, 0.7, n, 4, 7, 2 * math.pi)
    nu_i, nu_o, g_i, g_o = O.diagnostics(p, O.base_state(p))
    lam = 4.0 * math.pi * p.L_z * p.B
    tol = 1e-9 if n == 32 else 1e-12
    assert abs(nu_i - 1.0) < tol and abs(nu_o - 1.0) < tol
    assert abs(g_i - lam) < tol * abs(lam) and abs(g_o - lam) < tol * abs(lam)


def test_isothermal_has_no_nusselt():
    p = O.Params(0.5, 50.0, 0.0, 0.0, 1.0, 16, 4, 7, 2 * math.pi)
    nu_i, nu_o, _, _ = O.diagnostics(p, O.base_state(p))
    assert nu_i == 0.0 and nu_o == 0.0


def test_perturbation_changes_the_wall_fluxes_only_through_mode_00():
    p = O.Params(0.71, 50.0, 0.0, 2130.0, 0.7, 16, 4, 7, 2 * math.pi)
    u = O.base_state(p)
    d = direction(p.F, p.N_r, p.M_theta, p.M_z, 3)
    d[:, :, 0, p.K] = 0.0
    assert O.diagnostics(p, u + 1e-2 * d) == O.diagnostics(p, u)


def test_probe_matches_transform_at_grid_points():
    p = O.Params(0.71, 50.0, 0.0, 2130.0, 0.7, 12, 5, 9, 3.0)
    u = O.base_state(p) + 1e-2 * direction(p.F, p.N_r, p.M_theta, p.M_z, 4)
    phys = O.to_physical(p, u)  # [F][N_r][N_theta][N_z]
    rows, th, zz, want = [], [], [], []
    for (j, a, b) in [(0, 0, 0), (5, 3, 7), (11, 14, 2), (7, 9, 13)]:
        rows.append(j)
        th.append(2 * math.pi * a / p.N_theta)
        zz.append(p.L_z * b / p.N_z)
        want.append(phys[:, j, a, b])
    got = O.probe(p, u, rows, th, zz)
    want = torch.stack(want)
    assert float((got - want).abs().max() / want.abs().max()) < 1e-13
