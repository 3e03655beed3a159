"""The faster CPU evaluation of the step (oracle.fast) against the plain
oracle (oracle.tc): FFTs for DFT matrices, inverses kept per step size
for dense per-call solves -- the same arithmetic up to rounding order."""
import math

import pytest
import torch

import oracle as O
from oracle.fast import Stepper
from synthetic import mode_amplitudes

CASES = {
    "tiny": (0.5, 50.0, 0.0, 0.0, 1.0, 12, 4, 7, 2 * math.pi),
    "heated": (0.71, 100.0, -20.0, 1.0e4, 0.7, 16, 8, 15, 2 * math.pi),
    "ragged": (0.6, 80.0, 10.0, 0.0, 1.0, 13, 5, 9, 4.0),
}


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def _rel_fluct(p, a, b):
    """Relative to the modes other than (0,0), which the basic state and
    the base-flow terms would otherwise dominate in the maximum."""
    fl = torch.ones(p.M_theta, p.M_z, dtype=torch.bool)
    fl[0, p.K] = False
    return float((a - b)[..., fl].abs().max() / b[..., fl].abs().max())


def _state(p, amp=5e-2, seed=1000):
    return O.initial_state(p, mode_amplitudes(p.F, p.M_theta, p.M_z, amp, seed=seed))


@pytest.mark.parametrize("case", list(CASES))
def test_transforms_match_dft_matrices(case):
    p = O.Params(*CASES[case])
    s = Stepper(p, workers=2)
    g = torch.Generator().manual_seed(7)
    spec = torch.complex(torch.randn(3, p.M_theta, p.M_z, generator=g, dtype=torch.float64),
                         torch.randn(3, p.M_theta, p.M_z, generator=g, dtype=torch.float64))
    ref = O.to_physical(p, spec)
    got = s.to_physical(spec)
    assert _rel(got, ref) < 1e-13
    f = torch.randn(3, p.N_theta, p.N_z, generator=g, dtype=torch.float64)
    assert _rel(s.to_spectral(f), O.to_spectral(p, f)) < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_nonlinear_matches_oracle(case):
    p = O.Params(*CASES[case])
    u = _state(p)
    ref, dref = O.nonlinear(p, u)
    got, dgot = Stepper(p, workers=2).nonlinear(u)
    assert _rel_fluct(p, got, ref) < 1e-12
    assert _rel(got, ref) < 1e-13
    assert dgot == pytest.approx(dref, rel=1e-14)


@pytest.mark.parametrize("case", list(CASES))
def test_radial_solve_matches_oracle(case):
    p = O.Params(*CASES[case])
    u = _state(p)
    Nn, _ = O.nonlinear(p, u)
    Nq, _ = O.nonlinear(p, _state(p, seed=1001))
    ref, _ = O.radial_solve(p, u, Nn, Nq, 2e-3)
    got = Stepper(p, workers=2).radial_solve(u, Nn, Nq, 2e-3)
    assert _rel(got, ref) < 1e-13
    assert _rel_fluct(p, got, ref) < 1e-11


def test_steps_with_a_step_size_change_match_oracle():
    """Two steps at one size, one at another: the factorisations are
    redone on the change."""
    p = O.Params(*CASES["heated"])
    u = _state(p)
    s = Stepper(p, workers=2)
    ref = got = u
    for dt in (1e-3, 1e-3, 6e-4):
        ref, dref = O.step(p, ref, dt)
        got, dgot = s.step(got, dt)
        assert dgot == pytest.approx(dref, rel=1e-12)
    assert s.dt == (6e-4, 0.5)
    assert _rel(got, ref) < 1e-13
    assert _rel_fluct(p, got, ref) < 1e-11
