"""FP64 CPU oracle for the Taylor--Couette time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (no kernels, headers, helpers or constant tables).

The oracle is a plain, slow, obviously correct statement of the method of
the nsCouette paper (Lopez, Feldmann, Rampp, Vela-Martin, Shi, Avila):
Fourier--Galerkin in theta and z with 3/2-rule dealiased pseudospectral
products, high-order (9-point) finite differences in r, a predictor--corrector
time integrator with variable time step, Boussinesq heat transfer, and
divergence-free initial conditions (Functionality, section 2.1).  The paper
prints no equations; every formula here is a reading of its description,
stated where the formula is written.  Floating point is IEEE FP64 throughout.
Transforms are explicit DFT matrices (dense matmul), the radial systems are
dense LU solves (``torch.linalg.solve``), the time step is the explicit
predictor--corrector loop.  Written in plain PyTorch CPU ops so that autograd
provides an independent gradient for the adjoint tests.

``oracle.fast`` evaluates the same step faster on the host (FFTs, radial
systems inverted once per step size) for the benchmark's CPU reference
figure; the CPU tests hold it to ``oracle.tc``.
"""
from .tc import (  # noqa: F401
    Params, radial_grid, fornberg, fd_matrices, cc_weights, to_physical,
    to_spectral, herm, derived_fields, nonlinear, nonlinear_planes,
    nonlinear_planes_direct,
    l_operator, radial_solve, radial_solve_modes, step, next_dt, run,
    energy, base_state, initial_state, cfl_dt, weighted_norm,
    lagrange_matrix, remap_state, diagnostics, probe,
)
