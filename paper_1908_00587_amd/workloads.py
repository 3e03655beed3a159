"""Named Taylor--Couette workloads (synthetic, seeded).

Each entry: physical parameters for nsc_init, the perturbation amplitude of
the seeded initial condition, the time-step policy and the step count.  The
sizes follow the paper's classes of problems (section 2.3: N_r = 64 and 128
on one GPU; N_r = 512 with 513 x 1025 modes on a cluster).
"""
import math

TWO_PI = 2.0 * math.pi

WORKLOADS = {
    # tiny grid for brute-force checks
    "tiny": dict(eta=0.5, Re_i=50.0, Re_o=0.0, Ra=0.0, Pr=1.0, N_r=12, M_theta=4, M_z=7,
                 L_z=TWO_PI, amp=1e-2, amp_T=0.0, dt=1e-3, dynamic=False, steps=10, seed=999),
    # isothermal, plain FP64: Re_i = 50, 32 points, 16 x 31 modes -> 48 x 48
    "tc-iso-n32": dict(eta=0.5, Re_i=50.0, Re_o=0.0, Ra=0.0, Pr=1.0, N_r=32, M_theta=16,
                       M_z=31, L_z=TWO_PI, amp=1e-3, amp_T=0.0, dt=1e-3, dynamic=False,
                       steps=100, seed=1000),
    # heated: Ra = 1e4, Pr = 0.7, 64 points, 64 x 127 modes -> 192 x 192, CFL 0.5
    "tc-heated-n64": dict(eta=0.71, Re_i=100.0, Re_o=0.0, Ra=1.0e4, Pr=0.7, N_r=64,
                          M_theta=64, M_z=127, L_z=TWO_PI, amp=1e-3, amp_T=1e-3, dt=1e-3,
                          dynamic=True, steps=200, seed=1001),
    # adjoint workload: Re_i = 200, 64 points, 32 x 63 modes, dt = 5e-4
    "tc-adjoint-n64": dict(eta=0.71, Re_i=200.0, Re_o=0.0, Ra=0.0, Pr=1.0, N_r=64,
                           M_theta=32, M_z=63, L_z=TWO_PI, amp=1e-3, amp_T=0.0, dt=5e-4,
                           dynamic=False, steps=200, seed=1002),
    # counter-rotating turbulent: Re_i = 2000, Re_o = -1000, 128 points, 256 x 511 modes
    "tc-turb-n128": dict(eta=0.71, Re_i=2000.0, Re_o=-1000.0, Ra=0.0, Pr=1.0, N_r=128,
                         M_theta=256, M_z=511, L_z=TWO_PI, amp=1e-2, amp_T=0.0, dt=1e-3,
                         dynamic=True, steps=500, seed=1003),
    # large convective: Ra = 1e6, 256 points, 512 x 1023 modes -> 1536 x 1536
    "tc-conv-n256": dict(eta=0.5, Re_i=1000.0, Re_o=0.0, Ra=1.0e6, Pr=0.7, N_r=256,
                         M_theta=512, M_z=1023, L_z=TWO_PI, amp=1e-3, amp_T=1e-3, dt=1e-3,
                         dynamic=True, steps=100, seed=1004),
    # pipe flow (nsc_init_pipe): centreline speed Re = 4000 of the laminar
    # flow, 64 points axis to wall, 64 x 127 modes -> 192 x 192, period
    # 4 pi (about six diameters), CFL 0.5
    "pipe-n64": dict(geometry="pipe", Re=4000.0, Ra=0.0, N_r=64, M_theta=64, M_z=127,
                     L_z=2 * TWO_PI, amp=1.0, amp_T=0.0, dt=1e-4, dynamic=True, steps=200,
                     seed=1005),
}


def is_pipe(name):
    return WORKLOADS[name].get("geometry") == "pipe"


def pipe_params(name):
    """(Re, N_r, M_theta, M_z, L_z) of a pipe workload (nsc_init_pipe)."""
    w = WORKLOADS[name]
    return (w["Re"], w["N_r"], w["M_theta"], w["M_z"], w["L_z"])


def params(name):
    w = WORKLOADS[name]
    return (w["eta"], w["Re_i"], w["Re_o"], w["Ra"], w["Pr"], w["N_r"], w["M_theta"],
            w["M_z"], w["L_z"])


def amplitudes(name):
    """Seeded mode amplitudes [F][M_theta][M_z] of the workload's initial state
    (velocity amplitude amp, temperature amplitude amp_T)."""
    import torch

    from synthetic import mode_amplitudes
    w = WORKLOADS[name]
    F = 4 if w["Ra"] != 0 else 3
    a = mode_amplitudes(F, w["M_theta"], w["M_z"], 1.0, seed=w["seed"])
    scale = torch.tensor([w["amp"]] * 3 + ([w["amp_T"]] if F == 4 else []), dtype=torch.float64)
    return a * scale[:, None, None]
