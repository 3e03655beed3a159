"""Python surface of the Taylor--Couette time-step library.

Thin wrapper over the C ABI in include/nsc.h: tensors provide device memory
and the HIP stream (torch.cuda.current_stream()), the library does the work.
All spectral arrays are torch.complex128 CUDA tensors, contiguous, shaped
[F][N_r][M_theta][M_z] (F = 4 with temperature, else 3).
"""
import ctypes

import torch

from . import _lib
from ._lib import NSC_FP64, NSC_MIXED, check


# kernel order of nsc_get_timings
KERNELS = ["zinv", "theta", "zfwd", "remap", "rhs", "div", "sweep_pt", "sweep_vel",
           "influence", "finalize", "factor", "vel_rhs"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, shape, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128:
        raise TypeError(f"{name} must be a complex128 tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Context:
    """One problem instance (nsc_init): radius ratio eta, wall speeds Re_i and
    Re_o, Rayleigh and Prandtl numbers (Ra = 0: isothermal), N_r radial points,
    M_theta azimuthal and M_z (odd) axial Fourier modes, axial period L_z."""

    def __init__(self, eta, Re_i, Re_o, Ra, Pr, N_r, M_theta, M_z, L_z, device=None):
        self._L = _lib.lib()
        if device is not None:
            torch.cuda.set_device(device)
        h = ctypes.c_void_p()
        check(self._L.nsc_init(float(eta), float(Re_i), float(Re_o), float(Ra), float(Pr),
                               int(N_r), int(M_theta), int(M_z), float(L_z), ctypes.byref(h)),
              "nsc_init")
        self._h = h
        self.eta, self.Re_i, self.Re_o, self.Ra, self.Pr = eta, Re_i, Re_o, Ra, Pr
        self.N_r, self.M_theta, self.M_z, self.L_z = N_r, M_theta, M_z, L_z
        self.F = 4 if Ra != 0 else 3
        self.shape = (self.F, N_r, M_theta, M_z)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._dt = 1e-3
        self._settings = dict(dt=1e-3, dynamic=0, cfl=0.5, dt_max=1e-3, n_corr=1, c=0.5)

    @classmethod
    def pipe(cls, Re, N_r, M_theta, M_z, L_z, device=None):
        """Pipe-flow context (nsc_init_pipe): radius 1, driven by the mean
        pressure gradient 4 Re (laminar flow Re (1 - r^2)), N_r radial points
        between the axis and the wall, M_theta x M_z Fourier modes, period L_z."""
        self = cls.__new__(cls)
        self._L = _lib.lib()
        if device is not None:
            torch.cuda.set_device(device)
        h = ctypes.c_void_p()
        check(self._L.nsc_init_pipe(float(Re), int(N_r), int(M_theta), int(M_z), float(L_z),
                                    ctypes.byref(h)), "nsc_init_pipe")
        self._h = h
        self.eta, self.Re_i, self.Re_o, self.Ra, self.Pr = None, Re, 0.0, 0.0, 1.0
        self.Re = Re
        self.N_r, self.M_theta, self.M_z, self.L_z = N_r, M_theta, M_z, L_z
        self.F = 3
        self.shape = (3, N_r, M_theta, M_z)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._dt = 1e-3
        self._settings = dict(dt=1e-3, dynamic=0, cfl=0.5, dt_max=1e-3, n_corr=1, c=0.5)
        return self

    # -- plumbing ---------------------------------------------------------------
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(self._L.nsc_set_stream(self._h, ctypes.c_void_p(s)), "nsc_set_stream")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.nsc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        return torch.empty(self.shape, dtype=torch.complex128, device=self.device)

    # -- settings -----------------------------------------------------------------
    def set_precision(self, mode):
        """'fp64' or 'mixed' (FP32 transforms/products, FP64 solves)."""
        code = {"fp64": NSC_FP64, "mixed": NSC_MIXED}[mode] if isinstance(mode, str) else int(mode)
        check(self._L.nsc_set_precision(self._h, code), "nsc_set_precision")

    def set_timestep(self, dt=1e-3, dynamic=False, cfl=0.5, dt_max=1e-3, n_corr=1, c=0.5):
        check(self._L.nsc_set_timestep(self._h, float(dt), int(bool(dynamic)), float(cfl),
                                       float(dt_max), int(n_corr), float(c)), "nsc_set_timestep")
        self._settings = dict(dt=dt, dynamic=int(bool(dynamic)), cfl=cfl, dt_max=dt_max,
                              n_corr=n_corr, c=c)

    def grid(self):
        buf = (ctypes.c_double * self.N_r)()
        check(self._L.nsc_get_grid(self._h, buf, self.N_r), "nsc_get_grid")
        return torch.tensor(list(buf), dtype=torch.float64)

    # -- the method -----------------------------------------------------------------
    def nonlinear(self, u, out=None, cfl=False):
        """N(u); with cfl=True also returns a 1-element device tensor dt_cfl."""
        _need(u, self.shape, "u")
        if out is None:
            out = self.empty()
        _need(out, self.shape, "out")
        c = torch.empty(1, dtype=torch.float64, device=self.device) if cfl else None
        self._sync_stream()
        check(self._L.nsc_nonlinear(self._h, _ptr(u), _ptr(out),
                                    _ptr(c) if c is not None else None), "nsc_nonlinear")
        return (out, c) if cfl else out

    def radial_solve(self, u_n, n_n, n_q, out=None, pressure=False):
        """Implicit stage with the step set by set_timestep; returns the new
        state (and the pressure head [N_r][M_theta][M_z] if pressure=True)."""
        for t, nm in ((u_n, "u_n"), (n_n, "n_n"), (n_q, "n_q")):
            _need(t, self.shape, nm)
        if out is None:
            out = self.empty()
        _need(out, self.shape, "out")
        p = None
        if pressure:
            p = torch.empty(self.shape[1:], dtype=torch.complex128, device=self.device)
        self._sync_stream()
        check(self._L.nsc_radial_solve(self._h, _ptr(u_n), _ptr(n_n), _ptr(n_q), _ptr(out),
                                       _ptr(p) if p is not None else None), "nsc_radial_solve")
        return (out, p) if pressure else out

    def step(self, u, dt):
        """Advance u in place by one step of size dt; returns the next dt."""
        _need(u, self.shape, "u")
        d = ctypes.c_double(float(dt))
        self._sync_stream()
        check(self._L.nsc_step(self._h, _ptr(u), ctypes.byref(d)), "nsc_step")
        return d.value

    # -- diagnostics (section 3: Nusselt number, probe series) -----------------------
    def diagnostics(self, u):
        """Device tensor [Nu_i, Nu_o, G_i, G_o]: Nusselt numbers (0 without
        temperature) and torques at the inner and outer walls."""
        _need(u, self.shape, "u")
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(self._L.nsc_diagnostics(self._h, _ptr(u), _ptr(out)), "nsc_diagnostics")
        return out

    def probe(self, u, rows, theta, z):
        """Device tensor [n][F]: every field at the points (r_rows, theta, z)."""
        _need(u, self.shape, "u")
        n = len(rows)
        if not (len(theta) == n and len(z) == n):
            raise ValueError("rows, theta and z must have the same length")
        out = torch.empty(n, self.F, dtype=torch.float64, device=self.device)
        R = (ctypes.c_int * n)(*[int(x) for x in rows])
        T = (ctypes.c_double * n)(*[float(x) for x in theta])
        Z = (ctypes.c_double * n)(*[float(x) for x in z])
        self._sync_stream()
        check(self._L.nsc_probe(self._h, _ptr(u), n, R, T, Z, _ptr(out)), "nsc_probe")
        return out

    # -- checkpoint-restart (section 2.1: resolution change at a restart) ------------
    def save_state(self, u, path, time=0.0):
        """Write u (context shape) and the context's parameters to a state file."""
        _need(u, self.shape, "u")
        self._sync_stream()
        check(self._L.nsc_save_state(self._h, _ptr(u), float(time), str(path).encode()),
              "nsc_save_state")

    def load_state(self, path, out=None):
        """Read a state file of this geometry, at any resolution, into the
        context's shape; returns (u, time)."""
        if out is None:
            out = self.empty()
        _need(out, self.shape, "out")
        t = ctypes.c_double(0.0)
        self._sync_stream()
        check(self._L.nsc_load_state(self._h, str(path).encode(), _ptr(out), ctypes.byref(t)),
              "nsc_load_state")
        return out, t.value

    def remap_state(self, src, out=None):
        """A state src [F][N_r'][M_theta'][M_z'] of this geometry carried to the
        context's resolution (mode padding/truncation, radial interpolation)."""
        if not (isinstance(src, torch.Tensor) and src.dtype == torch.complex128 and src.is_cuda
                and src.is_contiguous() and src.dim() == 4 and src.shape[0] == self.F):
            raise TypeError("src must be a contiguous complex128 CUDA tensor [F][N_r][M_theta][M_z]")
        if out is None:
            out = self.empty()
        _need(out, self.shape, "out")
        self._sync_stream()
        check(self._L.nsc_remap_state(self._h, _ptr(src), int(src.shape[1]), int(src.shape[2]),
                                      int(src.shape[3]), _ptr(out)), "nsc_remap_state")
        return out

    def energy(self, u):
        _need(u, self.shape, "u")
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        self._sync_stream()
        check(self._L.nsc_energy(self._h, _ptr(u), _ptr(e)), "nsc_energy")
        return e

    def initial_state(self, amps):
        """Divergence-free initial condition from [F][M_theta][M_z] mode
        amplitudes (device complex128)."""
        _need(amps, (self.F, self.M_theta, self.M_z), "amps")
        out = self.empty()
        self._sync_stream()
        check(self._L.nsc_initial_state(self._h, _ptr(amps), _ptr(out)), "nsc_initial_state")
        return out

    def set_profiling(self, on=True):
        check(self._L.nsc_set_profiling(self._h, int(bool(on))), "nsc_set_profiling")

    def timings(self):
        """Per-stage device ms and launch counts since the last call."""
        names = KERNELS
        n = 2 * len(names)
        buf = (ctypes.c_double * n)()
        check(self._L.nsc_get_timings(self._h, buf, n), "nsc_get_timings")
        return {nm: (buf[i], int(buf[len(names) + i])) for i, nm in enumerate(names)}


def read_state_header(path):
    """Header of a state file (host only): dict with F, N_r, M_theta, M_z, eta,
    Re_i, Re_o, Ra, Pr, L_z and time."""
    L = _lib.lib()
    dims = (ctypes.c_int * 4)()
    par = (ctypes.c_double * 7)()
    check(L.nsc_read_state_header(str(path).encode(), dims, par), "nsc_read_state_header")
    out = dict(zip(("F", "N_r", "M_theta", "M_z"), list(dims)))
    out.update(zip(("eta", "Re_i", "Re_o", "Ra", "Pr", "L_z", "time"), list(par)))
    return out
