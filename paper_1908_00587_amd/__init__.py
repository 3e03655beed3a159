"""MI355X-native Taylor--Couette DNS time step (nsCouette method, arXiv 1908.00587).

The hot path -- pseudospectral nonlinear term and per-mode radial solves --
runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/nsc.h (libnsc.so, built in-tree).  This package is the Python
binding: argument marshalling, with PyTorch providing device memory and
streams.  Importing it loads libnsc.so and fails if it was not built.
"""
from ._lib import NscError, lib  # noqa: F401
from .api import Context, read_state_header  # noqa: F401

lib()  # fail loudly at import when the HIP library is missing

__all__ = ["Context", "NscError", "lib", "read_state_header"]
