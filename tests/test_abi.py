"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/nsc.h, and validates arguments before
touching the device."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nsc.h")


def _lib():
    from paper_1908_00587_amd import _lib
    return _lib.lib()


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nsc_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_core_calls():
    names = _declared()
    for required in ("nsc_init", "nsc_nonlinear", "nsc_radial_solve", "nsc_step",
                     "nsc_destroy", "nsc_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def _init(*args):
    L = _lib()
    h = ctypes.c_void_p(123)
    st = L.nsc_init(*[float(a) if i in (0, 1, 2, 3, 4, 8) else int(a) for i, a in enumerate(args)],
                    ctypes.byref(h))
    return st, h


GOOD = (0.5, 50.0, 0.0, 0.0, 1.0, 32, 16, 31, 2 * math.pi)


@pytest.mark.parametrize("idx,val", [
    (0, 0.0), (0, 1.0), (0, -0.3), (0, float("nan")),   # eta outside (0,1)
    (3, -1.0),                                           # Ra < 0
    (5, 8), (5, 0),                                      # N_r < 9
    (6, 0),                                              # M_theta < 1
    (7, 30), (7, 0),                                     # M_z even / zero
    (8, 0.0), (8, -1.0), (8, float("inf")),              # L_z
    (6, 7),                                              # N_theta = 21 = 3*7: radix 7 unsupported
])
def test_init_rejects_bad_arguments(idx, val):
    args = list(GOOD)
    args[idx] = val
    st, h = _init(*args)
    assert st == -1
    assert h.value is None


def test_init_rejects_bad_prandtl_when_heated():
    args = list(GOOD)
    args[3] = 1e4
    args[4] = 0.0
    st, _ = _init(*args)
    assert st == -1


def test_null_pointer_arguments():
    L = _lib()
    assert L.nsc_init(0.5, 0, 0, 0, 1, 32, 16, 31, 6.0, None) == -1
    assert L.nsc_step(None, None, None) == -1
    assert L.nsc_nonlinear(None, None, None, None) == -1
    assert L.nsc_radial_solve(None, None, None, None, None, None) == -1
    assert L.nsc_set_timestep(None, 1e-3, 0, 0.5, 1e-3, 1, 0.5) == -1
    assert L.nsc_destroy(None) == 0


def test_strerror_messages():
    L = _lib()
    for code in (0, -1, -2, -3, -4, -5, -6, 7):
        assert isinstance(L.nsc_strerror(code), bytes)
    assert b"argument" in L.nsc_strerror(-1)


def test_valid_arguments_reach_the_device_check():
    """Valid arguments pass validation; without a GPU the device query fails
    with NSC_ERR_DEVICE (on a GPU machine the context is created)."""
    import torch
    st, h = _init(*GOOD)
    if torch.cuda.is_available():
        assert st == 0
        _lib().nsc_destroy(h)
    else:
        assert st == -2
