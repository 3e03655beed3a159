"""ctypes binding of libnsc.so (include/nsc.h).  Argument marshalling only:
every step of the time step runs in the library's HIP kernels.  There is no
fallback: if the shared library is missing, importing fails loudly."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsc.so")

NSC_OK = 0
NSC_ERR_ARG = -1
NSC_ERR_DEVICE = -2
NSC_ERR_OOM = -3
NSC_ERR_NONFINITE = -4
NSC_ERR_DT = -5
NSC_ERR_STATE = -6
NSC_ERR_IO = -7
NSC_FP64 = 0
NSC_MIXED = 1

_lib = None


class NscError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().nsc_strerror(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")


def _bind(L):
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    sig = {
        "nsc_init": ([D, D, D, D, D, I, I, I, D, ctypes.POINTER(P)], I),
        "nsc_init_pipe": ([D, I, I, I, D, ctypes.POINTER(P)], I),
        "nsc_destroy": ([P], I),
        "nsc_set_stream": ([P, P], I),
        "nsc_set_precision": ([P, I], I),
        "nsc_set_timestep": ([P, D, I, D, D, I, D], I),
        "nsc_nonlinear": ([P, P, P, P], I),
        "nsc_radial_solve": ([P, P, P, P, P, P], I),
        "nsc_step": ([P, P, ctypes.POINTER(D)], I),
        "nsc_energy": ([P, P, P], I),
        "nsc_initial_state": ([P, P, P], I),
        "nsc_nonlinear_vjp": ([P, P, P, P], I),
        "nsc_radial_solve_vjp": ([P, P, P, P, P], I),
        "nsc_step_stages": ([P, P, P, P], I),
        "nsc_step_vjp": ([P, P, P, P, P], I),
        "nsc_step_vjp_noalloc": ([P, P, P, P, P], I),
        "nsc_energy_grad": ([P, P, P], I),
        "nsc_get_grid": ([P, ctypes.POINTER(D), I], I),
        "nsc_get_timings": ([P, ctypes.POINTER(D), I], I),
        "nsc_set_profiling": ([P, I], I),
        "nsc_diagnostics": ([P, P, P], I),
        "nsc_probe": ([P, P, I, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D), P], I),
        "nsc_save_state": ([P, P, D, ctypes.c_char_p], I),
        "nsc_read_state_header": ([ctypes.c_char_p, ctypes.POINTER(I), ctypes.POINTER(D)], I),
        "nsc_load_state": ([P, ctypes.c_char_p, P, ctypes.POINTER(D)], I),
        "nsc_remap_state": ([P, P, I, I, I, P], I),
        "nsc_strerror": ([I], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


def lib():
    """Load libnsc.so from the package directory (built in-tree)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(hipcc --offload-arch=gfx950); there is no fallback path")
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def check(code, where):
    if code != NSC_OK:
        raise NscError(code, where)
