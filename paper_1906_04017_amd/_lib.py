"""ctypes loader of libdgsn.so (the HIP library built in-tree by build.py).

Loading fails loudly when the shared library is missing: there is no CPU
fallback anywhere in the package.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgsn.so")

DGSN_OK = 0
DGSN_EINVAL = -1
DGSN_ENOMEM = -2
DGSN_EHIP = -3
DGSN_ENOTCONV = -4
DGSN_EFORMAT = -5
DGSN_EUNSUPPORTED = -6
DGSN_ETIMEOUT = -7
DGSN_FP32 = 0
DGSN_FP64 = 1
DGSN_GE = 0
DGSN_ANN = 1
DGSN_GE_DENSE = 2
DGSN_SI_MAXNORM = 0
DGSN_SI_EPS_S = 1
DGSN_SI_FIXED = 2
DGSN_ANN_BF16 = 0
DGSN_ANN_BF16X2 = 1
DGSN_DEBUG_POISON_FRONTS = 1
DGSN_SCHED_PLANES = 0
DGSN_SCHED_DATAFLOW = 1

ERROR_NAMES = {
    DGSN_EINVAL: "DGSN_EINVAL", DGSN_ENOMEM: "DGSN_ENOMEM", DGSN_EHIP: "DGSN_EHIP",
    DGSN_ENOTCONV: "DGSN_ENOTCONV", DGSN_EFORMAT: "DGSN_EFORMAT",
    DGSN_EUNSUPPORTED: "DGSN_EUNSUPPORTED", DGSN_ETIMEOUT: "DGSN_ETIMEOUT",
}


class DgsnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class ProblemDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("n_groups", ctypes.c_int), ("n_dirs", ctypes.c_int),
                ("omega", ctypes.POINTER(ctypes.c_double)),
                ("weight", ctypes.POINTER(ctypes.c_double)),
                ("precision", ctypes.c_int), ("solver", ctypes.c_int),
                ("store_psi", ctypes.c_int)]


_VP = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_LL = ctypes.c_longlong
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int)

# name -> (restype, argtypes); every symbol declared in include/dgsn.h
SIGNATURES = {
    "dgsn_version": (_I, []),
    "dgsn_last_error": (ctypes.c_char_p, []),
    "dgsn_ctx_create": (_I, [_I, ctypes.POINTER(_VP)]),
    "dgsn_ctx_destroy": (_I, [_VP]),
    "dgsn_quadrature_ls": (_I, [_I, _PD, _PD, _PI]),
    "dgsn_problem_validate": (_I, [ctypes.POINTER(ProblemDesc)]),
    "dgsn_problem_create": (_I, [_VP, ctypes.POINTER(ProblemDesc), ctypes.POINTER(_VP)]),
    "dgsn_problem_destroy": (_I, [_VP]),
    "dgsn_problem_set_materials": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "dgsn_problem_set_inflow": (_I, [_VP, _PD]),
    "dgsn_problem_set_ann": (_I, [_VP, _VP]),
    "dgsn_problem_set_scattering": (_I, [_VP, _VP, _VP]),
    "dgsn_problem_set_solver": (_I, [_VP, _I]),
    "dgsn_sweep": (_I, [_VP, _VP, _VP, _VP]),
    "dgsn_source_iterate": (_I, [_VP, _VP, _D, _I, _PI, _PD, _PD, _VP]),
    "dgsn_source_iterate_noalloc": (_I, [_VP, _VP, _D, _I, _PI, _PD, _PD, _VP]),
    "dgsn_adjoint_solve": (_I, [_VP, _VP, _VP, _VP, _D, _I, _PI, _VP]),
    "dgsn_local_solve": (_I, [_VP, _VP, _VP, _LL, _I, _VP]),
    "dgsn_ann_load": (_I, [_VP, ctypes.c_char_p, ctypes.POINTER(_VP)]),
    "dgsn_ann_destroy": (_I, [_VP]),
    "dgsn_ann_infer": (_I, [_VP, _VP, _VP, _LL, _VP]),
    "dgsn_ann_set_mode": (_I, [_VP, _I]),
    "dgsn_ann_info": (_I, [_VP, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                           ctypes.POINTER(_I)]),
    "dgsn_ann_infer_octant": (_I, [_VP, _I, _VP, _VP, _LL, _VP]),
    "dgsn_problem_stats": (_I, [_VP, ctypes.POINTER(_LL), _PI, _PD]),
    "dgsn_problem_set_balance": (_I, [_VP, _I]),
    "dgsn_problem_balance": (_I, [_VP, _PD, _VP]),
    "dgsn_problem_generation": (_I, [_VP, ctypes.POINTER(ctypes.c_ulonglong)]),
    "dgsn_problem_set_timing": (_I, [_VP, _I]),
    "dgsn_problem_set_si_criterion": (_I, [_VP, _I]),
    "dgsn_problem_si_history": (_I, [_VP, _PD, _PD, _I, _PI]),
    "dgsn_problem_set_anisotropy": (_I, [_VP, _I, _VP, _VP]),
    "dgsn_problem_set_anisotropy_gg": (_I, [_VP, _I, _VP, _VP]),
    "dgsn_problem_get_moments": (_I, [_VP, _VP, _VP]),
    "dgsn_real_ylm": (_I, [_I, _PD, _I, _PD]),
    "dgsn_problem_set_tile": (_I, [_VP, _I]),
    "dgsn_problem_get_tile": (_I, [_VP, _PI]),
    "dgsn_problem_autotune": (_I, [_VP, _VP, _PI, _PI, _PD]),
    "dgsn_problem_set_debug": (_I, [_VP, _I]),
    "dgsn_autotune_cache_clear": (_I, []),
    "dgsn_autotune_cache_size": (_I, [_PI]),
    "dgsn_autotune_cache_save": (_I, [ctypes.c_char_p]),
    "dgsn_autotune_cache_load": (_I, [ctypes.c_char_p]),
    "dgsn_problem_set_schedule": (_I, [_VP, _I, ctypes.c_uint]),
    "dgsn_problem_get_schedule": (_I, [_VP, _PI]),
    "dgsn_problem_check": (_I, [_VP, _VP]),
    "dgsn_problem_kernel_time": (_I, [_VP, _PD, _PI]),
    "dgsn_batch_create": (_I, [_VP, ctypes.POINTER(_VP), _I, ctypes.POINTER(_VP)]),
    "dgsn_batch_set_io": (_I, [_VP, _I, _VP, _VP]),
    "dgsn_batch_set_tiles": (_I, [_VP, _PI]),
    "dgsn_batch_set_schedule": (_I, [_VP, _I]),
    "dgsn_batch_get_schedule": (_I, [_VP, _PI]),
    "dgsn_batch_autotune": (_I, [_VP, _VP, _PD]),
    "dgsn_batch_run": (_I, [_VP, _VP]),
    "dgsn_batch_latencies_us": (_I, [_VP, _PD]),
    "dgsn_batch_destroy": (_I, [_VP]),
}

_lib = None


def load():
    """Load libdgsn.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libdgsn.so not found at {LIB_PATH}: build it with "
            "`python -m paper_1906_04017_amd.build` (hipcc, gfx950)")
    # torch first: it ships its own HIP runtime (same soname), and the library
    # must bind to that one.  Loaded the other way round, the process would
    # hold two HIP runtimes, and torch's device pointers and streams would not
    # be valid in the library's.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc, allow=()):
    if rc == DGSN_OK or rc in allow:
        return rc
    msg = load().dgsn_last_error()
    raise DgsnError(rc, msg.decode() if msg else "")
