"""ctypes view of the C ABI declared in include/elfpie.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

from . import build as _build

c_int32, c_uint32, c_double, c_void_p, c_size_t, c_float = (
    ctypes.c_int32, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_float)

OK, E_INVALID, E_RANGE, E_UNSUPPORTED, E_WORKSPACE, E_DEVICE, E_NONFINITE = range(7)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_RANGE", 3: "E_UNSUPPORTED", 4: "E_WORKSPACE",
                5: "E_DEVICE", 6: "E_NONFINITE"}
FID_AMPLITUDE, FID_INTENSITY, FID_GAMMA, FID_LOG = 0, 1, 2, 3
OPT_ELFPIE, OPT_SGD, OPT_NADAM, OPT_ADABELIEF = 0, 1, 2, 3
NORM_ANISO, NORM_ISO = 0, 1
F64, F32, F32_MFMA_BF16X3 = 0, 1, 2
LEARN_PUPIL, PUPIL_SUPPORT, PUPIL_FILTER = 1, 2, 4


class ProblemC(ctypes.Structure):
    _fields_ = [
        ("n_lo", c_int32), ("upsample", c_int32), ("K", c_int32),
        ("wavelength_um", c_double), ("na", c_double), ("dx_lo_um", c_double),
        ("led_k", ctypes.POINTER(c_double)),
        ("alpha", c_double), ("beta", c_double), ("lr", c_double),
        ("gamma1", c_double), ("gamma2", c_double), ("eta_opt", c_double),
        ("eta_h", c_double), ("l1_eps", c_double),
        ("fidelity", c_int32), ("norm", c_int32), ("precision", c_int32), ("flags", c_uint32),
        ("fid_gamma", c_double), ("optimizer", c_int32), ("mux", c_int32),
    ]


class StateC(ctypes.Structure):
    _fields_ = [(name, c_void_p) for name in
                ("psi", "P", "mu_psi", "v_psi", "delta_psi", "mu_P", "v_P", "delta_P", "t")]


FUNCTIONS = {
    "elfpie_problem_defaults": (c_int32, [ctypes.POINTER(ProblemC)]),
    "elfpie_workspace_bytes": (c_int32, [ctypes.POINTER(ProblemC), ctypes.POINTER(c_size_t)]),
    "elfpie_plan_create": (c_int32, [ctypes.POINTER(ProblemC), c_void_p, c_size_t, ctypes.POINTER(c_void_p)]),
    "elfpie_plan_destroy": (c_int32, [c_void_p]),
    "elfpie_plan_info": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "elfpie_plan_stats": (c_int32, [c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "elfpie_auto_penalty": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p]),
    "elfpie_plan_set_penalty": (c_int32, [c_void_p, c_double, c_double]),
    "elfpie_forward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "elfpie_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "elfpie_grad_fields": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p]),
    "elfpie_grad_noalloc": (c_int32, [ctypes.POINTER(ProblemC), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p]),
    "elfpie_step": (c_int32, [c_void_p, ctypes.POINTER(StateC), c_void_p, c_void_p, c_void_p]),
    "elfpie_run": (c_int32, [c_void_p, ctypes.POINTER(StateC), c_void_p, c_int32, c_void_p, c_int32, c_void_p]),
    "elfpie_object_from_spectrum": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "elfpie_spectrum_from_object": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "elfpie_init_state": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(StateC), c_void_p]),
    "elfpie_stage_timing": (c_int32, [c_void_p, ctypes.POINTER(StateC), c_void_p, c_int32,
                                      ctypes.POINTER(c_float), c_void_p]),
    "elfpie_batch_create": (c_int32, [ctypes.POINTER(c_void_p), ctypes.POINTER(StateC), ctypes.POINTER(c_void_p),
                                      c_int32, c_int32, ctypes.POINTER(c_void_p)]),
    "elfpie_batch_destroy": (c_int32, [c_void_p]),
    "elfpie_batch_run": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p), c_void_p]),
    "elfpie_batch_tune": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_float), ctypes.POINTER(c_int32),
                                    c_void_p]),
    "elfpie_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "elfpie_last_error": (ctypes.c_char_p, [c_void_p]),
}

_LIB = None


def library_path() -> str:
    """The in-tree build, or the library named by ELFPIE_LIB (an alternative build)."""
    return os.environ.get("ELFPIE_LIB") or _build.LIB


def load() -> ctypes.CDLL:
    """Load the built library; raise if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} is missing; run paper_2209_14671_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, (res, args) in FUNCTIONS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class ElfpieError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int, plan_handle=None) -> None:
    if status != OK:
        msg = load().elfpie_last_error(plan_handle)
        raise ElfpieError(status, msg.decode() if msg else "")
