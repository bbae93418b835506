"""ctypes binding of libpetto.so (the C ABI of include/petto.h): struct layouts,
argument and return types.  Argument marshalling only; all computation is in the
library.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpetto.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "petto.h")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID, ERR_HIP, ERR_DIVERGED, ERR_OOM, ERR_UNSUPPORTED = -1, -2, -3, -4, -5
ELASTIC, HEAT = 0, 1
FP32, FP64 = 0, 1
FIELD_STATE, FIELD_CELL = 0, 1
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_INVALID", -2: "ERR_HIP", -3: "ERR_DIVERGED",
                -4: "ERR_OOM", -5: "ERR_UNSUPPORTED"}


MAX_PHASES = 6          # PETTO_MAX_PHASES of the header


class Problem(C.Structure):
    _fields_ = [
        ("physics", C.c_int32), ("ndim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double),
        ("e0", C.c_double), ("emin", C.c_double), ("nu", C.c_double), ("p", C.c_double),
        ("nphase", C.c_int32), ("e_phase", C.c_double * (MAX_PHASES + 1)), ("side", C.c_int32 * 6),
        ("fixed", C.POINTER(C.c_uint8)), ("load", C.POINTER(C.c_double)), ("q", C.c_double),
        ("region", C.POINTER(C.c_uint8)),
    ]


class AptParams(C.Structure):
    _fields_ = [
        ("theta", C.c_double), ("dt", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
        ("check_every", C.c_int32), ("refine", C.c_int32), ("use_graph", C.c_int32),
        ("replay_iters", C.c_int32), ("adapt", C.c_int32), ("n_pt", C.c_int32), ("dt_pt", C.c_double),
    ]


class PhaseParams(C.Structure):
    _fields_ = [
        ("alpha_h", C.c_double), ("gamma", C.c_double), ("dt_ac", C.c_double),
        ("vol_frac", C.c_double * MAX_PHASES), ("bisect_passes", C.c_int32), ("model", C.c_int32),
        ("alpha_v", C.c_double), ("alpha_1", C.c_double), ("dt_ch", C.c_double), ("mobility", C.c_double),
        ("alpha_b", C.c_double),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("status", C.c_int32), ("outer", C.c_int32), ("pad_", C.c_int32),
        ("rel_res", C.c_double), ("r_pde", C.c_double), ("dt", C.c_double), ("theta", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("iters", "status", "outer", "rel_res", "r_pde", "dt", "theta")}


class PhaseInfo(C.Structure):
    _fields_ = [("shift", C.c_double * MAX_PHASES), ("volume", C.c_double * MAX_PHASES),
                ("gmax", C.c_double * MAX_PHASES)]

    def as_dict(self):
        return {"shift": list(self.shift), "volume": list(self.volume), "gmax": list(self.gmax)}


_lib = None


def declared_functions():
    """Names of the functions include/petto.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(petto_[a-z_0-9]+)\s*\(", txt)))


def load(path: str = LIB_PATH):
    """Load libpetto.so (cached).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2509_06971_amd.build` "
                          "(there is no CPU fallback for the HIP path)")
    lib = C.CDLL(path)
    vp, st = C.c_void_p, C.c_int32
    sig = {
        "petto_create": (st, [C.POINTER(Problem), C.c_int32, C.c_int32, C.POINTER(vp)]),
        "petto_destroy": (st, [vp]),
        "petto_field_offset": (C.c_size_t, [vp, C.c_int32, C.c_int32]),
        "petto_apt_solve": (st, [vp, vp, vp, vp, C.POINTER(AptParams), vp, C.POINTER(SolveInfo)]),
        "petto_residual": (st, [vp, vp, vp, vp, vp]),
        "petto_adjoint": (st, [vp, vp, vp, vp, C.c_int32, vp, vp, vp]),
        "petto_adjoint_noalloc": (st, [vp, vp, vp, vp, C.c_int32, vp, vp, vp]),
        "petto_phase_update": (st, [vp, vp, vp, C.POINTER(PhaseParams), vp, C.POINTER(PhaseInfo)]),
        "petto_step": (st, [vp, vp, vp, vp, vp, vp, C.POINTER(AptParams), C.POINTER(PhaseParams), vp,
                            C.POINTER(SolveInfo), C.POINTER(PhaseInfo)]),
        "petto_last_sweep_ms": (C.c_double, [vp, C.POINTER(C.c_int64)]),
        "petto_set_timing": (st, [vp, C.c_int32]),
        "petto_set_blocking": (st, [vp, C.c_int32]),
        "petto_blocking": (C.c_int32, [vp]),
        "petto_set_tile3d": (st, [vp, C.c_int32]),
        "petto_time_sweeps": (st, [vp, C.c_int32, vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "petto_tile3d": (C.c_int32, [vp]),
        "petto_last_error": (C.c_char_p, []),
        "petto_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class PettoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status < 0:
        raise PettoError(status, load().petto_last_error().decode())
    return status
