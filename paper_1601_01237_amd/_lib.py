"""ctypes binding of liblbm.so (the C ABI of include/lbm.h).

Argument marshalling only: every computation runs in the HIP library.  If the
library has not been built, :func:`load` raises instead of falling back to
anything else.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

Q = 19
DIAG_LEN = 16
STATIC_BLOCKS = 8192  # LBM_STATIC_BLOCKS
FP32, FP16, BF16 = 0, 1, 2
BGK, REGULARIZED, REGULARIZED3 = 0, 1, 2
EUNSTABLE = -4

STATUS = {0: "ok", -1: "invalid argument", -2: "HIP runtime error", -3: "invalid state",
          -4: "non-finite values (unstable run)", -5: "not supported"}


class LBMError(RuntimeError):
    def __init__(self, func, code):
        super().__init__(f"{func} failed: {STATUS.get(code, code)} ({code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("storage", C.c_int32),
        ("tau", C.c_double * 2),
        ("G", (C.c_double * 2) * 2),
        ("rho_shift", C.c_double * 2),
        ("rho_wall", C.c_double * 2),
        ("collision", C.c_int32),
    ]


class DiagRegion(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("r_in", C.c_double), ("r_out", C.c_double),
                ("thr", C.c_double)]


_lib = None


def _declare(lib):
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "lbm_version": (i32, []),
        "lbm_velocity_set": (i32, [C.POINTER(C.c_int32), dp]),
        "lbm_status_str": (C.c_char_p, [i32]),
        "lbm_plane_stride": (i64, [i32, i32, i32]),
        "lbm_row_block": (i32, [i32, i32, i32]),
        "lbm_state_elems": (i64, [i32, i32, i32, i32]),
        "lbm_row_half": (i32, [i32, i32, i32]),
        "lbm_init": (i32, [C.POINTER(vp), C.POINTER(Params), vp, vp, vp, vp, vp]),
        "lbm_step": (i32, [vp, i64]),
        "lbm_moments": (i32, [vp, vp, vp, vp, C.POINTER(DiagRegion)]),
        "lbm_moments_static": (i32, [vp, vp, vp, vp, C.POINTER(DiagRegion)]),
        "lbm_get_populations": (i32, [vp, vp]),
        "lbm_set_populations": (i32, [vp, vp]),
        "lbm_time": (i64, [vp]),
        "lbm_set_time": (i32, [vp, i64]),
        "lbm_set_tiling": (i32, [vp, i32, i32]),
        "lbm_set_placement": (i32, [vp, i32, i32]),
        "lbm_wall_classes": (i32, [vp]),
        "lbm_adjoint_work_bytes": (C.c_size_t, [vp]),
        "lbm_set_adjoint_tiling": (i32, [vp, i32, i32]),
        "lbm_adjoint_step": (i32, [vp, vp, vp, vp, vp, C.c_size_t, vp, vp]),
        "lbm_adjoint_step_fields": (i32, [vp, vp, vp, vp, vp, vp, C.c_size_t, vp, vp]),
        "lbm_step_fields": (i32, [vp, vp]),
        "lbm_adjoint_seed": (i32, [vp, vp, vp]),
        "lbm_stream_copy": (i32, [vp, vp, C.c_size_t, vp]),
        "lbm_march_copy": (i32, [vp, vp, vp]),
        "lbm_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load():
    """Load liblbm.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1601_01237_amd.build` "
                "(the HIP library is the only compute path)")
        _lib = _declare(C.CDLL(LIB_PATH))
    return _lib


def check(func, code):
    if code != 0:
        raise LBMError(func, code)


EXPORTED = ["lbm_version", "lbm_velocity_set", "lbm_status_str", "lbm_plane_stride", "lbm_row_block",
            "lbm_state_elems", "lbm_row_half", "lbm_init", "lbm_step",
            "lbm_moments", "lbm_moments_static", "lbm_get_populations", "lbm_set_populations", "lbm_time",
            "lbm_set_time", "lbm_set_tiling", "lbm_set_placement", "lbm_wall_classes", "lbm_adjoint_work_bytes",
            "lbm_set_adjoint_tiling", "lbm_adjoint_step", "lbm_adjoint_step_fields", "lbm_step_fields",
            "lbm_adjoint_seed", "lbm_stream_copy", "lbm_march_copy", "lbm_destroy"]


def velocity_set():
    """(c, w) of the library's D3Q19 ordering (pure host call)."""
    lib = load()
    c = (C.c_int32 * (3 * Q))()
    w = (C.c_double * Q)()
    check("lbm_velocity_set", lib.lbm_velocity_set(c, w))
    return [tuple(c[3 * i:3 * i + 3]) for i in range(Q)], list(w)
