"""ctypes declarations of include/htr.h.  Loads the in-tree libhtr.so and
fails loudly if it is missing: there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhtr.so")

HTR_OK, HTR_EINVAL, HTR_ENOMEM, HTR_EDEVICE, HTR_ENONFINITE, HTR_ENEWTON, HTR_ETRANGE, HTR_EUNSUPPORTED = range(8)
STATUS_NAMES = {0: "HTR_OK", 1: "HTR_EINVAL", 2: "HTR_ENOMEM", 3: "HTR_EDEVICE", 4: "HTR_ENONFINITE",
                5: "HTR_ENEWTON", 6: "HTR_ETRANGE", 7: "HTR_EUNSUPPORTED"}
HTR_MAX_NS, HTR_MAX_NR, HTR_MAX_SIDE = 12, 64, 3
HTR_CHEM_OFF, HTR_VISC_OFF, HTR_FORCE_CENTRAL, HTR_FORCE_TENO, HTR_WENO3Z = 1, 2, 4, 8, 16
HTR_BC_PERIODIC, HTR_BC_WALL, HTR_BC_INFLOW, HTR_BC_OUTFLOW = 0, 1, 2, 3

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class htr_mech_desc(C.Structure):
    _fields_ = [("ns", C.c_int32), ("nr", C.c_int32), ("W", _dp), ("nasa7", _dp), ("lj_sigma", _dp),
                ("lj_epsk", _dp), ("lnA", _dp), ("beta", _dp), ("Ea", _dp), ("nu_f", _ip), ("nu_r", _ip),
                ("Tmin", C.c_double), ("Tmax", C.c_double)]


class htr_grid_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("xnode", _dp * 3), ("xi_node", _dp * 3), ("xi_face", _dp * 3),
                ("L", C.c_double * 3)]


class htr_curv_grid_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("xyz", _dp), ("period", (C.c_double * 3) * 3)]


class htr_laser(C.Structure):
    _fields_ = [("E", C.c_double), ("center", C.c_double * 3), ("sigma_r", C.c_double), ("t0", C.c_double),
                ("sigma_t", C.c_double), ("on", C.c_int32)]


class htr_member_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dx", C.c_double * 3), ("laser", htr_laser), ("dlnA", _dp)]


class htr_scheme(C.Structure):
    _fields_ = [("cfl", C.c_double), ("theta_c", C.c_double), ("psi_c", C.c_double), ("teno_CT", C.c_double),
                ("flags", C.c_uint32)]


class HTRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_02319_amd.build` "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    sig = {
        "htr_create": (st, [C.POINTER(htr_mech_desc), C.POINTER(htr_grid_desc), C.POINTER(htr_scheme),
                            C.POINTER(vp)]),
        "htr_create_curvilinear": (st, [C.POINTER(htr_mech_desc), C.POINTER(htr_curv_grid_desc),
                                        C.POINTER(htr_scheme), C.POINTER(vp)]),
        "htr_grid_metrics": (st, [vp, vp, vp, vp]),
        "htr_destroy": (st, [vp]),
        "htr_set_flags": (st, [vp, C.c_uint32]),
        "htr_set_boundaries": (st, [vp, vp, vp, vp]),
        "htr_num_cells": (C.c_int64, [vp]),
        "htr_prim_to_cons": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "htr_rhs": (st, [vp, vp, vp, C.c_double, C.POINTER(htr_laser), vp, vp, vp]),
        "htr_cells": (st, [vp, vp, vp, C.c_double, C.POINTER(htr_laser), vp, vp]),
        "htr_stable_dt": (st, [vp, vp, vp, vp, vp]),
        "htr_work_bytes": (C.c_size_t, [vp]),
        "htr_rk3_step": (st, [vp, vp, vp, vp, vp, C.c_int, C.POINTER(htr_laser), vp, vp, vp, vp]),
        "htr_rk3_step_noalloc": (st, [vp, vp, vp, vp, vp, C.c_int, C.POINTER(htr_laser), vp, vp, vp]),
        "htr_timing": (st, [vp, C.c_int]),
        "htr_timing_read": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "htr_check": (st, [vp, vp]),
        "htr_adjoint_work_bytes": (C.c_size_t, [vp]),
        "htr_rhs_adjoint": (st, [vp, vp, vp, C.c_double, C.POINTER(htr_laser), vp, vp, C.c_double, C.c_double, vp,
                                 vp, vp, vp]),
        "htr_rk3_step_adjoint": (st, [vp, vp, vp, vp, C.c_double, C.c_double, C.POINTER(htr_laser), vp,
                                      C.c_double, vp, vp, vp, vp, vp]),
        "htr_tape_bytes": (C.c_size_t, [vp]),
        "htr_rk3_step_taped": (st, [vp, vp, vp, vp, vp, C.c_int, C.POINTER(htr_laser), vp, vp, vp, vp, vp]),
        "htr_batch_create": (st, [vp, C.c_int32, C.POINTER(htr_member_desc), C.POINTER(vp)]),
        "htr_batch_destroy": (st, [vp]),
        "htr_batch_cells": (C.c_int64, [vp, C.POINTER(C.c_int64)]),
        "htr_batch_prim_to_cons": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "htr_rhs_batched": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "htr_batch_work_bytes": (C.c_size_t, [vp]),
        "htr_rk3_steps_batched": (st, [vp, vp, vp, vp, vp, C.c_int, C.c_int, vp, vp, C.c_int, vp]),
        "htr_batch_check": (st, [vp, vp]),
        "htr_batch_member_max": (st, [vp, vp, vp, C.c_int, vp]),
        "htr_tile_shape_check": (st, [C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "htr_set_tiling": (st, [vp, C.POINTER(C.c_int32), C.c_int32]),
        "htr_get_tiling": (st, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "htr_set_conv_split": (st, [vp, C.c_int32]),
        "htr_get_conv_split": (st, [vp, C.POINTER(C.c_int32)]),
        "htr_batch_set_conv_split": (st, [vp, C.c_int32]),
        "htr_batch_get_conv_split": (st, [vp, C.POINTER(C.c_int32)]),
        "htr_autotune": (st, [vp, vp, vp, vp, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "htr_batch_set_tiling": (st, [vp, C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
        "htr_batch_get_tiling": (st, [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "htr_batch_autotune": (st, [vp, vp, vp, vp, vp]),
        "htr_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names of the C entry points declared in include/htr.h."""
    hdr = os.path.join(os.path.dirname(HERE), "include", "htr.h")
    import re
    names = []
    for line in open(hdr):
        m = re.match(r"^\s*(?:htr_status|size_t|int64_t|const char\*)\s+(htr_\w+)\s*\(", line)
        if m:
            names.append(m.group(1))
    return names


def check(code):
    if code != HTR_OK:
        msg = load().htr_last_error().decode(errors="replace")
        raise HTRError(code, msg)
