"""ctypes declarations mirroring include/pfsolve.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfsolve.so")

_D = C.c_double

PF_OK, PF_ERR_INVALID_ARG, PF_ERR_STATE, PF_ERR_UNSTABLE = 0, 1, 2, 3
PF_ERR_OOM, PF_ERR_DEVICE, PF_ERR_NONFINITE, PF_ERR_IO = 4, 5, 6, 7
STATUS_NAMES = {
    0: "OK", 1: "INVALID_ARG", 2: "STATE", 3: "UNSTABLE", 4: "OOM", 5: "DEVICE", 6: "NONFINITE",
    7: "IO",
}
PF_FP64, PF_FP32 = 0, 1
PF_INIT_VORONOI, PF_INIT_HOST = 0, 1

# every symbol the header declares, for the export check
EXPORTS = [
    "pf_required_bytes", "pf_create_domain", "pf_set_params", "pf_get_dt", "pf_init_fields",
    "pf_set_time", "pf_step", "pf_step_timed", "pf_sync", "pf_read_fields", "pf_get_step",
    "pf_destroy", "pf_pack_create", "pf_pack_add", "pf_pack_step", "pf_pack_remaining",
    "pf_pack_remove", "pf_pack_sync", "pf_pack_destroy", "pf_set_variant", "pf_last_error",
    "pf_checkpoint_save", "pf_checkpoint_load", "pf_mesh_phase", "pf_diag_fields_noalloc",
]


class PfDomainDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("prec", C.c_int32),
                ("dx", _D)]


class PfDeviceBuffer(C.Structure):
    _fields_ = [("base", C.c_void_p), ("bytes", C.c_size_t)]


class PfParams(C.Structure):
    _fields_ = [
        ("eps", _D), ("tau", _D * 4), ("gamma", (_D * 4) * 4), ("gamma3", _D),
        ("aniso_delta", (_D * 4) * 4), ("chi0", (_D * 2) * 4), ("chi1", (_D * 2) * 4),
        ("c0", (_D * 2) * 4), ("c1", (_D * 2) * 4), ("w0", _D * 4), ("w1", _D * 4),
        ("D", _D * 4), ("TE", _D), ("T0", _D), ("G", _D), ("v", _D), ("zoff", _D), ("dt", _D),
        ("antitrapping", C.c_int32), ("mu_frozen", C.c_int32), ("diag_every", C.c_int32),
        ("shortcuts", C.c_int32), ("window_z", C.c_int32), ("top_bc", C.c_int32),
        ("mu_fill", _D * 2),
    ]


class PfInit(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("nseeds", C.c_int32), ("seed", C.c_uint64),
        ("solid_height", C.c_int32), ("reserved", C.c_int32), ("mu_init", _D * 2),
        ("phi", C.POINTER(_D)), ("mu", C.POINTER(_D)),
    ]


class PfDiag(C.Structure):
    _fields_ = [
        ("t", _D), ("step", C.c_int64), ("sum_c", _D * 2), ("sum_phi", _D * 4),
        ("max_simplex_dev", _D), ("phi_min", _D), ("phi_max", _D), ("nonfinite", C.c_int64),
        ("window_shifts", C.c_int64),
        ("light_items", C.c_int32),
        ("work_items", C.c_int32),
        ("fixed_items", C.c_int32),
        ("mu_pure_items", C.c_int32),
        ("copied_items", C.c_int32),
        ("reserved", C.c_int32),
    ]


def declare(lib: C.CDLL) -> C.CDLL:
    P = C.c_void_p
    I32, I64 = C.c_int32, C.c_int64
    sig = {
        "pf_required_bytes": (C.c_int, [C.POINTER(PfDomainDesc), C.POINTER(C.c_size_t)]),
        "pf_create_domain": (C.c_int, [C.POINTER(PfDomainDesc), C.POINTER(PfDeviceBuffer), P,
                                       C.POINTER(P)]),
        "pf_set_params": (C.c_int, [P, C.POINTER(PfParams)]),
        "pf_get_dt": (C.c_int, [P, C.POINTER(_D), C.POINTER(_D)]),
        "pf_init_fields": (C.c_int, [P, C.POINTER(PfInit)]),
        "pf_set_time": (C.c_int, [P, I64]),
        "pf_step": (C.c_int, [P, I64]),
        "pf_step_timed": (C.c_int, [P, I64, C.POINTER(_D), C.POINTER(_D)]),
        "pf_sync": (C.c_int, [P]),
        "pf_read_fields": (C.c_int, [P, C.POINTER(_D), C.POINTER(_D), C.POINTER(PfDiag)]),
        "pf_get_step": (C.c_int, [P, C.POINTER(I64)]),
        "pf_destroy": (None, [P]),
        "pf_pack_create": (C.c_int, [I32, P, I32, C.POINTER(P)]),
        "pf_pack_add": (C.c_int, [P, P, I64]),
        "pf_pack_step": (C.c_int, [P, I64, C.POINTER(I32)]),
        "pf_pack_remaining": (C.c_int, [P, P, C.POINTER(I64)]),
        "pf_pack_remove": (C.c_int, [P, P]),
        "pf_pack_sync": (C.c_int, [P]),
        "pf_pack_destroy": (None, [P]),
        "pf_set_variant": (C.c_int, [I32]),
        "pf_last_error": (C.c_char_p, []),
        "pf_checkpoint_save": (C.c_int, [P, C.c_char_p]),
        "pf_checkpoint_load": (C.c_int, [P, C.c_char_p]),
        "pf_mesh_phase": (C.c_int, [P, I32, _D, C.POINTER(PfDeviceBuffer), C.POINTER(I64)]),
        "pf_diag_fields_noalloc": (C.c_int, [C.POINTER(PfDomainDesc), C.POINTER(PfParams), P, _D,
                                             P, C.POINTER(PfDiag)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
