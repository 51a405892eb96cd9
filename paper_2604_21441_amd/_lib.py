"""ctypes declarations of the C ABI in include/nnp.h (argument marshalling only).

The shared library is ``libnnp.so`` next to this file, built by
``python -m paper_2604_21441_amd.build``.  Loading fails loudly when it is
missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnnp.so")

# nnp_status
NNP_OK = 0
NNP_EINVAL = -1
NNP_ESPECIES = -2
NNP_EBOX = -3
NNP_ECAPACITY = -4
NNP_EHIP = -5
NNP_ESTATE = -6
NNP_ENONFINITE = -7

# nnp_precision
NNP_FP32 = 0
NNP_BF16 = 1

# nnp_buffer
NNP_BUF_PERM = 0
NNP_BUF_KEY = 1
NNP_BUF_BIN_START = 2
NNP_BUF_NBR_COUNT = 3
NNP_BUF_NBR_RAD = 4
NNP_BUF_NBR_ANG = 5
NNP_BUF_DESCRIPTOR = 6
NNP_BUF_ATOM_ENERGY = 7
NNP_BUF_DEDX = 8
NNP_BUF_GRID = 9
NNP_BUF_ORDER = 10
NNP_BUF_CHARGE = 11
NNP_BUF_GRAPH = 12

# nnp_stage
STAGES = ["cells", "neighbours", "descriptor", "mm", "network", "energy", "adjoint", "gather", "mm_adjoint"]
NNP_STAGE_COUNT = len(STAGES)


class nnp_config(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32),
        ("atomic_numbers_host", C.POINTER(C.c_int32)),
        ("rc_rad", C.c_float), ("rc_ang", C.c_float),
        ("eta_rad", C.c_float), ("eta_ang", C.c_float), ("zeta", C.c_float),
        ("n_rad_shift", C.c_int32), ("n_ang_shift", C.c_int32), ("n_ang_sect", C.c_int32),
        ("rad_shift_host", C.POINTER(C.c_float)),
        ("ang_shift_host", C.POINTER(C.c_float)),
        ("ang_sect_host", C.POINTER(C.c_float)),
        ("n_layers", C.c_int32),
        ("widths_host", C.POINTER(C.c_int32)),
        ("celu_alpha", C.c_float),
        ("extra_inputs", C.c_int32),
        ("mm_cutoff", C.c_float),
        ("ke_coulomb", C.c_double),
        ("n_members", C.c_int32),
    ]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_F32P = C.POINTER(C.c_float)

# name -> (restype, argtypes)
SIGNATURES = {
    "nnp_create": (C.c_int, [C.POINTER(nnp_config), C.c_uint64, _F32P, C.c_int, C.POINTER(_P)]),
    "nnp_reserve": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "nnp_compute": (C.c_int, [_P, C.c_int32, _P, _I32P, _F32P, C.c_int32, _I32P, C.c_int32, _P, _P,
                              _P, _P, _P, C.c_int32, _P]),
    "nnp_compute_pairs": (C.c_int, [_P, C.c_int32, _P, _I32P, _F32P, C.c_int32, _I32P, C.c_int32, _P, C.c_int32,
                                    _P, _P, _P, _P, _P, C.c_int32, _P]),
    "nnp_compute_batch": (C.c_int, [_P, C.c_int32, _I32P, _P, _I32P, _F32P, _P, _P, _P]),
    "nnp_compute_noalloc": (C.c_int, [_P, C.c_int32, _P, _I32P, _F32P, _P, _P, _P]),
    "nnp_get_status": (C.c_int, [_P, _P]),
    "nnp_read_buffer": (C.c_int, [_P, C.c_int, _P, C.c_size_t, C.POINTER(C.c_int64), C.POINTER(C.c_int32), _P]),
    "nnp_set_graph": (C.c_int, [_P, C.c_int32]),
    "nnp_set_links": (C.c_int, [_P, C.c_int32, _I32P, _I32P, C.c_float, C.c_int32]),
    "nnp_autotune": (C.c_int, [_P, C.c_int32, _I32P, _P]),
    "nnp_set_variant": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "nnp_get_variants": (C.c_int, [_P, _I32P]),
    "nnp_me_coupling": (C.c_int, [C.c_int32, _P, _P, C.c_int32, _P, _P, _F32P, C.c_float, C.c_float, _P, _P, _P,
                                  C.c_int32, _P]),
    "nnp_profile_enable": (C.c_int, [_P, C.c_int32]),
    "nnp_profile_read": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64), _P]),
    "nnp_destroy": (None, [_P]),
    "nnp_status_string": (C.c_char_p, [C.c_int]),
    "nnp_last_error": (C.c_char_p, []),
    "nnp_version": (C.c_char_p, []),
}

_lib = None


def load(path: str | None = None):
    """Load libnnp.so (once) and declare every entry point's signature."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2604_21441_amd.build` "
                           "(the NNP path has no non-HIP fallback)")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib
