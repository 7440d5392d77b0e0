"""ctypes declarations of the C ABI in include/rpa.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpa_mi355x.so")

c_int = ctypes.c_int
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_size_t = ctypes.c_size_t
P_i32 = ctypes.POINTER(ctypes.c_int32)
P_f64 = ctypes.POINTER(ctypes.c_double)

RPA_OK = 0
RPA_ERR_INPUT = -1
RPA_ERR_SHAPE = -2
RPA_ERR_ALIAS = -3
RPA_ERR_NOMEM = -4
RPA_ERR_NOT_PD = -5
RPA_ERR_HIP = -6
RPA_ERR_UNSUPPORTED = -7

PRECISION = {"fp64": 0, "split_bf16": 1, "split_fp16": 2}


class RpaCell(ctypes.Structure):
    _fields_ = [("A", c_double * 9), ("n", c_int * 3)]


class RpaSymop(ctypes.Structure):
    _fields_ = [
        ("rot", (ctypes.c_int32 * 3) * 3),
        ("time_reversal", ctypes.c_int32),
        ("gshift", ctypes.c_int32 * 3),
        ("kibz", c_double * 3),
        ("atom_map", P_i32),
        ("atom_shift", P_i32),
        ("proj_rot", P_f64),
    ]


class RpaStates(ctypes.Structure):
    _fields_ = [
        ("nbands", c_int),
        ("nQ", c_int),
        ("miller", P_i32),
        ("C", c_void_p),
        ("eps", P_f64),
        ("f", P_f64),
        ("natoms", c_int),
        ("proj_off", P_i32),
        ("P", c_void_p),
        ("kpt", c_double * 3),
        ("weight", c_double),
        ("dfde", P_f64),
        ("sym", ctypes.POINTER(RpaSymop)),
    ]


class RpaQSpec(ctypes.Structure):
    _fields_ = [
        ("q", c_double * 3),
        ("optical", c_int),
        ("qhat", c_double * 3),
        ("NG", c_int),
        ("gmiller", P_i32),
        ("Qpaw", c_void_p),
        ("Dpaw", P_f64),
        ("weight", c_double),
    ]


class RpaFreq(ctypes.Structure):
    _fields_ = [("nw", c_int), ("omega", P_f64), ("weight", P_f64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "rpa_create": (c_int, [ctypes.POINTER(c_void_p), ctypes.POINTER(RpaCell), c_int, c_size_t]),
    "rpa_destroy": (c_int, [c_void_p]),
    "rpa_gsphere": (c_int, [ctypes.POINTER(RpaCell), P_f64, c_double, P_i32, c_int, ctypes.POINTER(c_int)]),
    "rpa_pair_density": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates),
                                 ctypes.POINTER(RpaQSpec), c_int, P_i32, P_i32, c_int, c_void_p, c_void_p]),
    "rpa_chi0": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates), c_int,
                         ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_int, c_void_p, c_void_p]),
    "rpa_chi0_real": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates), c_int,
                              ctypes.POINTER(RpaQSpec), P_f64, c_int, c_double, c_int, c_void_p, c_void_p]),
    "rpa_chi0_add": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates), c_int,
                             ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_int, c_void_p, c_void_p]),
    "rpa_ec_from_chi0": (c_int, [c_void_p, ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_void_p,
                                 c_void_p, c_void_p, c_void_p]),
    "rpa_ec": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates), c_int,
                       ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_int, c_void_p, c_void_p, c_void_p]),
    "rpa_ec_noalloc": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates), c_int,
                               ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_int, c_void_p, c_void_p,
                               c_void_p]),
    "rpa_ec_batched": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates), c_int, c_int,
                               ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_int, c_void_p, c_void_p, c_int,
                               c_void_p]),
    "rpa_ec_batched_sets": (c_int, [c_void_p, c_int, ctypes.POINTER(ctypes.POINTER(RpaStates)),
                                    ctypes.POINTER(ctypes.POINTER(RpaStates)), ctypes.POINTER(c_int),
                                    ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_int, c_void_p, c_void_p,
                                    c_int, c_void_p]),
    "rpa_ec_backward": (c_int, [c_void_p, ctypes.POINTER(RpaStates), ctypes.POINTER(RpaStates), c_int,
                                ctypes.POINTER(RpaQSpec), ctypes.POINTER(RpaFreq), c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "rpa_autotune": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_void_p]),
    "rpa_tune_set": (c_int, [c_void_p, c_int, c_int, c_int]),
    "rpa_set_pair_path": (c_int, [c_void_p, c_int]),
    "rpa_set_chunk_pairs": (c_int, [c_void_p, c_int]),
    "rpa_set_paw_window": (c_int, [c_void_p, c_int]),
    "rpa_set_autotune": (c_int, [c_void_p, c_int]),
    "rpa_tune_get": (c_int, [c_void_p, c_int, c_int, ctypes.POINTER(c_int)]),
    "rpa_tune_cache_io": (c_int, [c_void_p, ctypes.c_char_p, c_int]),
    "rpa_check": (c_int, [c_void_p, c_void_p]),
    "rpa_profile": (c_int, [c_void_p, c_int]),
    "rpa_profile_get": (c_int, [c_void_p, ctypes.c_char_p, ctypes.POINTER(c_double),
                                ctypes.POINTER(ctypes.c_longlong)]),
    "rpa_status_string": (ctypes.c_char_p, [c_int]),
    "rpa_last_error": (ctypes.c_char_p, [c_void_p]),
}

_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1307_8052_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB
