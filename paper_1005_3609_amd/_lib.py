"""ctypes loader for libchromstrip.so.  Fails loudly when the library is
missing: there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libchromstrip.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "chromstrip.h")

CHROM_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED"}
SQUARE, TRIANGULAR = 0, 1
MODES = {"plain": 0, "batched": 1, "graph": 2, "resident": 3, "grouped": 4}
SPACE_NCNNN, SPACE_SQ_INTER, SPACE_LAST = 0, 1, 2


class ChromError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chromstrip {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Tuning(C.Structure):
    _fields_ = [("lanes_v", C.c_int), ("targets_per_wave", C.c_int), ("waves_per_block", C.c_int),
                ("xcd_order", C.c_int), ("unroll", C.c_int), ("streams", C.c_int), ("fuse", C.c_int),
                ("stage", C.c_int)]


class Job(C.Structure):
    _fields_ = [("lattice", C.c_int), ("m", C.c_int), ("n_max", C.c_int),
                ("q_points", C.POINTER(C.c_uint32)), ("nq", C.c_int),
                ("primes", C.POINTER(C.c_uint32)), ("np", C.c_int),
                ("d_out", C.c_void_p)]


class Slot(C.Structure):
    _fields_ = [("lattice", C.c_int), ("m", C.c_int), ("n_max", C.c_int), ("rows_done", C.c_int),
                ("nq", C.c_int), ("np", C.c_int),
                ("q_points", C.POINTER(C.c_uint32)), ("primes", C.POINTER(C.c_uint32)),
                ("d_state", C.c_void_p), ("state_bytes", C.c_size_t), ("d_out", C.c_void_p)]


class MapsInfo(C.Structure):
    _fields_ = [("n_factors", C.c_int), ("n_last", C.c_int), ("n_codes", C.c_int),
                ("total_nnz", C.c_int64), ("max_states", C.c_int64)]


_SIGS = {
    "chromatic_strip": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p]),
    "chromatic_strip_batched": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                          C.c_int, C.POINTER(Tuning), C.c_void_p]),
    "chromatic_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                               C.POINTER(Tuning)]),
    "chromatic_strip_async": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                        C.c_int, C.POINTER(Tuning), C.c_void_p, C.c_size_t, C.c_void_p,
                                        C.c_void_p]),
    "chromatic_strip_noalloc": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                          C.POINTER(Tuning), C.c_void_p, C.c_void_p]),
    "chromatic_factor_launches": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                            C.POINTER(Tuning), C.c_void_p, C.c_size_t, C.c_void_p]),
    "chromatic_prepare": (C.c_int, [C.c_int, C.c_int]),
    "chromatic_prepare_host": (C.c_int, [C.c_int, C.c_int, C.c_int]),
    "chromatic_check_expansion": (C.c_int, [C.c_int, C.c_int, C.c_int]),
    "chromatic_prepare_series": (C.c_int, [C.c_int, C.c_int]),
    "chromatic_series_map_export": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_void_p,
                                              C.c_void_p]),
    "chromatic_release_maps": (None, []),
    "chromatic_batch_workspace_bytes": (C.c_size_t, [C.POINTER(Job), C.c_int, C.POINTER(Tuning)]),
    "chromatic_batch": (C.c_int, [C.POINTER(Job), C.c_int, C.POINTER(Tuning), C.c_void_p, C.c_size_t,
                                  C.c_void_p]),
    "chromatic_slot_state_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(Tuning)]),
    "chromatic_server_step": (C.c_int, [C.POINTER(Slot), C.c_int, C.c_int, C.POINTER(Tuning), C.c_void_p]),
    "chromatic_device_status": (C.c_int, [C.c_void_p]),
    "chromatic_motzkin": (C.c_int64, [C.c_int]),
    "chromatic_space_size": (C.c_int64, [C.c_int, C.c_int, C.c_int]),
    "chromatic_rank": (C.c_int64, [C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "chromatic_unrank": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int64, C.c_void_p]),
    "chromatic_maps_info": (C.c_int, [C.c_int, C.c_int, C.POINTER(MapsInfo)]),
    "chromatic_family_info": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.c_void_p]),
    "chromatic_map_export": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "chromatic_stage_export": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "chromatic_op_export": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "chromatic_cluster_export": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                           C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "chromatic_series_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                                  C.POINTER(Tuning)]),
    "chromatic_series_async": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                         C.POINTER(Tuning), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "chromatic_series": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                   C.POINTER(Tuning), C.c_void_p]),
    "chromatic_code_table": (C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_void_p]),
    "chromatic_last_error": (C.c_char_p, []),
    "chromatic_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1005_3609_amd.build` "
                          "(there is no fallback implementation)")
    # torch ships its own HIP runtime.  Import it first so that the library
    # binds to that same runtime (one runtime per process; torch's streams and
    # allocations are then valid handles for the library).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    h = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(h, name)
        fn.restype = res
        fn.argtypes = args
    _lib = h
    return h


def check(rc: int):
    if rc != CHROM_OK:
        raise ChromError(rc, lib().chromatic_last_error().decode())
    return rc


def header_functions() -> list[str]:
    """Names of the functions declared in include/chromstrip.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chromatic_\w+)\s*\(", text)))


def tuning(t) -> "Tuning | None":
    if t is None:
        return None
    if isinstance(t, Tuning):
        return t
    return Tuning(int(t.get("lanes_v", 0)), int(t.get("targets_per_wave", 0)), int(t.get("waves_per_block", 0)),
                  int(t.get("xcd_order", 0)), int(t.get("unroll", 0)), int(t.get("streams", 0)),
                  int(t.get("fuse", 0)), int(t.get("stage", 0)))
