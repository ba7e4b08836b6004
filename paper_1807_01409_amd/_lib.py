"""ctypes declarations of libtid.so (include/tid.h).  Loading fails loudly if
the library has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtid.so")

TID_MAX_COLS = 32
TID_MAX_MULTI = 16

STATUS = {
    0: "TID_OK", -1: "TID_E_INVALID_ARG", -2: "TID_E_OOM", -3: "TID_E_CAPACITY",
    -4: "TID_E_UNSUPPORTED", -5: "TID_E_SCHEMA", -6: "TID_E_HIP", -7: "TID_E_INTERNAL",
}


class tid_pattern(ctypes.Structure):
    _fields_ = [("s", ctypes.c_uint32), ("p", ctypes.c_uint32), ("o", ctypes.c_uint32),
                ("vs", ctypes.c_int32), ("vp", ctypes.c_int32), ("vo", ctypes.c_int32),
                ("range_pos", ctypes.c_int32), ("lo", ctypes.c_uint32), ("hi", ctypes.c_uint32)]


class tid_plan(ctypes.Structure):
    _fields_ = [("n_patterns", ctypes.c_int32), ("patterns", ctypes.POINTER(tid_pattern)),
                ("n_ops", ctypes.c_int32), ("ops", ctypes.POINTER(ctypes.c_uint32))]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                           ctypes.c_void_p)

_lib = None

# name -> (restype, argtypes)
_VP = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_U32P = ctypes.POINTER(ctypes.c_uint32)
_I32P = ctypes.POINTER(ctypes.c_int32)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_I64P = ctypes.POINTER(ctypes.c_int64)
_S = ctypes.c_int32

SIGNATURES = {
    "tid_ctx_create": (_S, [ctypes.c_int, _VP, ALLOC_FN, FREE_FN, _VP, _PP]),
    "tid_ctx_destroy": (None, [_VP]),
    "tid_last_error": (ctypes.c_char_p, [_VP]),
    "tid_ctx_synchronize": (_S, [_VP]),
    "tid_ctx_set_option": (_S, [_VP, ctypes.c_char_p, ctypes.c_int64]),
    "tid_ctx_get_option": (_S, [_VP, ctypes.c_char_p, _I64P]),
    "tid_load": (_S, [_VP, _VP, ctypes.c_uint64, ctypes.c_int, _PP]),
    "tid_load_file": (_S, [_VP, ctypes.c_char_p, _PP]),
    "tid_graph_info": (_S, [_VP, _U64P, _PP]),
    "tid_graph_count": (_S, [_VP, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32, _U64P]),
    "tid_graph_free": (None, [_VP]),
    "tid_read_probe": (_S, [_VP, _VP, ctypes.c_uint64, ctypes.c_int32]),
    "tid_scan_keyed": (_S, [_VP, _VP, _VP, ctypes.c_int32, _VP, ctypes.c_int32, _PP]),
    "tid_entail": (_S, [_VP, _VP, ctypes.c_int32, _VP, _PP]),
    "tid_graph_partition": (_S, [_VP, _VP, ctypes.c_int32]),
    "tid_encode": (_S, [_VP, _VP, ctypes.c_uint64, _VP, ctypes.c_uint64, ctypes.c_int, _VP,
                        _PP]),
    "tid_dict_info": (_S, [_VP, _U64P, _U64P]),
    "tid_decode": (_S, [_VP, _VP, _VP, ctypes.c_uint64, ctypes.c_int, _VP, _VP,
                        ctypes.c_uint64]),
    "tid_dict_free": (None, [_VP]),
    "tid_serve_open": (_S, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _PP]),
    "tid_serve_submit": (_S, [_VP, _VP, _U64P]),
    "tid_serve_step": (_S, [_VP, _U64P, ctypes.c_int32, _I32P]),
    "tid_serve_result": (_S, [_VP, ctypes.c_uint64, _PP]),
    "tid_serve_info": (_S, [_VP, _I32P, _I32P, _I32P]),
    "tid_serve_close": (None, [_VP]),
    "tid_scan_noalloc": (_S, [_VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_uint64, _VP]),
    "tid_table_info": (_S, [_VP, _VP, _U64P, _I32P, _I32P]),
    "tid_table_column": (_S, [_VP, ctypes.c_int32, _PP]),
    "tid_table_to_host": (_S, [_VP, _VP, _VP, ctypes.c_uint64]),
    "tid_table_from_columns": (_S, [_VP, _PP, ctypes.c_int32, _I32P, ctypes.c_uint64,
                                    ctypes.c_int, _PP]),
    "tid_table_free": (None, [_VP]),
    "tid_scan": (_S, [_VP, _VP, ctypes.POINTER(tid_pattern), _PP]),
    "tid_scan_multi": (_S, [_VP, _VP, ctypes.POINTER(tid_pattern), ctypes.c_int32, _PP]),
    "tid_filter": (_S, [_VP, _VP, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32, _PP]),
    "tid_join": (_S, [_VP, _VP, ctypes.c_int32, _VP, ctypes.c_int32, ctypes.c_int32, _PP]),
    "tid_join_outer": (_S, [_VP, _VP, ctypes.c_int32, _VP, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32, _PP]),
    "tid_union": (_S, [_VP, _PP, ctypes.c_int32, ctypes.c_int32, _PP]),
    "tid_sort": (_S, [_VP, _VP, ctypes.c_int32, _PP]),
    "tid_query": (_S, [_VP, _VP, ctypes.POINTER(tid_plan), _PP]),
    "tid_query_batch": (_S, [_VP, _VP, ctypes.POINTER(ctypes.POINTER(tid_plan)), ctypes.c_int32,
                             _PP]),
    "tid_plan_estimate": (_S, [_VP, _VP, ctypes.POINTER(tid_plan), _U64P]),
}


def load_library(path: str = LIB_PATH):
    """Load libtid.so and declare every entry point.  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; "
            "g.build()').  There is no CPU fallback.")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
