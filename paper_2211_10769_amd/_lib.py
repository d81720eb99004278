"""ctypes binding of libswh.so (declarations mirror include/swh.h).

Argument marshalling only: every step of the alignment runs in the HIP
library.  Importing this module fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswh.so")

SWH_OK = 0
STATUS_NAMES = {0: "SWH_OK", -1: "SWH_E_INVAL", -2: "SWH_E_ALPHABET", -3: "SWH_E_NOMEM",
                -4: "SWH_E_RANGE", -5: "SWH_E_DEVICE", -6: "SWH_E_TIMEOUT", -7: "SWH_E_CANCELLED"}
MODE_SCORE, MODE_COORDS, MODE_CIGAR = 0, 1, 2
# context options (swh_set_option)
OPTIONS = {"rows_per_lane": 1, "grid": 2, "band_rows": 3, "tb_leaf": 4, "graph": 5, "prune": 6, "mem_cap": 7,
           "int16": 8, "inter_max": 9, "fault_nomem": 10, "pf_rank": 11, "db_waves": 12, "db_route": 13}
GLOBAL = 0x100          # OR'd into mode: global (Needleman-Wunsch) alignment
SEMIGLOBAL = 0x200      # OR'd into mode: semi-global (whole query, free target ends)
OVERLAP = 0x400         # OR'd into mode: overlap (end gaps of both sequences free)


class swh_scoring(ctypes.Structure):
    _fields_ = [("alphabet", ctypes.c_char_p), ("alphabet_size", ctypes.c_int32),
                ("matrix", ctypes.c_void_p), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32)]


class swh_alignment(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("q_begin", ctypes.c_int64), ("q_end", ctypes.c_int64),
                ("t_begin", ctypes.c_int64), ("t_end", ctypes.c_int64)]


class swh_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("cells_forward", ctypes.c_double), ("ms_forward", ctypes.c_double),
                ("ms_reverse", ctypes.c_double), ("ms_traceback", ctypes.c_double),
                ("cells_traceback", ctypes.c_double), ("traceback_bands", ctypes.c_int64),
                ("traceback_retries", ctypes.c_int64), ("passes_int16", ctypes.c_int64),
                ("saturated_int16", ctypes.c_int64)]


class swh_hit(ctypes.Structure):
    _fields_ = [("db_index", ctypes.c_int64), ("score", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class swh_search_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("cells", ctypes.c_double), ("ms_inter", ctypes.c_double), ("ms_intra", ctypes.c_double),
                ("ms_topk", ctypes.c_double), ("saturated", ctypes.c_int64), ("intra_pairs", ctypes.c_int64),
                ("graph", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class swh_tune_entry(ctypes.Structure):
    _fields_ = [("max_rows", ctypes.c_int64), ("rows_per_lane", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32)]


class swh_train_cfg(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("epochs", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_double), ("seed", ctypes.c_uint64)]


class swh_train_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("first_epoch_loss", ctypes.c_double), ("final_epoch_loss", ctypes.c_double),
                ("ms_label", ctypes.c_double), ("ms_features", ctypes.c_double), ("ms_train", ctypes.c_double),
                ("cells_label", ctypes.c_double), ("steps", ctypes.c_int64), ("graph", ctypes.c_int32),
                ("reserved2", ctypes.c_int32)]


class swh_prefilter_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("candidates", ctypes.c_int64), ("audited", ctypes.c_int64), ("fallbacks", ctypes.c_int64),
                ("cells_rescored", ctypes.c_double), ("cells_exhaustive", ctypes.c_double),
                ("ms_features", ctypes.c_double), ("ms_predict", ctypes.c_double), ("ms_select", ctypes.c_double),
                ("ms_rescore", ctypes.c_double), ("ms_topk", ctypes.c_double), ("ms_fallback", ctypes.c_double)]


MODEL_PARAMS = 168961
MODEL_INPUTS = 401

# name -> (restype, argtypes); the C-ABI surface declared in include/swh.h
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I64P = ctypes.POINTER(ctypes.c_int64)
SIGNATURES = {
    "swh_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)]),
    "swh_destroy": (None, [_P]),
    "swh_last_error": (ctypes.c_char_p, [_P]),
    "swh_cancel": (ctypes.c_int, [_P]),
    "swh_set_option": (ctypes.c_int, [_P, ctypes.c_int32, _I64]),
    "swh_get_option": (ctypes.c_int, [_P, ctypes.c_int32, _I64P]),
    "swh_align": (ctypes.c_int, [_P, _P, _I64, _P, _I64, ctypes.POINTER(swh_scoring), ctypes.c_int,
                                 ctypes.POINTER(swh_alignment), _P, _I64, _I64P,
                                 ctypes.POINTER(swh_stats)]),
    "swh_align_dev": (ctypes.c_int, [_P, _P, _I64, _P, _I64, ctypes.POINTER(swh_scoring), ctypes.c_int,
                                     _P, ctypes.POINTER(swh_alignment), _P, _I64, _I64P,
                                     ctypes.POINTER(swh_stats)]),
    "swh_align_dev_noalloc": (ctypes.c_int, [ctypes.c_int, _P, _I64, _P, _I64, ctypes.POINTER(swh_scoring),
                                             ctypes.c_int, _P, ctypes.POINTER(swh_alignment)]),
    "swh_align_batch": (ctypes.c_int, [_P, _I64, _P, _P, _P, _P, ctypes.POINTER(swh_scoring), ctypes.c_int,
                                       _P, _P, _I64, _P, ctypes.POINTER(swh_stats)]),
    "swh_align_batch_dev": (ctypes.c_int, [_P, _I64, _P, _P, _P, _P, ctypes.POINTER(swh_scoring), ctypes.c_int,
                                           _P, _P, _P, _I64, _P, ctypes.POINTER(swh_stats)]),
    "swh_autotune": (ctypes.c_int, [_P, ctypes.POINTER(swh_scoring), _I64, ctypes.c_double]),
    "swh_autotune_db": (ctypes.c_int, [_P, ctypes.POINTER(swh_scoring), ctypes.POINTER(ctypes.c_int32)]),
    "swh_tune_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "swh_tune_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "swh_tune_get": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "swh_tune_set": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "swh_model_create": (ctypes.c_int, [_P, ctypes.POINTER(swh_scoring), _P, _P, _P, ctypes.c_uint64,
                                        ctypes.POINTER(_P)]),
    "swh_model_destroy": (None, [_P]),
    "swh_model_get": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "swh_model_set": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "swh_model_save": (ctypes.c_int, [_P, _P, ctypes.c_char_p]),
    "swh_model_load": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.POINTER(_P)]),
    "swh_prefilter_train": (ctypes.c_int, [_P, _P, ctypes.POINTER(swh_scoring), _I64, _P, _P, _I64, _P, _P, _P,
                                           ctypes.POINTER(swh_train_cfg), _P, ctypes.POINTER(swh_train_stats)]),
    "swh_prefilter_search": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_uint64, _P,
                                            ctypes.POINTER(swh_prefilter_stats)]),
    "swh_prefilter_predict": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, _P]),
    "swh_dipeptide_counts": (ctypes.c_int, [_P, ctypes.POINTER(swh_scoring), _I64, _P, _P, _P]),
    "swh_mlp_grad": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "swh_mlp_train_steps": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_double]),
    "swh_db_create": (ctypes.c_int, [_P, _I64, _P, _P, ctypes.POINTER(swh_scoring), ctypes.POINTER(_P)]),
    "swh_db_destroy": (None, [_P]),
    "swh_db_search": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P,
                                     ctypes.POINTER(swh_search_stats)]),
    "swh_db_search_dev": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P,
                                         ctypes.POINTER(swh_search_stats)]),
    "swh_db_scores": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, ctypes.POINTER(swh_search_stats)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libswh.so; raises RuntimeError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        # PyTorch ships its own HIP runtime under the same soname
        # (libamdhip64.so.7).  Loaded first, it is the one libswh.so binds to,
        # so the process holds a single runtime and device pointers and
        # streams from torch are valid in the library; loaded after libswh.so
        # it would be a second runtime that cannot initialise the device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
