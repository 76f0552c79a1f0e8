"""ctypes loader for libttround.so (argument marshalling only).

The library must have been built (``paper_2110_04393_amd.build.build()``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttround.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tt_round.h")

TT_OK, TT_EINVAL, TT_ENOMEM, TT_EHIP, TT_ENUMERIC, TT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
TT_F64, TT_F32, TT_BF16 = 0, 1, 2
TT_PREC_F64, TT_PREC_F32, TT_PREC_MIXED_BF16 = 0, 1, 2
TT_BATCH_GRAPH, TT_BATCH_AUTOTUNE = 1, 2

_STATUS_NAMES = {0: "TT_OK", -1: "TT_EINVAL", -2: "TT_ENOMEM", -3: "TT_EHIP",
                 -4: "TT_ENUMERIC", -5: "TT_EUNSUPPORTED"}

c_i32, c_i64, c_u64, c_dbl, c_size = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_double, ctypes.c_size_t)
P_i64 = ctypes.POINTER(c_i64)
P_dbl = ctypes.POINTER(c_dbl)
P_size = ctypes.POINTER(c_size)
P_vp = ctypes.POINTER(ctypes.c_void_p)
vp = ctypes.c_void_p


class TTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_SIGS = {
    "tt_last_error": (ctypes.c_char_p, []),
    "tt_version": (ctypes.c_int, []),
    "tt_round_rand_plan": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, c_i64, P_i64, P_i64]),
    "tt_round_rand_workspace": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, c_i64, c_i32, P_size]),
    "tt_make_sketch": (ctypes.c_int, [c_u64, c_i32, P_i64, P_i64, c_i32, P_vp, vp]),
    "tt_partial_contractions_rl_workspace": (ctypes.c_int, [c_i32, P_i64, P_i64, P_i64, c_i32,
                                                            P_size]),
    "tt_partial_contractions_rl": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, P_i64, P_vp, c_i32,
                                                  P_vp, vp, c_size, vp]),
    "tt_round_rand": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_i64, c_i64, c_u64,
                                     c_i32, P_vp, vp, c_size, vp]),
    "tt_round_rand_eps_workspace": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, c_i32, P_size]),
    "tt_round_rand_eps": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_i64, c_dbl, c_u64,
                                         c_i32, P_vp, P_i64, vp, c_size, vp]),
    "tt_sum_round_eps_workspace": (ctypes.c_int, [c_i32, c_i32, P_i64, P_i64, c_i64, c_i32,
                                                  P_size]),
    "tt_sum_round_eps": (ctypes.c_int, [c_i32, c_i32, P_i64, P_i64, P_vp, P_dbl, c_i32, c_i64,
                                        c_dbl, c_u64, c_i32, P_vp, P_i64, vp, c_size, vp]),
    "tt_round_orth_rand_plan": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, c_i64, P_i64, P_i64]),
    "tt_round_orth_rand_workspace": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, c_i64, c_i32,
                                                    P_size]),
    "tt_round_orth_rand": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_i64, c_i64, c_u64,
                                          c_i32, P_vp, vp, c_size, vp]),
    "tt_gmres_workspace": (ctypes.c_int, [c_i32, P_i64, c_i32, P_i64, c_i64, c_i32, P_size]),
    "tt_gmres": (ctypes.c_int, [c_i32, P_i64, c_i32, P_vp, vp, P_i64, P_vp, c_i32, c_i64, c_dbl,
                                c_dbl, c_i32, c_u64, P_vp, P_i64, P_dbl,
                                ctypes.POINTER(c_i32), vp, c_size, vp]),
    "tt_round_rand_noalloc": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_i64, c_i64,
                                             c_u64, c_i32, P_vp, vp]),
    "tt_round_rand_with_sketch": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_i64, c_i64,
                                                 P_i64, P_vp, c_i32, P_vp, vp, c_size, vp]),
    "tt_sum_round_workspace": (ctypes.c_int, [c_i32, c_i32, P_i64, P_i64, c_i64, c_i64, c_i32,
                                              P_size]),
    "tt_round_svd_plan": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, P_i64]),
    "tt_round_svd_workspace": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, c_i32, P_size]),
    "tt_round_svd": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_dbl, c_i64, c_i32, P_vp,
                                    P_i64, vp, c_size, vp]),
    "tt_round_two_sided_plan": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, P_i64, P_i64]),
    "tt_round_two_sided_workspace": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, P_size]),
    "tt_round_two_sided": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_i64, c_u64, c_u64,
                                          P_vp, vp, c_size, vp]),
    "tt_round_rand_backward_workspace": (ctypes.c_int, [c_i32, P_i64, P_i64, c_i64, c_i64, c_i32,
                                                        P_size]),
    "tt_round_rand_backward": (ctypes.c_int, [c_i32, P_i64, P_i64, P_vp, c_i32, c_i64, c_i64, c_u64,
                                              c_i32, P_vp, P_vp, vp, c_size, vp]),
    "tt_batch_workspace": (ctypes.c_int, [c_i32, ctypes.POINTER(c_i32), P_i64, P_i64, P_i64, P_i64,
                                          c_i32, P_size]),
    "tt_batch_create": (ctypes.c_int, [c_i32, ctypes.POINTER(c_i32), P_i64, P_i64, P_i64, P_i64,
                                       ctypes.POINTER(c_u64), c_i32, c_i32, P_vp, P_vp, vp, c_size,
                                       c_i32, vp, P_vp]),
    "tt_batch_run": (ctypes.c_int, [vp, vp]),
    "tt_batch_info": (ctypes.c_int, [vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                                     ctypes.POINTER(c_i32)]),
    "tt_batch_destroy": (ctypes.c_int, [vp]),
    "tt_timing_start": (ctypes.c_int, [c_i32, c_i32]),
    "tt_timing_stop": (ctypes.c_int, [P_dbl, ctypes.POINTER(c_i32)]),
    "tt_sum_round": (ctypes.c_int, [c_i32, c_i32, P_i64, P_i64, P_vp, P_dbl, c_i32, c_i64, c_i64,
                                    c_u64, c_i32, P_vp, vp, c_size, vp]),
}

_lib = None


def header_functions():
    """Names of the functions include/tt_round.h declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"TT_API\s+[\w\s\*]*?\b(tt_\w+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2110_04393_amd.build` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != TT_OK:
        msg = lib().tt_last_error().decode(errors="replace")
        raise TTError(status, msg)


def i64_array(vals):
    vals = [int(v) for v in vals]
    return (c_i64 * max(1, len(vals)))(*vals)


def ptr_array(ptrs):
    ptrs = [int(p) for p in ptrs]
    return (ctypes.c_void_p * max(1, len(ptrs)))(*ptrs)
