"""ctypes binding of libbfc.so (the C ABI declared in include/bfc.h).

Argument marshalling only: every computation happens in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfc.so")

BFC_OK = 0
BFC_HASH_OFF = 0xFFFFFFFF
BFC_SIDE_AUTO, BFC_SIDE_L, BFC_SIDE_R = 0, 1, 2
ERROR_NAMES = {
    -1: "BFC_E_NULL", -2: "BFC_E_ARG", -3: "BFC_E_ID_RANGE", -4: "BFC_E_DUP_EDGE",
    -5: "BFC_E_TOO_LARGE", -6: "BFC_E_WS_SMALL", -7: "BFC_E_PROBS",
    -8: "BFC_E_OVERFLOW_RISK", -9: "BFC_E_HIP", -10: "BFC_E_ALIGN",
}

u32p = C.POINTER(C.c_uint32)
u64p = C.POINTER(C.c_uint64)


class bfc_graph(C.Structure):
    _fields_ = [
        ("n_left", C.c_uint32), ("n_right", C.c_uint32), ("n_edges", C.c_uint64),
        ("off_l", C.c_void_p), ("adj_l", C.c_void_p), ("eid_l", C.c_void_p),
        ("xpos_l", C.c_void_p), ("rank_l", C.c_void_p), ("id_l", C.c_void_p),
        ("off_r", C.c_void_p), ("adj_r", C.c_void_p), ("eid_r", C.c_void_p),
        ("xpos_r", C.c_void_p), ("rank_r", C.c_void_p), ("id_r", C.c_void_p),
        ("sumsq_l", C.c_uint64), ("sumsq_r", C.c_uint64),
        ("wedges_mid_l", C.c_uint64), ("wedges_mid_r", C.c_uint64),
        ("max_deg_l", C.c_uint32), ("max_deg_r", C.c_uint32),
        ("device", C.c_int),
    ]


class bfc_tuning(C.Structure):
    _fields_ = [("narrow_max", C.c_uint32), ("chunk", C.c_uint32),
                ("narrow_waves_per_cu", C.c_uint32), ("wide_groups_per_cu", C.c_uint32),
                ("hash_small_max", C.c_uint32), ("hash_mid_max", C.c_uint32),
                ("hash_passes", C.c_uint32), ("hash_max_density", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


BFC_REPLICA_ESPAR, BFC_REPLICA_CLRSPAR = 0, 1


class bfc_replica(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("ncolors", C.c_uint32), ("p", C.c_double),
                ("seed", C.c_uint64)]


class bfc_replica_info(C.Structure):
    _fields_ = [("kept", C.c_uint64), ("n_left", C.c_uint32), ("n_right", C.c_uint32),
                ("sumsq_left", C.c_uint64), ("sumsq_right", C.c_uint64)]


class BfcError(RuntimeError):
    def __init__(self, code, what=""):
        name = ERROR_NAMES.get(code, str(code))
        msg = f"{what}: {name}"
        if code == -9 and _lib is not None:
            msg += " (" + _lib.bfc_last_hip_error().decode() + ")"
        super().__init__(msg)
        self.code = code


# Exported symbols and their signatures (None restype = int status).
SIGNATURES = {
    "bfc_status_str": ([C.c_int], C.c_char_p),
    "bfc_last_hip_error": ([], C.c_char_p),
    "bfc_graph_storage_size": ([C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_graph_build_ws_size": ([C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_graph_build": ([C.c_uint32, C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p,
                         C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p,
                         C.POINTER(bfc_graph)], C.c_int),
    "bfc_graph_build_parts": ([C.c_uint32, C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p,
                               C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                               C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(bfc_graph)], C.c_int),
    "bfc_side_used": ([C.POINTER(bfc_graph), C.c_int], C.c_int),
    "bfc_wedges": ([C.POINTER(bfc_graph), C.c_int, u64p], C.c_int),
    "bfc_exact_ws_size": ([C.POINTER(bfc_graph), C.c_int, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_exact": ([C.POINTER(bfc_graph), C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                   C.c_void_p], C.c_int),
    "bfc_exact_plan": ([C.POINTER(bfc_graph), C.c_int, C.c_void_p, C.c_size_t, C.c_void_p],
                       C.c_int),
    "bfc_exact_count": ([C.POINTER(bfc_graph), C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                         C.c_void_p], C.c_int),
    "bfc_exact_noalloc": ([C.POINTER(bfc_graph), C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "bfc_local_ws_size": ([C.POINTER(bfc_graph), C.POINTER(C.c_size_t)], C.c_int),
    "bfc_local": ([C.POINTER(bfc_graph), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                   C.c_size_t, C.c_void_p], C.c_int),
    "bfc_local_split_ws_size": ([C.POINTER(bfc_graph), C.c_uint64, C.POINTER(C.c_size_t)],
                                C.c_int),
    "bfc_local_split": ([C.POINTER(bfc_graph), C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_per_vertex": ([C.POINTER(bfc_graph), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                        C.c_void_p], C.c_int),
    "bfc_per_edge": ([C.POINTER(bfc_graph), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
                     C.c_int),
    "bfc_probs_check_ws_size": ([C.POINTER(C.c_size_t)], C.c_int),
    "bfc_probs_check": ([C.c_void_p, C.c_uint64, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_spar_ws_size": ([C.POINTER(bfc_graph), C.POINTER(C.c_size_t)], C.c_int),
    "bfc_espar": ([C.POINTER(bfc_graph), C.c_double, C.c_uint64, C.c_void_p, C.c_void_p,
                   C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_clrspar": ([C.POINTER(bfc_graph), C.c_uint32, C.c_uint64, C.c_void_p, C.c_void_p,
                     C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_vsamp_ws_size": ([C.POINTER(bfc_graph), C.c_uint64, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_vsamp": ([C.POINTER(bfc_graph), C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p,
                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_vsamp_draws_ws_size": ([C.POINTER(bfc_graph), C.c_uint64, C.POINTER(C.c_size_t)],
                                C.c_int),
    "bfc_vsamp_draws": ([C.POINTER(bfc_graph), C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p,
                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_esamp_ws_size": ([C.POINTER(bfc_graph), C.c_uint64, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_esamp": ([C.POINTER(bfc_graph), C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p,
                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_esamp_fast_ws_size": ([C.POINTER(bfc_graph), C.c_uint64, C.POINTER(C.c_size_t)],
                               C.c_int),
    "bfc_esamp_fast": ([C.POINTER(bfc_graph), C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64,
                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
                       C.c_int),
    "bfc_wsamp_ws_size": ([C.POINTER(bfc_graph), C.c_uint64, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_wsamp": ([C.POINTER(bfc_graph), C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p,
                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_spar_threshold": ([C.c_int, C.c_double, C.c_uint32, C.POINTER(C.c_double),
                            C.POINTER(C.c_uint32)], C.c_int),
    "bfc_eps_delta_plan": ([C.c_double, C.c_double, C.POINTER(C.c_uint32),
                            C.POINTER(C.c_uint32)], C.c_int),
    "bfc_median_of_means": ([C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p,
                             C.c_void_p], C.c_int),
    "bfc_exact_tuned": ([C.POINTER(bfc_graph), C.c_int, C.POINTER(bfc_tuning), C.c_void_p,
                         C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_exact_parts_ws_size": ([C.POINTER(bfc_graph), C.POINTER(C.c_size_t)], C.c_int),
    "bfc_exact_parts": ([C.POINTER(bfc_graph), C.c_uint32, C.c_void_p, C.POINTER(bfc_tuning),
                         C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_autotune_ws_size": ([C.POINTER(bfc_graph), C.POINTER(C.c_size_t)], C.c_int),
    "bfc_autotune": ([C.POINTER(bfc_graph), C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                      C.c_size_t, C.c_void_p, C.POINTER(bfc_tuning), C.POINTER(C.c_float)],
                     C.c_int),
    "bfc_batch_union_ws_size": ([C.c_uint32, u32p, u32p, u64p, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_batch_union": ([C.c_uint32, u32p, u32p, u64p, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p, u32p, u32p, C.POINTER(C.c_uint8), C.c_void_p, C.c_size_t,
                         C.c_void_p], C.c_int),
    "bfc_spar_batch_filter_ws_size": ([C.POINTER(bfc_graph), C.c_uint32, C.POINTER(C.c_size_t)],
                                      C.c_int),
    "bfc_spar_batch_filter": ([C.POINTER(bfc_graph), C.c_uint32, C.POINTER(bfc_replica),
                               C.POINTER(bfc_replica_info), C.c_void_p, C.c_size_t, C.c_void_p],
                              C.c_int),
    "bfc_spar_batch_ws_size": ([C.POINTER(bfc_graph), C.c_uint32, C.POINTER(bfc_replica),
                                C.POINTER(bfc_replica_info), C.POINTER(C.c_size_t)], C.c_int),
    "bfc_spar_batch": ([C.POINTER(bfc_graph), C.c_uint32, C.POINTER(bfc_replica),
                        C.POINTER(bfc_replica_info),
                        C.POINTER(bfc_tuning), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                        C.c_void_p], C.c_int),
    "bfc_mlp_param_count": ([], C.c_int),
    "bfc_features": ([C.POINTER(bfc_graph), C.c_void_p, C.c_void_p], C.c_int),
    "bfc_mlp_bf16": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "bfc_mlp_forward": ([C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                        C.c_int),
    "bfc_mlp_targets": ([C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p], C.c_int),
    "bfc_mlp_grad_ws_size": ([C.c_uint32, C.POINTER(C.c_size_t)], C.c_int),
    "bfc_mlp_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "bfc_adam_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                       C.c_float, C.c_float, C.c_float, C.c_uint32, C.c_void_p], C.c_int),
    "bfc_probs_ws_size": ([C.POINTER(C.c_size_t)], C.c_int),
    "bfc_probs_from_predictions": ([C.c_void_p, C.c_uint64, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
}

_lib = None


def lib():
    """Load libbfc.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc, what=""):
    if rc != BFC_OK:
        raise BfcError(rc, what)
    return rc
