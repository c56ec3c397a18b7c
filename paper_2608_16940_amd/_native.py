"""ctypes binding of libsv.so (argument marshalling only).

Every function here forwards to the C-ABI declared in ``include/*.h``.  There
is no fallback: if the library has not been built, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsv.so")

SV_OK = 0
SV_ERR_ARG = -1
SV_ERR_DEVICE = -2
SV_ERR_UNSUPPORTED = -3
SV_ERR_STATE = -4

NOALLOC_MAX_QUBITS = 26

OPT_VARIANT = 1
OPT_PRECISION = 2
OPT_MFMA_MIN_K = 3
OPT_LAZY_RELABEL = 4
OPT_LOW_BITS = 5
OPT_MFMA_OPERAND = 6
OPT_POLICY = 7
OPT_TILE_ORDER = 8
POLICY = {"belady": 0, "first_free": 1, "lru": 2}
MFMA_OPERAND = {"regs": 0, "lds": 1, "global": 2, "auto": 3}

SCORE = {"paper": 0, "learned": 1, "roofline": 2}

VARIANT = {"auto": 0, "valu": 1, "shuffle": 2, "mfma": 3, "generic": 4, "diag": 5}
PRECISION = {"fp32": 0, "bf16x3": 1}


class SvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libsv error %d: %s" % (code, msg))
        self.code = code


class sv_stats(ctypes.Structure):
    _fields_ = [("gate_sweeps", ctypes.c_int64), ("swap_half_sweeps", ctypes.c_int64),
                ("relabels", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("by_variant", ctypes.c_int64 * 6), ("permute_sweeps", ctypes.c_int64),
                ("layout_only", ctypes.c_int64), ("diag_chunks", ctypes.c_int64)]


class sv_batch_circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("kinds", ctypes.POINTER(ctypes.c_int32)), ("qubits", ctypes.POINTER(ctypes.c_int32)),
                ("mats", ctypes.POINTER(ctypes.c_double))]


BATCH_CONFIG_LEN = 19

_lib = None

# (name, restype, argtypes) of every exported entry point
_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
SIGNATURES = [
    ("sv_workspace_bytes", ctypes.c_size_t, [ctypes.c_int]),
    ("sv_alloc", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp]),
    ("sv_free", ctypes.c_int, [_vp]),
    ("sv_reset", ctypes.c_int, [_vp]),
    ("sv_apply_fused", ctypes.c_int, [_vp, _dp, _i32p, ctypes.c_int]),
    ("sv_permute_layout", ctypes.c_int, [_vp, _i32p]),
    ("sv_get_layout", ctypes.c_int, [_vp, _i32p]),
    ("sv_probs", ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    ("sv_norm", ctypes.c_int, [_vp, _dp]),
    ("sv_sample", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int64, _u64p]),
    ("sv_sample_probs", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, _u64p, _vp,
                                       ctypes.c_size_t, _vp]),
    ("sv_sample_probs_noalloc", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, _u64p, _vp]),
    ("sv_sync", ctypes.c_int, [_vp]),
    ("sv_copy_out", ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    ("sv_dm_state_bytes", ctypes.c_size_t, [ctypes.c_int]),
    ("sv_dm_workspace_bytes", ctypes.c_size_t, [ctypes.c_int]),
    ("sv_dm_alloc", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t,
                                   _vp]),
    ("sv_dm_qubits", ctypes.c_int, [_vp]),
    ("sv_dm_superop", ctypes.c_int, [_dp, ctypes.c_int, ctypes.c_int, _dp]),
    ("sv_dm_apply_channel", ctypes.c_int, [_vp, _dp, ctypes.c_int, _i32p, ctypes.c_int]),
    ("sv_dm_probs", ctypes.c_int, [_vp, _vp]),
    ("sv_dm_trace", ctypes.c_int, [_vp, _dp]),
    ("sv_dm_sample", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int64, _u64p, _vp]),
    ("sv_last_error", ctypes.c_char_p, []),
    ("sv_set_option", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    ("sv_get_option", ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    ("sv_get_stats", ctypes.c_int, [_vp, ctypes.POINTER(sv_stats)]),
    ("sv_plan_greedy", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, _dp, ctypes.POINTER(ctypes.c_int8),
                                      ctypes.c_int, ctypes.POINTER(_vp)]),
    ("sv_plan_num_blocks", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    ("sv_plan_block_info", ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _i32p,
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    ("sv_plan_block_matrix", ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    ("sv_run_plan", ctypes.c_int, [_vp, _vp]),
    ("sv_plan_free", ctypes.c_int, [_vp]),
    ("sv_batch_prepare", ctypes.c_int, [ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64), _i32p,
                                        _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    ("sv_batch_launch", ctypes.c_int, [_vp, _vp, _dp, _vp]),
    ("sv_batch_prepared_free", ctypes.c_int, [_vp]),
    ("sv_batch_records", ctypes.c_int, [_vp, ctypes.c_int, _i32p, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_int)]),
    ("sv_bound_bytes", ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]),
    ("sv_plan_bind", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    ("sv_bound_run", ctypes.c_int, [_vp]),
    ("sv_bound_graph_run", ctypes.c_int, [_vp]),
    ("sv_bound_free", ctypes.c_int, [_vp]),
    ("sv_hint_next_use", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    ("sv_mlp_param_count", ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    ("sv_mlp_cache_floats", ctypes.c_int64, [ctypes.c_int, ctypes.c_int]),
    ("sv_mlp_forward", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp]),
    ("sv_mlp_backward", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp,
                                       _vp]),
    ("sv_mlp_adam", ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, _vp]),
    ("sv_mlp_forward_host", ctypes.c_int, [ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_float), ctypes.c_int, _dp]),
    ("sv_plan_swaps", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.POINTER(ctypes.c_int)]),
    ("sv_plan_block_swap", ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _i32p]),
    ("sv_plan_dp", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, _dp, ctypes.POINTER(ctypes.c_int8),
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(_vp)]),
    ("sv_cost_features", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_float)]),
    ("sv_diag_sweep_cost", ctypes.c_int, [ctypes.c_int, _dp, _i32p, _dp, ctypes.POINTER(ctypes.c_int)]),
    ("sv_batch_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(sv_batch_circuit)]),
    ("sv_batch_run", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(sv_batch_circuit), _vp, ctypes.c_size_t,
                                    ctypes.POINTER(ctypes.c_int64), _dp, _i32p, _vp, ctypes.c_size_t, _vp]),
    ("sv_batch_autotune", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(sv_batch_circuit), _vp, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_int, _i32p, _dp, _vp,
                                         ctypes.c_size_t, _vp]),
    ("sv_policy_simulate", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _i32p,
                                          ctypes.POINTER(ctypes.c_int64)]),
]


def lib():
    """Load libsv.so (raises if it has not been built; there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsv.so not built at %s; run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> int:
    if rc != SV_OK:
        msg = lib().sv_last_error()
        raise SvError(rc, msg.decode() if msg else "")
    return rc
