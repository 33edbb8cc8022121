"""ctypes view of libtdp.so (the C ABI declared in include/tdp.h).

Only argument marshalling lives here; every step of every operator runs in
the library's HIP kernels.  Importing this module on a machine without the
built library raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdp.so")

TDP_OK, TDP_EINVAL, TDP_ECAPACITY, TDP_EWORKSPACE, TDP_EUNSUPPORTED, TDP_EDEVICE = 0, -1, -2, -3, -4, -5
FLAG_KEY_DOMAIN, FLAG_DUP_BUILD, FLAG_GROUP_RANGE, FLAG_TABLE_FULL, FLAG_SPIN, FLAG_BAD_PARAM = 1, 2, 4, 8, 16, 32
I8, I32, I64, F32 = 1, 2, 3, 4
LT, LE, GT, GE, EQ, NE = range(6)
PROBE, BUILD = 0, 1
JOIN_PAIRS, JOIN_COUNT = 0, 1
EXPR_COL, EXPR_MUL, EXPR_MUL_CONST_SUB, EXPR_NONE = range(4)
PROBE_AUTO, PROBE_DIRECT, PROBE_STAGED, PROBE_PARTITIONED = range(4)
STAGE_NONE, STAGE_RP_SCATTER, STAGE_RP_PROBE, STAGE_FUSED_PROBE = range(4)

CMP = {"<": LT, "<=": LE, ">": GT, ">=": GE, "==": EQ, "!=": NE}
DTYPE = {torch.int8: I8, torch.int32: I32, torch.int64: I64, torch.float32: F32}


class Col(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("side", C.c_int32), ("n", C.c_int64)]


class JoinDesc(C.Structure):
    _fields_ = [("build_key", C.c_void_p), ("n_build", C.c_int64), ("probe_key", C.c_void_p), ("n_probe", C.c_int64),
                ("probe_sel", C.c_void_p), ("n_probe_sel", C.c_int64), ("build_unique", C.c_int32),
                ("load_pct", C.c_int32), ("max_distinct", C.c_int64)]


class Pred(C.Structure):
    _fields_ = [("col", Col), ("cmp", C.c_int32), ("reserved", C.c_int32), ("literal", C.c_int64),
                ("literal_f", C.c_double)]


MAX_MORE_PREDS = 3


class GroupbyDesc(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("has_pred", C.c_int32), ("pred_cmp", C.c_int32), ("pred_literal", C.c_int64),
                ("pred", Col), ("sel", C.c_void_p), ("n_sel", C.c_int64), ("join", C.POINTER(JoinDesc)),
                ("n_keys", C.c_int32), ("expr", C.c_int32), ("key", Col * 2), ("key_lo", C.c_int64 * 2),
                ("key_card", C.c_int64 * 2), ("a", Col), ("b", Col), ("k", C.c_int64), ("topk", C.c_int32),
                ("strategy", C.c_int32), ("more_preds", C.POINTER(Pred)), ("n_more_preds", C.c_int32),
                ("reserved", C.c_int32)]


class GroupbyOut(C.Structure):
    _fields_ = [("cap", C.c_int64), ("d_n_groups", C.c_void_p), ("key0", C.c_void_p), ("key1", C.c_void_p),
                ("sum", C.c_void_p), ("count", C.c_void_p), ("avg", C.c_void_p)]


class AdamTensor(C.Structure):
    _fields_ = [("p", C.c_void_p), ("g", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("p_bf16", C.c_void_p),
                ("n", C.c_int64)]


class TdpError(RuntimeError):
    def __init__(self, fn, code, text):
        super().__init__(f"{fn} failed with status {code} ({text})")
        self.code = code


_lib = None

_SIGS = {
    "tdp_status_string": (C.c_char_p, [C.c_int]),
    "tdp_last_error": (C.c_char_p, []),
    "tdp_last_needed": (C.c_int64, []),
    "tdp_stage_timer": (C.c_int, [C.c_int]),
    "tdp_stage_time": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "tdp_filter_workspace_size": (C.c_size_t, [C.c_int64]),
    "tdp_filter": (C.c_int, [C.POINTER(Col), C.c_int32, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_filter_noalloc_max_candidates": (C.c_int64, []),
    "tdp_filter_noalloc": (C.c_int, [C.POINTER(Col), C.c_int32, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_hash_join_workspace_size": (C.c_size_t, [C.POINTER(JoinDesc)]),
    "tdp_hash_join": (C.c_int, [C.POINTER(JoinDesc), C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_groupby_workspace_size": (C.c_size_t, [C.POINTER(GroupbyDesc)]),
    "tdp_groupby_agg": (C.c_int, [C.POINTER(GroupbyDesc), C.POINTER(GroupbyOut), C.c_void_p, C.c_void_p, C.c_size_t,
                                  C.c_void_p]),
    "tdp_groupby_build": (C.c_int, [C.POINTER(GroupbyDesc), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_groupby_probe": (C.c_int, [C.POINTER(GroupbyDesc), C.POINTER(GroupbyOut), C.c_void_p, C.c_void_p,
                                    C.c_size_t, C.c_void_p]),
    "tdp_soft_workspace_size": (C.c_size_t, []),
    "tdp_soft_workspace_init": (C.c_int, [C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_soft_filter": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_float, C.c_void_p, C.c_void_p]),
    "tdp_soft_filter_bwd": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_float, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_soft_groupby": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_soft_groupby_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                       C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_soft_pe_groupby": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                      C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_soft_pe_groupby_bwd": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                          C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_soft_filter_groupby": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_float,
                                          C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_soft_filter_groupby_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_float,
                                              C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_soft_query": (C.c_int, [C.POINTER(GroupbyDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_soft_query_bwd": (C.c_int, [C.POINTER(GroupbyDesc), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_llp_bag_count": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int64,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p]),
    "tdp_llp_workspace_size": (C.c_size_t, [C.c_int32]),
    "tdp_llp_bag_count_bwd": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                        C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                        C.c_void_p]),
    "tdp_llp_predict": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                  C.c_void_p]),
    "tdp_count_table": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                  C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_segment_ids": (C.c_int, [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "tdp_dict_build_workspace_size": (C.c_size_t, [C.c_int64, C.c_int64]),
    "tdp_dict_build": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tdp_dict_lookup": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "tdp_dict_decode": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "tdp_mse_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_image_to_bf16": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "tdp_f32_to_bf16": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "tdp_conv3x3_fwd_bf16": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_int] * 6 + [C.c_void_p, C.c_void_p]),
    "tdp_conv3x3_dgrad_bf16": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_int] * 5 + [C.c_void_p, C.c_void_p]),
    "tdp_conv3x3_wgrad_bf16": (C.c_int, [C.c_void_p, C.c_void_p] + [C.c_int] * 5 + [C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_linear_fwd_bf16": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_int] * 4 +
                            [C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_linear_dgrad_bf16": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_int] * 3 + [C.c_void_p, C.c_void_p]),
    "tdp_linear_wgrad_bf16": (C.c_int, [C.c_void_p, C.c_void_p] + [C.c_int] * 3 + [C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_maxpool2_fwd_bf16": (C.c_int, [C.c_void_p] + [C.c_int] * 4 + [C.c_void_p, C.c_void_p]),
    "tdp_maxpool2_bwd_bf16": (C.c_int, [C.c_void_p, C.c_void_p] + [C.c_int] * 5 + [C.c_void_p, C.c_void_p]),
    "tdp_softmax_expect_fwd": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_softmax_expect_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "tdp_softmax_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tdp_argmax_rows": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "tdp_adam_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_float,
                                C.c_float, C.c_float, C.c_int, C.c_void_p, C.c_void_p]),
    "tdp_adam_step_multi": (C.c_int, [C.c_void_p, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int,
                                      C.c_void_p]),
}

OPTIONAL_SIGS: dict = {}


def declared_symbols():
    """Names of every function the binding declares (all of include/tdp.h)."""
    return sorted(list(_SIGS) + list(OPTIONAL_SIGS))


def load():
    """Load libtdp.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in {**_SIGS, **OPTIONAL_SIGS}.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(fn: str, code: int):
    if code != TDP_OK:
        L = load()
        text = L.tdp_last_error().decode()
        if code in (TDP_ECAPACITY, TDP_EWORKSPACE):
            text += f" (needed {int(L.tdp_last_needed())})"
        raise TdpError(fn, code, text)


def ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def stream_handle(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def col(t: torch.Tensor, side: int = PROBE) -> Col:
    if not t.is_contiguous():
        raise ValueError("columns must be contiguous")
    return Col(t.data_ptr(), DTYPE[t.dtype], side, t.numel())


def segment_ids(n: int, width: int, device) -> torch.Tensor:
    """int32 [n] with i // width (library kernel)."""
    out = torch.empty(max(int(n), 1), dtype=torch.int32, device=device)
    check("tdp_segment_ids", load().tdp_segment_ids(int(n), int(width), ptr(out), stream_handle(device)))
    return out[:n]


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def stage_timer(stage: int):
    """Select the stage whose launches are bracketed by HIP events (clears the record)."""
    check("tdp_stage_timer", load().tdp_stage_timer(int(stage)))


def stage_time():
    """(total ms, launches) timed since the last stage_timer call."""
    t = C.c_double(0.0)
    n = C.c_int64(0)
    check("tdp_stage_time", load().tdp_stage_time(C.byref(t), C.byref(n)))
    return t.value, int(n.value)
