"""Order-preserving dictionary encoding of string columns (Section 2 of the
paper: plain encoding for numbers, an order-preserving dictionary for
strings, encode / decode to move between the forms).

A string column is a zero-padded uint8 tensor [n][L]; `encode` returns the
dictionary (the sorted distinct strings, [d][L]) and the int32 codes, which
the exact operators take as keys.  `literal_predicate` turns a comparison of
the column with a string literal into the equivalent comparison of the codes
(planner work on the host, from one lookup in the dictionary).
"""
from __future__ import annotations

import torch

from . import _lib as L
from .query import check_flags


def _status(dev):
    return torch.zeros(1, dtype=torch.int32, device=dev)


def encode(strs: torch.Tensor, max_distinct: int = 0):
    """(dictionary uint8 [d][L], codes int32 [n]) of a string column."""
    lib = L.load()
    if strs.dtype != torch.uint8 or strs.dim() != 2 or not strs.is_contiguous():
        raise TypeError("strings must be a contiguous uint8 [n][L] tensor")
    n, width = strs.shape
    dev = strs.device
    md = max_distinct or n
    dict_buf = torch.zeros((max(md, 1), width), dtype=torch.uint8, device=dev)
    codes = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    d_n = torch.zeros(1, dtype=torch.int64, device=dev)
    st = _status(dev)
    ws = L.workspace(lib.tdp_dict_build_workspace_size(n, max_distinct), dev)
    L.check("tdp_dict_build", lib.tdp_dict_build(L.ptr(strs), n, width, int(max_distinct), L.ptr(dict_buf), L.ptr(d_n),
                                                 L.ptr(codes), L.ptr(st), L.ptr(ws), ws.numel(), L.stream_handle(dev)))
    d = int(d_n.item())
    check_flags(st, "tdp_dict_build")
    return dict_buf[:d], codes[:n]


def lookup(dictionary: torch.Tensor, strs: torch.Tensor):
    """(pos int32, found int8): lower bound of each string in the dictionary."""
    lib = L.load()
    n, width = strs.shape
    dev = strs.device
    pos = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    found = torch.empty(max(n, 1), dtype=torch.int8, device=dev)
    L.check("tdp_dict_lookup", lib.tdp_dict_lookup(L.ptr(dictionary), dictionary.shape[0], width, L.ptr(strs), n,
                                                   L.ptr(pos), L.ptr(found), L.stream_handle(dev)))
    return pos[:n], found[:n]


def decode(dictionary: torch.Tensor, codes: torch.Tensor) -> torch.Tensor:
    lib = L.load()
    n = codes.numel()
    width = dictionary.shape[1]
    dev = codes.device
    out = torch.empty((max(n, 1), width), dtype=torch.uint8, device=dev)
    st = _status(dev)
    L.check("tdp_dict_decode", lib.tdp_dict_decode(L.ptr(codes), n, L.ptr(dictionary), dictionary.shape[0], width,
                                                   L.ptr(out), L.ptr(st), L.stream_handle(dev)))
    check_flags(st, "tdp_dict_decode")
    return out[:n]


def pad(words, width: int) -> torch.Tensor:
    """Byte strings -> zero-padded uint8 [len(words)][width] (host tensor)."""
    out = torch.zeros((len(words), width), dtype=torch.uint8)
    for i, w in enumerate(words):
        if len(w) > width or bytes(1) in w:
            raise ValueError(f"{w!r} does not fit a width of {width} without zero bytes")
        if w:
            out[i, :len(w)] = torch.tensor(list(w), dtype=torch.uint8)
    return out


def literal_predicate(dictionary: torch.Tensor, op: str, literal: bytes):
    """(op, code literal) with `code op' lit'` true exactly when
    `string op literal` is: with lb the literal's lower bound and f = 1 when
    it is in the dictionary, s < lit  <=>  code < lb;  s <= lit  <=>
    code < lb + f;  s > lit  <=>  code >= lb + f;  s >= lit  <=>  code >= lb;
    s == lit  <=>  code == lb when f (no row otherwise: code == -1);
    s != lit  <=>  code != lb when f (every row otherwise: code != -1)."""
    lit = pad([literal], dictionary.shape[1]).to(dictionary.device)
    pos, found = lookup(dictionary, lit)
    lb, f = int(pos.item()), int(found.item())
    return {"<": ("<", lb), "<=": ("<", lb + f), ">": (">=", lb + f), ">=": (">=", lb),
            "==": ("==", lb if f else -1), "!=": ("!=", lb if f else -1)}[op]
