"""The C-ABI library loads and exports every symbol include/tdp.h declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdp.h")
LIB = os.path.join(ROOT, "paper_2211_02753_amd", "libtdp.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtdp.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_operator_calls():
    names = declared()
    for must in ["tdp_filter", "tdp_hash_join", "tdp_groupby_agg", "tdp_soft_filter", "tdp_soft_filter_bwd",
                 "tdp_soft_groupby", "tdp_soft_groupby_bwd", "tdp_soft_filter_groupby", "tdp_soft_filter_groupby_bwd"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (tdp_\w+)", out))
    assert set(declared()) <= exported


def test_binding_declares_every_symbol():
    from paper_2211_02753_amd import _lib
    assert set(declared()) == set(_lib.declared_symbols())


def test_host_side_validation_without_launch(lib):
    """Argument errors return before any launch, so they are testable here."""
    from paper_2211_02753_amd import _lib
    L = _lib.load()
    assert L.tdp_status_string(-3) == b"workspace too small"
    # null column
    rc = L.tdp_filter(None, 0, 0, None, 0, None, 0, None, None, None, 0, None)
    assert rc == _lib.TDP_EINVAL
    c = _lib.Col(0x1000, _lib.I32, 0, 100)
    n_out = ctypes.c_int64()
    rc = L.tdp_filter(ctypes.byref(c), 0, 0, None, 0, ctypes.c_void_p(0x2000), 10, ctypes.byref(n_out), None,
                      ctypes.c_void_p(0x4000), 1 << 20, None)
    assert rc == _lib.TDP_ECAPACITY
    assert L.tdp_last_needed() == 100  # the candidates rows_out must hold
    assert b"cap" in L.tdp_last_error()
    rc = L.tdp_filter(ctypes.byref(c), 0, 0, None, 0, ctypes.c_void_p(0x2000), 100, ctypes.byref(n_out), None,
                      ctypes.c_void_p(0x4000), 16, None)
    assert rc == _lib.TDP_EWORKSPACE
    c.dtype = _lib.F32
    rc = L.tdp_filter(ctypes.byref(c), 0, 0, None, 0, ctypes.c_void_p(0x2000), 100, ctypes.byref(n_out), None,
                      ctypes.c_void_p(0x4000), 1 << 20, None)
    assert rc == _lib.TDP_EUNSUPPORTED
    # tau must be positive
    assert L.tdp_soft_filter(ctypes.c_void_p(0x1000), 10, ctypes.c_void_p(0x10), 0.0, ctypes.c_void_p(0x2000), None) \
        == _lib.TDP_EINVAL
    # soft group-by K/G range
    assert L.tdp_soft_groupby(ctypes.c_void_p(0x10), None, ctypes.c_void_p(0x10), 4, 17, 3, ctypes.c_void_p(0x10),
                              None, None, 0, None) == _lib.TDP_EINVAL


def test_groupby_plan_validation(lib):
    from paper_2211_02753_amd import _lib
    L = _lib.load()
    d = _lib.GroupbyDesc()
    d.n_rows = 10
    d.n_keys = 1
    d.expr = _lib.EXPR_NONE
    d.key[0] = _lib.Col(0x1000, _lib.I32, _lib.PROBE, 10)
    d.key_lo[0] = 0
    d.key_card[0] = 4
    assert L.tdp_groupby_workspace_size(ctypes.byref(d)) > 0
    d.key_card[0] = 0
    assert L.tdp_groupby_workspace_size(ctypes.byref(d)) == 0
    d.key_card[0] = 4
    # build-side key without a join
    d.key[0] = _lib.Col(0x1000, _lib.I32, _lib.BUILD, 10)
    assert L.tdp_groupby_agg(ctypes.byref(d), None, None, None, 0, None) == _lib.TDP_EINVAL
    # non-unique build with a build-side group key is unsupported
    jd = _lib.JoinDesc(0x2000, 5, 0x3000, 10, None, 0, 0, 0, 0)
    d.join = ctypes.pointer(jd)
    assert L.tdp_groupby_agg(ctypes.byref(d), None, None, None, 0, None) == _lib.TDP_EUNSUPPORTED


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, from a host C program."""
    import subprocess
    import tempfile
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "tdp.h"', "int main(void) {",
           f'  printf("%zu\\n", sizeof({struct}));']
    src += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(c, "w") as fh:
            fh.write("\n".join(src))
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                        "-D__HIP_PLATFORM_AMD__", c, "-o", exe], check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("name,cls", [("tdp_col", "Col"), ("tdp_pred", "Pred"), ("tdp_join_desc", "JoinDesc"),
                                      ("tdp_groupby_desc", "GroupbyDesc"), ("tdp_groupby_out", "GroupbyOut"),
                                      ("tdp_adam_tensor", "AdamTensor")])
def test_struct_layout_matches_header(name, cls):
    from paper_2211_02753_amd import _lib
    py = getattr(_lib, cls)
    fields = [f[0] for f in py._fields_]
    size, offs = _c_layout(name, fields)
    assert ctypes.sizeof(py) == size
    assert [getattr(py, f).offset for f in fields] == offs


def test_max_distinct_sizes_the_table(lib):
    from paper_2211_02753_amd import _lib
    L = _lib.load()
    jd = _lib.JoinDesc(0x2000, 1_000_000, 0x3000, 10, None, 0, 0, 0, 0)
    full = L.tdp_hash_join_workspace_size(ctypes.byref(jd))
    jd.max_distinct = 1000
    small = L.tdp_hash_join_workspace_size(ctypes.byref(jd))
    assert 0 < small < full
    jd.max_distinct = 10_000_000  # above n_build: taken as n_build
    assert L.tdp_hash_join_workspace_size(ctypes.byref(jd)) == full
    jd.max_distinct = -1
    n_out = ctypes.c_int64()
    assert L.tdp_hash_join(ctypes.byref(jd), _lib.JOIN_COUNT, None, None, 0, ctypes.byref(n_out), None,
                           ctypes.c_void_p(0x4000), 1 << 30, None) == _lib.TDP_EINVAL


def test_soft_binding_rejects_mistyped_tensors():
    """An int64 group column (torch's default integer) or a host tensor is
    refused before any launch instead of being read as int32 device data."""
    import torch
    from paper_2211_02753_amd import soft
    with pytest.raises(TypeError, match="int32"):
        soft.soft_groupby(torch.zeros(4, dtype=torch.int64), None, torch.zeros(4), 3)
    with pytest.raises(TypeError, match="float32"):
        soft.soft_pe_groupby(torch.zeros((4, 2), dtype=torch.float64), None, None, 1)


def test_stage_timer_argument_checks(lib):
    """The measurement hook rejects an unknown stage and null outputs before
    touching the device."""
    from paper_2211_02753_amd import _lib
    L = _lib.load()
    assert L.tdp_stage_timer(-1) == _lib.TDP_EINVAL
    assert L.tdp_stage_timer(_lib.STAGE_FUSED_PROBE + 1) == _lib.TDP_EINVAL
    assert L.tdp_stage_time(None, None) == _lib.TDP_EINVAL
