"""The C-ABI library loads on the host and exports every declared symbol.

No compute call is made: these run without a GPU.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mipdhg_\w+)\s*\(", text))
    return names


def test_header_declares_entry_points():
    names = _declared()
    for n in ("mipdhg_solve", "mipdhg_workspace_size", "mipdhg_default_options",
              "mipdhg_status_string", "mipdhg_last_error", "mipdhg_sizeof"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2603_03150_amd import _lib
    lib = _lib.load()
    for name in sorted(_declared()):
        assert hasattr(lib, name), name
    missing = sorted(_declared() - set(_lib.SIGNATURES))
    assert not missing, f"binding lacks signatures for {missing}"


def test_struct_layouts_and_defaults():
    import paper_2603_03150_amd as P
    from paper_2603_03150_amd import _lib
    lib = _lib.load()
    assert lib.mipdhg_sizeof(0) == C.sizeof(_lib.LPStruct)
    assert lib.mipdhg_sizeof(1) == C.sizeof(_lib.OptionsStruct)
    assert lib.mipdhg_sizeof(2) == C.sizeof(_lib.InfoStruct)
    assert lib.mipdhg_sizeof(4) == C.sizeof(_lib.IpmOptionsStruct)
    assert lib.mipdhg_sizeof(5) == C.sizeof(_lib.IpmInfoStruct)
    d = P.default_options()
    assert d["ruiz_iters"] == 10 and d["eval_every"] == 64 and abs(d["beta_art"] - 0.36) < 1e-15
    assert lib.mipdhg_status_string(0) == b"OPTIMAL"
    assert lib.mipdhg_status_string(-3) == b"ERR_TRANSPOSE"


def test_host_side_argument_errors():
    from paper_2603_03150_amd import _lib
    lib = _lib.load()
    o = _lib.OptionsStruct()
    lib.mipdhg_default_options(C.byref(o))
    nb = C.c_size_t(0)
    s = _lib.LPStruct()
    s.m, s.n, s.nnz = 0, 5, 0
    assert lib.mipdhg_workspace_size(C.byref(s), C.byref(o), C.byref(nb)) == -1
    assert b"m >= 1" in lib.mipdhg_last_error()
    s.m, s.n, s.nnz = 3, 5, 4
    s.a_rowptr = s.at_rowptr = s.a_col = s.a_val = s.at_col = s.at_val = s.b = s.c = 8  # never dereferenced
    assert lib.mipdhg_workspace_size(C.byref(s), C.byref(o), C.byref(nb)) == 0
    assert nb.value > 0 and nb.value % 256 == 0
    o.eval_every = 0
    assert lib.mipdhg_workspace_size(C.byref(s), C.byref(o), C.byref(nb)) == -1
    lib.mipdhg_default_options(C.byref(o))
    o.lanes_a = 3
    assert lib.mipdhg_workspace_size(C.byref(s), C.byref(o), C.byref(nb)) == -1
    # solve rejects a NULL workspace before touching any device memory
    assert lib.mipdhg_solve(C.byref(s), C.byref(o), 1e-4, None, 0, None, None, None, None, None, None,
                            None, None, None) == -1


def test_batched_option_errors_on_the_host():
    # a two-instance batch described on the host (device pointers never
    # dereferenced by the workspace query); the batched options are checked
    from paper_2603_03150_amd import _lib
    lib = _lib.load()
    o = _lib.OptionsStruct()
    lib.mipdhg_default_options(C.byref(o))
    assert o.batch_split == 0 and o.batch_block_iters == 0
    row_off = (C.c_int32 * 3)(0, 2, 5)
    col_off = (C.c_int32 * 3)(0, 4, 9)
    nnz_off = (C.c_int64 * 3)(0, 6, 14)
    bt = _lib.BatchStruct()
    bt.count = 2
    bt.row_off, bt.col_off, bt.nnz_off = (C.cast(v, C.c_void_p) for v in (row_off, col_off, nnz_off))
    w = bt.whole
    w.m, w.n, w.nnz = 5, 9, 14
    w.a_rowptr = w.at_rowptr = w.a_col = w.a_val = w.at_col = w.at_val = w.b = w.c = 8
    nb = C.c_size_t(0)
    assert lib.mipdhg_batch_workspace_size(C.byref(bt), C.byref(o), C.byref(nb)) == 0 and nb.value > 0
    for field, bad in (("batch_block_iters", -1), ("batch_split", -1), ("batch_split", 150 * 1024 + 1)):
        lib.mipdhg_default_options(C.byref(o))
        setattr(o, field, bad)
        assert lib.mipdhg_batch_workspace_size(C.byref(bt), C.byref(o), C.byref(nb)) == -1, field
        assert field.encode() in lib.mipdhg_last_error()
    lib.mipdhg_default_options(C.byref(o))
    o.batch_block_iters, o.batch_split = 128, 4096
    assert lib.mipdhg_batch_workspace_size(C.byref(bt), C.byref(o), C.byref(nb)) == 0
    # the instance offsets must end at the whole matrix's sizes
    nnz_off[2] = 13
    assert lib.mipdhg_batch_workspace_size(C.byref(bt), C.byref(o), C.byref(nb)) == -1
    assert lib.mipdhg_status_string(6) == b"IN_PROGRESS"
