"""The C-ABI library loads on the CPU and exports every entry point include/rbns.h declares.

No compute call is made here (there is no GPU in the build container)."""

import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbns.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*(rb_[a-z_]+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for fn in ("rb_create", "rb_destroy", "rb_last_error", "rb_load_tensors", "rb_theta",
               "rb_solve_batch", "rb_solve_uneven", "rb_recover_pressure", "rb_hbm_used"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    from paper_1807_11866_amd import rbns
    if not os.path.exists(rbns.LIB_PATH):
        pytest.skip("librbns.so not built (run __graft_entry__.build())")
    lib = ct.CDLL(rbns.LIB_PATH)
    for fn in declared_functions():
        assert hasattr(lib, fn), fn
    assert set(rbns.EXPORTED) == set(declared_functions())


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1807_11866_amd import rbns
    saved = rbns._lib
    try:
        rbns._lib = None
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            rbns.load(str(tmp_path / "missing.so"))
    finally:
        rbns._lib = saved


def test_last_error_is_empty_string_initially():
    from paper_1807_11866_amd import rbns
    if not os.path.exists(rbns.LIB_PATH):
        pytest.skip("librbns.so not built")
    lib = rbns.load()
    assert isinstance(lib.rb_last_error(), bytes)
