"""The C-ABI library loads without a GPU and exports every function that
include/abddc.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "abddc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(abddc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("abddc_assemble", "abddc_setup_coarse_space", "abddc_apply_bddc", "abddc_gmres_solve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2501_01676_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libabddc_hip.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.SIGNATURES) == set(_declared())


def test_error_path_without_context():
    from paper_2501_01676_amd import _lib
    lib = _lib.load()
    rc = lib.abddc_apply_bddc(None, None, None)
    assert rc == _lib.EINVAL
    assert b"null" in lib.abddc_last_error()
