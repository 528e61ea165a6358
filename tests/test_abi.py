"""CPU checks of the C ABI library: it loads, and it exports every function
declared in include/rdl.h (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "rdl.h")
LIB = os.path.join(ROOT, "paper_2309_11072_amd", "librdl.so")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rdl_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rdl_encode_enh", "rdl_decode_enh", "rdl_encode_batch", "rdl_create", "rdl_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("librdl.so not built: run __graft_entry__.build()")
    import torch  # noqa: F401  (the HIP runtime is loaded through torch first)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_2309_11072_amd import rdl
    assert set(declared_functions()) == set(rdl._SIGS)


def test_header_layout_matches_dtype():
    from paper_2309_11072_amd import rdl
    assert rdl.HEADER_BYTES == 7232
    assert rdl.HEADER_DTYPE.fields["a_q"][1] == 64
    assert rdl.HEADER_DTYPE.fields["present"][1] == 64 + 2 * 3072
