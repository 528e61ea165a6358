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


def _lib():
    if not os.path.exists(LIB):
        pytest.fail("librdl.so not built: run __graft_entry__.build()")
    from paper_2309_11072_amd import rdl
    return rdl, rdl.load_library()


def test_size_limits_host_only():
    rdl, L = _lib()
    assert L.rdl_resid_bytes(3, 5) == 105
    assert L.rdl_resid_bytes(0, 5) == 0 and L.rdl_resid_bytes(5, 0) == 0
    assert L.rdl_resid_bytes(1, 1 << 28) == 7 << 28
    assert L.rdl_resid_bytes(1, (1 << 28) + 1) == 0      # width limit (32-bit row offsets)
    assert L.rdl_resid_bytes(1 << 16, 1 << 15) == 0      # H*W = 2^31
    assert L.rdl_header_bytes() == rdl.HEADER_BYTES


def test_header_validate_bounds_host_only():
    """rdl_header_validate accepts exactly the coefficient ranges a
    least-squares line through 8-bit data can take: |a_q| <= 255 2^22 and
    -65025 2^14 <= b_q <= 65280 2^14."""
    import ctypes
    import numpy as np
    rdl, L = _lib()
    h = np.zeros(1, rdl.HEADER_DTYPE)
    h["magic"], h["version"], h["H"], h["W"], h["q"] = rdl.RDL_MAGIC, 1, 7, 9, 75
    h["present"][0, 17] = 1

    def check(aq, bq):
        g = h.copy()
        g["a_q"][0, 1, 17] = aq
        g["b_q"][0, 1, 17] = bq
        return L.rdl_header_validate(g.ctypes.data_as(ctypes.c_void_p), 7, 9)

    ok, bad = rdl.RDL_OK, rdl.RDL_ECORRUPT
    assert check(0, 0) == ok
    assert check(255 << 22, 65280 << 14) == ok and check(-(255 << 22), -65025 << 14) == ok
    assert check((255 << 22) + 1, 0) == bad and check(-(255 << 22) - 1, 0) == bad
    assert check(0, (65280 << 14) + 1) == bad and check(0, (-65025 << 14) - 1) == bad
    assert L.rdl_header_validate(h.ctypes.data_as(ctypes.c_void_p), 7, 10) == bad


def test_launch_mode_rejects_null_context_host_only():
    rdl, L = _lib()
    assert L.rdl_set_launch_mode(None, 0) == rdl.RDL_EINVAL
    assert L.rdl_set_launch_mode(None, 1) == rdl.RDL_EINVAL
    assert (rdl.LAUNCH_DIRECT, rdl.LAUNCH_GRAPH) == (0, 1)


def test_entropy_bound_and_argument_checks_host_only(O):
    """The library's stream bound equals the oracle's; bad sizes, group sizes
    and null pointers are rejected before any device work."""
    rdl, L = _lib()
    src = open(HDR).read()
    assert int(re.search(r"#define RDL_ENT_HEADER_BYTES (\d+)", src).group(1)) == rdl.ENT_HEADER_BYTES == O.ENT_HDR
    for H, W, k in [(1, 1, 4), (7, 9, 8), (2160, 3840, 8), (4321, 7679, 12), (1, 1 << 20, 4)]:
        assert L.rdl_ent_bound(H, W, k) == O.ent_bound(H, W, k)
    for H, W, k in [(0, 5, 8), (5, 0, 8), (3, 3, 3), (3, 3, 13), (1 << 16, 1 << 15, 8)]:
        assert L.rdl_ent_bound(H, W, k) == 0
    assert L.rdl_ent_encode(None, None, 3, 3, 8, None, 0, None, None) == rdl.RDL_EINVAL
    assert L.rdl_ent_decode(None, None, 0, None, 3, 3, None, None, None) == rdl.RDL_EINVAL
    assert L.rdl_set_ent_predict(None, 1) == rdl.RDL_EINVAL


def test_entropy_context_bound_and_argument_checks_host_only(O):
    """The context stream's header size and bound equal the oracle's; a
    missing base layer and null pointers are rejected before device work."""
    rdl, L = _lib()
    src = open(HDR).read()
    assert (int(re.search(r"#define RDL_ENT_CTX_HEADER_BYTES (\d+)", src).group(1)) == rdl.ENT_CTX_HEADER_BYTES
            == O.ENT_HDR_CTX == 40 + 1024 * 25)
    for H, W, k in [(1, 1, 4), (7, 9, 8), (2160, 3840, 8), (4321, 7679, 12)]:
        assert L.rdl_ent_bound_ctx(H, W, k) == O.ent_bound(H, W, k, contexts=True)
        assert L.rdl_ent_bound_ctx(H, W, k) == L.rdl_ent_bound(H, W, k) + O.ENT_HDR_CTX - O.ENT_HDR
    assert L.rdl_ent_bound_ctx(0, 5, 8) == 0 and L.rdl_ent_bound_ctx(3, 3, 13) == 0
    assert L.rdl_ent_encode_ctx(None, None, None, 3, 3, 8, None, 0, None, None) == rdl.RDL_EINVAL
    assert L.rdl_ent_decode_ctx(None, None, 0, None, None, 3, 3, None, None, None) == rdl.RDL_EINVAL


def test_jpeg_bound_host_only():
    rdl, L = _lib()
    assert L.rdl_jpeg_bound(0, 5) == 0 and L.rdl_jpeg_bound(70000, 5) == 0 and L.rdl_jpeg_bound(5, 65536) == 0
    # 1024 header bytes, then per scan a 10-byte SOS and twice the most bytes of its blocks, then EOI
    assert L.rdl_jpeg_bound(8, 8) == 1024 + 3 * (10 + 2 * 256) + 2
    assert L.rdl_jpeg_encode(None, None, 8, 8, 75, None, 0, None, None) == rdl.RDL_EINVAL
    assert L.rdl_set_gf(None, 1) == rdl.RDL_EINVAL and L.rdl_decode_batch(None, None, 0, None) == rdl.RDL_EINVAL
