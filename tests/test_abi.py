"""The C ABI library loads without a GPU and exports every declared symbol;
the binding refuses to run when the library or the device is missing."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpap.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpap_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1705_02408_amd import mpap
    if not os.path.exists(mpap.LIB_PATH):
        from paper_1705_02408_amd import build
        build.build()
    return ctypes.CDLL(mpap.LIB_PATH)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("mpap_build_graph", "mpap_search", "mpap_goal_front", "mpap_graph_from_csr"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1705_02408_amd import mpap
    assert sorted(mpap.SYMBOLS) == declared_symbols()


def test_status_strings(lib):
    lib.mpap_status_string.restype = ctypes.c_char_p
    assert lib.mpap_status_string(0) == b"ok"
    assert b"capacity" in lib.mpap_status_string(5)


def test_missing_library_fails_loudly(tmp_path):
    from paper_1705_02408_amd import mpap
    saved = mpap._lib
    try:
        mpap._lib = None
        with pytest.raises(RuntimeError):
            mpap.load(str(tmp_path / "nope.so"))
    finally:
        mpap._lib = saved
