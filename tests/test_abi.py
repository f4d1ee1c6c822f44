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


def test_binding_structs_match_the_header(tmp_path):
    """Every public struct of the header has the binding's size and field
    offsets (a C program built with gcc prints them; a field the binding
    names with a trailing underscore, a Python keyword, has it without in C)."""
    import subprocess
    from paper_1705_02408_amd import mpap
    structs = [getattr(mpap, n) for n in ("mpap_env", "mpap_graph_params", "mpap_search_params",
                                          "mpap_stats", "mpap_mc_params", "mpap_mc_stats")]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpap.h"', 'int main(void) {']
    for st in structs:
        name = st.__name__
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in st._fields_:
            cname = fname.rstrip("_")  # a Python keyword gets a trailing underscore
            lines.append(f'    printf("{name} {fname} %zu\\n", offsetof({name}, {cname}));')
    lines += ['    return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for st in structs:
        name = st.__name__
        assert got[(name, "size")] == ctypes.sizeof(st), name
        for fname, _ in st._fields_:
            assert got[(name, fname)] == getattr(st, fname).offset, (name, fname)
