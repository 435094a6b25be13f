"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "parem.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(parem_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["parem_compile", "parem_match", "parem_match_async", "parem_free", "parem_strerror",
              "parem_workspace_size", "parem_describe"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1412_1741_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTED) == sorted(declared_functions())
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(parem_\w+)", out))
    assert set(declared_functions()) <= exported


def test_strerror_texts():
    import paper_1412_1741_amd as P
    assert P.parem_strerror(P.PAREM_OK) == "ok"
    assert "alphabet" in P.parem_strerror(P.PAREM_ESYMBOL)
    assert P.parem_strerror(12345) == "unknown status"


def test_result_struct_layout():
    import paper_1412_1741_amd as P
    assert ctypes.sizeof(P.Result) == 40
    assert P.Result.count.offset == 8 and P.Result.rerun_chunks.offset == 32
