"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("parem.h", "parem_measure.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(parem_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


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


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the C compiler's sizes and offsets."""
    import paper_1412_1741_amd as P
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "parem.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
    printf("parem_options %zu\n", sizeof(parem_options));
    F(parem_options, chunk_len); F(parem_options, layout); F(parem_options, group); F(parem_options, policy);
    F(parem_options, tile); F(parem_options, no_merge); F(parem_options, lookback); F(parem_options, partial);
    printf("parem_result %zu\n", sizeof(parem_result));
    F(parem_result, final_state); F(parem_result, accept); F(parem_result, count); F(parem_result, chunks);
    F(parem_result, spec_runs); F(parem_result, rerun_chunks);
    printf("parem_batch_info %zu\n", sizeof(parem_batch_info));
    F(parem_batch_info, pairs); F(parem_batch_info, walk_launches); F(parem_batch_info, walk_items);
    F(parem_batch_info, levels); F(parem_batch_info, graph_nodes); F(parem_batch_info, learned_pairs);
    F(parem_batch_info, chunks); F(parem_batch_info, text_bytes); F(parem_batch_info, workspace_bytes);
    return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    for cname, cls in (("parem_options", P.Options), ("parem_result", P.Result), ("parem_batch_info", P.BatchInfo)):
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert int(got[f"{cname}.{field}"]) == getattr(cls, field).offset, (cname, field)
