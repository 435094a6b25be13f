"""Driver for test_sanitizers.py: runs the library's host code (DFA validation,
completion of partial tables, speculated sets, every table layout, the
regular-expression front-end) through a build whose host objects carry
AddressSanitizer and UndefinedBehaviorSanitizer. Started in a child process
with the sanitizer runtime preloaded; argv[1] is that library. Without a GPU
a valid compile ends in PAREM_EDEVICE after all host work; with one it
returns a handle."""
import itertools
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import paper_1412_1741_amd as P  # noqa: E402
import workloads as W  # noqa: E402
from regex_cases import FIXED, random_expression  # noqa: E402

P.LIB_PATH = sys.argv[1]
VALID = (P.PAREM_OK, P.PAREM_EDEVICE)


def compile_status(table, alphabet, start, accepting, **opts):
    try:
        h = P.parem_compile(table, alphabet, start, accepting, **opts)
    except P.ParemError as e:
        return e.status
    P.parem_free(h)
    return P.PAREM_OK


def expect(status, allowed, what):
    if status not in allowed:
        raise SystemExit(f"{what}: status {status}, expected one of {allowed}")


rng = np.random.default_rng(12)
cases = [
    ("table I", W.TABLE1.astype(np.uint32), W.PAREL, 0, [5]),
    ("dna motif", W.dna_motif_dfa().table, b"ACGT", 0, W.dna_motif_dfa().accepting),
    ("sparse 4096", W.sparse4096_dfa().table, bytes(range(256)), 0, W.sparse4096_dfa().accepting),
]
for q, a in ((3, 1), (40, 4), (300, 20), (1200, 4), (2500, 4), (70, 256)):
    d = W.random_dense_dfa(rng, q, bytes(rng.choice(256, size=a, replace=False).astype(np.uint8)), 3)
    cases.append((f"dense {q}x{a}", d.table, d.alphabet, d.start, d.accepting))
for spec in W.batch_specs()[:40:3]:
    d, _ = W.batch_pair(spec, with_text=False)
    cases.append((f"batch pair {spec.index}", d.table, d.alphabet, d.start, d.accepting))

options = [{}, {"layout": P.LAYOUT_BYTE_GLOBAL}, {"layout": P.LAYOUT_HOT_LDS}, {"layout": P.LAYOUT_CLASS_LDS},
           {"layout": P.LAYOUT_SPARSE_LDS}, {"layout": P.LAYOUT_BYTE_LDS}, {"lookback": 16},
           {"policy": P.POLICY_ENUMERATE}, {"group": 2, "tile": 64, "chunk_len": 4096}, {"no_merge": True}]
for name, table, alpha, start, acc in cases:
    for opt in options:
        expect(compile_status(table, alpha, start, acc, **opt), VALID + (P.PAREM_EUNSUPPORTED,), f"{name} {opt}")
    for dt in (np.uint8, np.uint16):
        if table.shape[0] <= np.iinfo(dt).max:
            expect(compile_status(table.astype(dt), alpha, start, acc), VALID, f"{name} {dt.__name__}")
    # a partial copy: a quarter of the entries undefined
    part = table.astype(np.int64)
    part[rng.random(part.shape) < 0.25] = -1
    expect(compile_status(part, alpha, start, acc, partial=True), VALID, f"{name} partial")
    # errors the host must catch
    bad = table.astype(np.uint32).copy()
    bad[0, 0] = table.shape[0]
    expect(compile_status(bad, alpha, start, acc), (P.PAREM_ESTATE,), f"{name} target out of range")
    expect(compile_status(table, alpha, table.shape[0], acc), (P.PAREM_ESTATE, P.PAREM_EINVAL), f"{name} start")
    expect(compile_status(table, alpha[:-1] + alpha[:1] if len(alpha) > 1 else b"", start, acc),
           (P.PAREM_EINVAL,), f"{name} alphabet")

# regular-expression front-end
for ours, _py, alpha in FIXED:
    for mode in (P.RE_ANCHORED, P.RE_SEARCH):
        for partial in (False, True):
            t, f = P.parem_regex_dfa(ours, alpha, mode, partial=partial)
            assert t.shape[0] == f.shape[0] >= 1
for i in range(80):
    ours, _py = random_expression(rng, b"xyz", 4)
    P.parem_regex_dfa(ours, b"xyz", P.RE_SEARCH)
for bad in (b"(", b"a)", b"[]", b"[b..a]", b"*a", b"a|*", b"[a", b"\\", b"(a|b", b"a]"):
    try:
        P.parem_regex_dfa(bad, b"ab*()[]|\\")
        raise SystemExit(f"{bad!r} parsed")
    except P.ParemError as e:
        assert e.status == P.PAREM_ESYNTAX
print("host paths done", len(cases), "tables")
