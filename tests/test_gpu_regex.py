"""Regular expressions matched on the GPU: parem_compile_regex (the
Section III front-end) then the speculative walk, against the oracle's run
of the expression's automaton on sets of states (oracle/regex.py, pinned to
Python's re). Total and partial forms, anchored and search modes; the
partial form dies (PAREM_DEAD_STATE) exactly when the oracle's set of states
empties."""
import sys

import numpy as np
import pytest

from oracle import regex as R
import workloads as W
from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_1412_1741_amd as P


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    (b"parallel", b"parel"),
    (b"(a|b)?c*[0..3]b+", b"abc0123"),
    (b"A[C..G]?(T|GA)+C", b"ACGT"),
    (b"(AC|GT)*A+G?", b"ACGT"),
    (b"[0..9]+(\\.[0..9]+)?", b"0123456789.x"),
]


def texts(rng, alphabet, n):
    yield W.uniform_text(rng, alphabet, n)
    # skewed: long runs of one symbol keep anchored runs alive longer
    t = W.uniform_text(rng, alphabet[:2], n)
    t[rng.integers(0, n, size=8)] = alphabet[-1]
    yield t


@pytest.mark.parametrize("pattern,alphabet", CASES)
def test_regex_on_gpu_matches_oracle(pattern, alphabet):
    rng = np.random.default_rng(len(pattern))
    for mode, name in ((P.RE_SEARCH, "search"), (P.RE_ANCHORED, "anchored")):
        for partial in (False, True):
            m = P.Matcher.from_regex(pattern, alphabet, mode, partial=partial, chunk_len=1024)
            for i, text in enumerate(texts(rng, alphabet, 300_007)):
                want = R.run(pattern, alphabet, text, name)
                got = m.match(torch.from_numpy(text).cuda())
                say(f"[case] regex {pattern!r} {name} partial={partial} text {i}: count {want.count}")
                assert (got.accept, got.count) == (want.accept, want.count)
                if partial:
                    assert (got.final_state == P.DEAD_STATE) == want.empty
            m.close()


def test_regex_search_positions_and_layouts():
    """Search for a DNA expression over 8 MiB: the count equals the oracle's
    on every table layout, and the match positions' count equals it too."""
    rng = np.random.default_rng(3)
    alphabet = b"ACGT"
    pattern = b"GA(T|C)+[A..C]AG"
    text = W.uniform_text(rng, alphabet, 8 << 20)
    want = R.run(pattern, alphabet, text, "search")
    d = torch.from_numpy(text).cuda()
    for lay in (P.LAYOUT_AUTO, P.LAYOUT_BYTE_LDS, P.LAYOUT_CLASS_LDS, P.LAYOUT_BYTE_GLOBAL, P.LAYOUT_SPARSE_LDS):
        m = P.Matcher.from_regex(pattern, alphabet, P.RE_SEARCH, layout=lay)
        got = m.match(d)
        assert (got.accept, got.count) == (want.accept, want.count), lay
        pos, res = m.positions(d)
        assert res.count == want.count and pos.numel() == want.count
        m.close()


def test_regex_errors():
    with pytest.raises(P.ParemError) as ei:
        P.Matcher.from_regex(b"(ab", b"ab")
    assert ei.value.status == P.PAREM_ESYNTAX
