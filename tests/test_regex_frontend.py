"""The library's regular-expression front-end (Section III, Table III's
operators): parem_regex_dfa (parse, Thompson construction, removal of empty
moves, subset construction; host code) is held to Python's re on every
string up to a length, to the oracle's run of the expression's automaton
(pinned in test_oracle_regex.py) on long texts, and its search automaton
for "parallel" is Table I. No GPU here.
"""
import itertools
import os
import re

import numpy as np
import pytest

from oracle import regex as R
from regex_cases import FIXED, brute, dfa_run, random_expression
import paper_1412_1741_amd as P
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("ours,py,alpha", FIXED)
def test_library_front_end_matches_python_re(ours, py, alpha):
    syms = [bytes([c]) for c in alpha]
    maxlen = 5 if len(alpha) <= 4 else 4
    for mode, m in (("anchored", P.RE_ANCHORED), ("search", P.RE_SEARCH)):
        table, fin = P.parem_regex_dfa(ours, alpha, m)
        ptab, pfin = P.parem_regex_dfa(ours, alpha, m, partial=True)
        for n in range(0, maxlen + 1):
            for tup in itertools.product(syms, repeat=n):
                s = b"".join(tup)
                want = brute(py, s, mode)
                acc, cnt, _ = dfa_run(table, fin, s, alpha)
                assert (acc, cnt) == want, (ours, mode, s)
                acc, cnt, died = dfa_run(ptab, pfin, s, alpha)
                assert (acc, cnt) == want, (ours, mode, s, "partial")
                if died:
                    # no continuation of s matches: the oracle's set is empty
                    assert R.run(ours, alpha, s, mode).empty


def test_search_automaton_of_parallel_is_table1(golden_dir):
    rows = [[int(v) for v in line.split()] for line in open(os.path.join(golden_dir, "table1_parallel.txt"))
            if line.strip() and not line.startswith("#")]
    table, fin = P.parem_regex_dfa(b"parallel", b"parel", P.RE_SEARCH)
    assert np.array_equal(table, np.asarray(rows, dtype=np.uint32))
    assert fin.tolist() == [0] * 8 + [1]


def test_random_expressions_oracle_and_library():
    rng = np.random.default_rng(2014)
    alpha = b"xyz"
    syms = [bytes([c]) for c in alpha]
    strings = [b"".join(t) for n in range(5) for t in itertools.product(syms, repeat=n)]
    for i in range(60):
        ours, py = random_expression(rng, alpha, 3)
        for mode, m in (("anchored", P.RE_ANCHORED), ("search", P.RE_SEARCH)):
            table, fin = P.parem_regex_dfa(ours, alpha, m)
            for s in strings:
                want = brute(py, s, mode)
                r = R.run(ours, alpha, s, mode)
                assert (r.accept, r.count) == want, (ours, py, mode, s)
                assert dfa_run(table, fin, s, alpha)[:2] == want, (ours, py, mode, s)


def test_library_front_end_matches_oracle_on_long_texts():
    rng = np.random.default_rng(7)
    alpha = b"ACGT"
    for ours in (b"A(C|G)*T", b"(AC|GT)+[A..C]?", b"T?(A|C)+G*T", b"[A..G]+T+A"):
        text = W.uniform_text(rng, alpha, 20000)
        for mode, m in (("anchored", P.RE_ANCHORED), ("search", P.RE_SEARCH)):
            table, fin = P.parem_regex_dfa(ours, alpha, m)
            r = R.run(ours, alpha, text, mode)
            acc, cnt, _ = dfa_run(table, fin, text.tobytes(), alpha)
            assert (acc, cnt) == (r.accept, r.count), (ours, mode)


@pytest.mark.parametrize("bad", [b"(", b"a)", b"[]", b"[b..a]", b"*a", b"a|*", b"[a", b"\\", b"(a|b", b"a]"])
def test_syntax_errors(bad):
    with pytest.raises(P.ParemError) as ei:
        P.parem_regex_dfa(bad, b"ab*()[]|\\")
    assert ei.value.status == P.PAREM_ESYNTAX
