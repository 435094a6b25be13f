"""Pins of the regular-expression oracle (Section III, Table III's operators).

The oracle (oracle/regex.py: a recursive-descent parser, the Thompson
construction, and a run simulated on sets of states by the C oracle) is
held to Python's re on every string up to a length over small alphabets: for
the paper's example expression (a|b)?c*[0..3]b+, hand-written precedence
cases and random expressions written in both syntaxes; anchored (prefixes in
the language) and search (ends of matches) counts alike. No GPU here.
"""
import itertools
import re

import numpy as np
import pytest

from oracle import regex as R
from regex_cases import FIXED, brute, random_expression


@pytest.mark.parametrize("ours,py,alpha", FIXED)
def test_oracle_matches_python_re(ours, py, alpha):
    syms = [bytes([c]) for c in alpha]
    maxlen = 5 if len(alpha) <= 4 else 4
    for mode in ("anchored", "search"):
        for n in range(0, maxlen + 1):
            for tup in itertools.product(syms, repeat=n):
                s = b"".join(tup)
                r = R.run(ours, alpha, s, mode)
                assert (r.accept, r.count) == brute(py, s, mode), (ours, mode, s)


def test_oracle_random_expressions():
    rng = np.random.default_rng(2015)
    alpha = b"xyz"
    syms = [bytes([c]) for c in alpha]
    strings = [b"".join(t) for n in range(5) for t in itertools.product(syms, repeat=n)]
    for _ in range(60):
        ours, py = random_expression(rng, alpha, 3)
        for mode in ("anchored", "search"):
            for s in strings:
                r = R.run(ours, alpha, s, mode)
                assert (r.accept, r.count) == brute(py, s, mode), (ours, py, mode, s)


def test_oracle_empty_set_means_no_match_can_follow():
    """The set of states empties exactly when no continuation of the text is
    in the language (checked against re on every continuation up to 3)."""
    alpha = b"abc0123"
    py = re.compile(b"(a|b)?c*[0-3]b+")
    syms = [bytes([c]) for c in alpha]
    conts = [b"".join(t) for n in range(4) for t in itertools.product(syms, repeat=n)]
    for n in range(4):
        for tup in itertools.product(syms, repeat=n):
            s = b"".join(tup)
            r = R.run(b"(a|b)?c*[0..3]b+", alpha, s)
            alive = any(py.fullmatch(s + c) for c in conts)
            if r.empty:
                assert not alive, s
            elif len(s) <= 2:
                assert alive, s


@pytest.mark.parametrize("bad", [b"(", b"a)", b"[]", b"[b..a]", b"*a", b"a|*", b"[a", b"\\", b"(a|b", b"a]"])
def test_oracle_syntax_errors(bad):
    with pytest.raises(R.RegexSyntaxError):
        R.parse(bad)
