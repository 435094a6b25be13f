"""CPU oracle of the regular-expression front-end (TEST INFRASTRUCTURE ONLY).

Section III of the paper accepts regular expressions built from the
operators of Table III: concatenation, Kleene star, union, positive closure,
range ([0..9]), optionality and groups. It parses them into an abstract
syntax tree and builds an automaton with the McNaughton-Yamada-Thompson
construction. This module does the same for testing, independently of the
library's C++ front-end: a recursive-descent parser, the Thompson
construction, and a run of the resulting automaton simulated on sets of
states by the C oracle (``oracle_nfa_walk``); nothing here is determinised.

Grammar (bytes):
    union   := concat ('|' concat)*
    concat  := repeat*                      (empty: the empty word)
    repeat  := atom ('*' | '+' | '?')*
    atom    := '(' union ')' | '[' item+ ']' | '\\' byte | byte
    item    := c | c '..' c | c '-' c       (c: a byte, or '\\' byte)
Bytes ( ) [ ] | * + ? \\ are operators outside brackets; every other byte is
itself. A range x..y holds the bytes from x to y in code order.

Modes: ``anchored`` counts the prefixes of the text in the language;
``search`` counts the positions where some match ends (the language of
Sigma* followed by the expression, Sigma the text alphabet).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import OracleError, _load, _ptr, _text

SPECIAL = set(b"()[]|*+?\\")


class RegexSyntaxError(ValueError):
    pass


# --- abstract syntax tree: tuples (kind, ...) -------------------------------
#   ("set", frozenset of bytes) | ("empty",) | ("cat", a, b) | ("alt", a, b)
#   ("star", a) | ("plus", a) | ("opt", a)

def parse(pattern: bytes):
    p = bytes(pattern)
    pos = 0

    def peek():
        return p[pos] if pos < len(p) else None

    def take():
        nonlocal pos
        if pos >= len(p):
            raise RegexSyntaxError("unexpected end of pattern")
        c = p[pos]
        pos += 1
        return c

    def union():
        node = concat()
        while peek() == ord("|"):
            take()
            node = ("alt", node, concat())
        return node

    def concat():
        node = None
        while peek() is not None and peek() not in (ord("|"), ord(")")):
            r = repeat()
            node = r if node is None else ("cat", node, r)
        return ("empty",) if node is None else node

    def repeat():
        node = atom()
        while peek() is not None and peek() in (ord("*"), ord("+"), ord("?")):
            op = take()
            node = {ord("*"): "star", ord("+"): "plus", ord("?"): "opt"}[op], node
            node = tuple(node)
        return node

    def bracket_byte():
        c = take()
        if c == ord("\\"):
            return take()
        if c == ord("]"):
            raise RegexSyntaxError("empty item in a range")
        return c

    def atom():
        c = take()
        if c == ord("("):
            node = union()
            if take() != ord(")"):
                raise RegexSyntaxError("unbalanced group")
            return node
        if c == ord("["):
            members = set()
            if peek() == ord("]"):
                raise RegexSyntaxError("empty range")
            while peek() != ord("]"):
                if peek() is None:
                    raise RegexSyntaxError("unterminated range")
                lo = bracket_byte()
                hi = lo
                if p[pos:pos + 2] == b".." and pos + 2 < len(p) and p[pos + 2] != ord("]"):
                    take()
                    take()
                    hi = bracket_byte()
                elif peek() == ord("-") and pos + 1 < len(p) and p[pos + 1] != ord("]"):
                    take()
                    hi = bracket_byte()
                if hi < lo:
                    raise RegexSyntaxError("reversed range")
                members.update(range(lo, hi + 1))
            take()
            return ("set", frozenset(members))
        if c == ord("\\"):
            return ("set", frozenset([take()]))
        if c in SPECIAL:
            raise RegexSyntaxError(f"unexpected {chr(c)!r}")
        return ("set", frozenset([c]))

    node = union()
    if pos != len(p):
        raise RegexSyntaxError("unbalanced ')'")
    return node


# --- McNaughton-Yamada-Thompson construction ---------------------------------

@dataclass
class Nfa:
    n: int = 0
    edges: list = field(default_factory=list)   # (from, lo, hi, to)
    eps: list = field(default_factory=list)     # (from, to)
    start: int = 0
    accept: int = 0

    def new(self) -> int:
        self.n += 1
        return self.n - 1


def _ranges(members):
    """Sorted byte set -> list of (lo, hi) runs."""
    out = []
    for b in sorted(members):
        if out and out[-1][1] == b - 1:
            out[-1][1] = b
        else:
            out.append([b, b])
    return [(lo, hi) for lo, hi in out]


def thompson(node, nfa: Nfa):
    """Fragment (start, accept) for `node`: each operator adds its states and
    empty moves around its operands' fragments."""
    kind = node[0]
    if kind == "set":
        s, f = nfa.new(), nfa.new()
        for lo, hi in _ranges(node[1]):
            nfa.edges.append((s, lo, hi, f))
        return s, f
    if kind == "empty":
        s, f = nfa.new(), nfa.new()
        nfa.eps.append((s, f))
        return s, f
    if kind == "cat":
        a = thompson(node[1], nfa)
        b = thompson(node[2], nfa)
        nfa.eps.append((a[1], b[0]))
        return a[0], b[1]
    if kind == "alt":
        a = thompson(node[1], nfa)
        b = thompson(node[2], nfa)
        s, f = nfa.new(), nfa.new()
        nfa.eps += [(s, a[0]), (s, b[0]), (a[1], f), (b[1], f)]
        return s, f
    a = thompson(node[1], nfa)
    s, f = nfa.new(), nfa.new()
    if kind == "star":
        nfa.eps += [(s, a[0]), (s, f), (a[1], a[0]), (a[1], f)]
    elif kind == "plus":
        nfa.eps += [(s, a[0]), (a[1], a[0]), (a[1], f)]
    elif kind == "opt":
        nfa.eps += [(s, a[0]), (s, f), (a[1], f)]
    else:
        raise ValueError(kind)
    return s, f


def build(pattern: bytes, alphabet: bytes, mode: str = "anchored") -> Nfa:
    """The automaton of `pattern`; in search mode a start state that loops on
    every byte of `alphabet` precedes it."""
    nfa = Nfa()
    s, f = thompson(parse(pattern), nfa)
    nfa.start, nfa.accept = s, f
    if mode == "search":
        loop = nfa.new()
        for b in alphabet:
            nfa.edges.append((loop, b, b, loop))
        nfa.eps.append((loop, s))
        nfa.start = loop
    elif mode != "anchored":
        raise ValueError(mode)
    return nfa


@dataclass
class NfaResult:
    accept: bool
    count: int
    empty: bool   # the set of states became empty (nothing can match any more)


def run(pattern: bytes, alphabet: bytes, text, mode: str = "anchored") -> NfaResult:
    """Simulate the automaton of `pattern` over `text` (C oracle)."""
    lib = _load()
    nfa = build(pattern, alphabet, mode)
    acc = np.zeros(nfa.n, dtype=np.uint8)
    acc[nfa.accept] = 1
    edges = np.asarray(nfa.edges, dtype=np.uint32).reshape(-1, 4) if nfa.edges else np.zeros((0, 4), np.uint32)
    eps = np.asarray(nfa.eps, dtype=np.uint32).reshape(-1, 2) if nfa.eps else np.zeros((0, 2), np.uint32)
    edges = np.ascontiguousarray(edges)
    eps = np.ascontiguousarray(eps)
    alpha = np.frombuffer(bytes(alphabet), dtype=np.uint8).copy()
    x = _text(text)
    a = ctypes.c_uint8(0)
    e = ctypes.c_uint8(0)
    cnt = ctypes.c_uint64(0)
    bad = ctypes.c_uint64(0)
    rc = lib.oracle_nfa_walk(nfa.n, nfa.start, _ptr(acc, ctypes.c_uint8), _ptr(edges, ctypes.c_uint32),
                             edges.shape[0], _ptr(eps, ctypes.c_uint32), eps.shape[0],
                             _ptr(alpha, ctypes.c_uint8), alpha.size, _ptr(x, ctypes.c_uint8), x.size,
                             ctypes.byref(a), ctypes.byref(cnt), ctypes.byref(e), ctypes.byref(bad))
    if rc:
        err = OracleError(rc, "oracle_nfa_walk")
        err.bad_pos = int(bad.value)
        raise err
    return NfaResult(bool(a.value), int(cnt.value), bool(e.value))
