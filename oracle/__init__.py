"""CPU oracle for the speculative chunked DFA walk.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library under
``paper_1412_1741_amd`` never does, and this package imports nothing from it.

The C part (``parem_oracle.c``) is a plain single-threaded DFA run (also on
partial tables, and listing match positions) plus a step-by-step execution
of the paper's Algorithm 1 (and of the Enumeration policy); this module loads it with
ctypes (building it with gcc when no build exists yet) and converts numpy
arrays to its plain-pointer interface.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "parem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ESYMBOL, ESTATE, EJOIN = 0, -1, -4, -5, -6
PARTIAL = 1
UNDEF = 0xFFFFFFFF        # table entry of an undefined transition (u32)
DEAD = 0xFFFFFFFE         # final state of a run that met an undefined transition
POLICY_PAREM, POLICY_ENUMERATE = 0, 1


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: oracle status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no tuning)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.oracle_walk.restype = ctypes.c_int
        u32 = ctypes.c_uint32
        lib.oracle_walk.argtypes = [u32p, u32, u8p, u32, u32, u32, u8p, u8p, ctypes.c_uint64, u32p, u64p, u64p]
        lib.oracle_states_at.restype = ctypes.c_int
        lib.oracle_states_at.argtypes = [u32p, u32, u8p, u32, u32, u32, u8p, u8p, ctypes.c_uint64, u64p,
                                         ctypes.c_uint64, u32p, u64p]
        lib.oracle_parem.restype = ctypes.c_int
        lib.oracle_parem.argtypes = [u32p, u32, u8p, u32, u32, u32, u32, u8p, u8p, ctypes.c_uint64,
                                     ctypes.c_uint64, u32p, u64p, u64p, u32p, u32p, u32p, ctypes.c_uint64, u64p]
        lib.oracle_nfa_walk.restype = ctypes.c_int
        lib.oracle_nfa_walk.argtypes = [u32, u32, u8p, u32p, u32, u32p, u32, u8p, u32, u8p, ctypes.c_uint64, u8p,
                                        u64p, u8p, u64p]
        lib.oracle_positions.restype = ctypes.c_int
        lib.oracle_positions.argtypes = [u32p, u32, u8p, u32, u32, u32, u8p, u8p, ctypes.c_uint64, u64p,
                                         ctypes.c_uint64, u64p, u64p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _prep(table, alphabet, accepting, partial=False):
    """u32 table, alphabet bytes, final flags. With ``partial`` an entry equal
    to the all-ones value of an unsigned table's type (or a negative entry of
    a signed one) is an undefined transition (UNDEF)."""
    src = np.asarray(table)
    if src.ndim != 2:
        raise ValueError("table must be 2-D [Q, A]")
    t = np.ascontiguousarray(src.astype(np.int64) if src.dtype.kind == "i" else src)
    if partial:
        undef = (t < 0) if t.dtype.kind == "i" else (t == np.iinfo(t.dtype).max)
        t = np.where(undef, UNDEF, t)
    t = np.ascontiguousarray(t, dtype=np.uint32)
    q = t.shape[0]
    alpha = np.frombuffer(bytes(alphabet), dtype=np.uint8).copy()
    fin = np.zeros(max(q, 1), dtype=np.uint8)
    acc = np.asarray(accepting, dtype=np.int64).reshape(-1)
    if acc.size and (acc.min() < 0 or acc.max() >= q):
        raise ValueError("accepting state out of range")
    fin[acc] = 1
    return t, alpha, fin


def _text(text) -> np.ndarray:
    if isinstance(text, (bytes, bytearray)):
        return np.frombuffer(bytes(text), dtype=np.uint8)
    return np.ascontiguousarray(text, dtype=np.uint8).reshape(-1)


@dataclass
class WalkResult:
    final_state: int
    accept: bool
    count: int


def walk(table, alphabet, start, accepting, text, partial: bool = False) -> WalkResult:
    """Sequential DFA run: final state, accept flag, number of steps whose
    destination is final. Raises OracleError(-4) on a byte outside the
    alphabet (``.bad_pos`` holds its offset). With ``partial``, a run that
    meets an undefined transition ends in DEAD (not accepting)."""
    lib = _load()
    t, alpha, fin = _prep(table, alphabet, accepting, partial)
    x = _text(text)
    fq = ctypes.c_uint32(0)
    cnt = ctypes.c_uint64(0)
    bad = ctypes.c_uint64(0)
    rc = lib.oracle_walk(_ptr(t, ctypes.c_uint32), t.shape[0], _ptr(alpha, ctypes.c_uint8), t.shape[1],
                         int(start), PARTIAL if partial else 0, _ptr(fin, ctypes.c_uint8),
                         _ptr(x, ctypes.c_uint8), x.size, ctypes.byref(fq), ctypes.byref(cnt), ctypes.byref(bad))
    if rc:
        err = OracleError(rc, "oracle_walk")
        err.bad_pos = int(bad.value)
        raise err
    f = int(fq.value)
    return WalkResult(f, bool(f < t.shape[0] and fin[f]), int(cnt.value))


def walk_dfa(dfa, text) -> WalkResult:
    return walk(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, partial=getattr(dfa, "partial", False))


def states_at(table, alphabet, start, accepting, text, positions, partial: bool = False):
    """State (and running count) after each prefix length in ``positions``
    (DEAD after a partial table's run died)."""
    lib = _load()
    t, alpha, fin = _prep(table, alphabet, accepting, partial)
    x = _text(text)
    pos = np.ascontiguousarray(positions, dtype=np.uint64).reshape(-1)
    st = np.zeros(pos.size, dtype=np.uint32)
    cn = np.zeros(pos.size, dtype=np.uint64)
    rc = lib.oracle_states_at(_ptr(t, ctypes.c_uint32), t.shape[0], _ptr(alpha, ctypes.c_uint8),
                              t.shape[1], int(start), PARTIAL if partial else 0, _ptr(fin, ctypes.c_uint8),
                              _ptr(x, ctypes.c_uint8), x.size, _ptr(pos, ctypes.c_uint64), pos.size,
                              _ptr(st, ctypes.c_uint32), _ptr(cn, ctypes.c_uint64))
    if rc:
        raise OracleError(rc, "oracle_states_at")
    return st, cn


def positions(table, alphabet, start, accepting, text, cap: int | None = None, partial: bool = False):
    """Offsets of the symbols whose step enters a final state (ascending):
    (first min(cap, total) offsets as uint64, total)."""
    lib = _load()
    t, alpha, fin = _prep(table, alphabet, accepting, partial)
    x = _text(text)
    total = ctypes.c_uint64(0)
    bad = ctypes.c_uint64(0)
    if cap is None:
        rc = lib.oracle_positions(_ptr(t, ctypes.c_uint32), t.shape[0], _ptr(alpha, ctypes.c_uint8), t.shape[1],
                                  int(start), PARTIAL if partial else 0, _ptr(fin, ctypes.c_uint8),
                                  _ptr(x, ctypes.c_uint8), x.size, None, 0, ctypes.byref(total), ctypes.byref(bad))
        if rc:
            raise OracleError(rc, "oracle_positions")
        cap = int(total.value)
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    rc = lib.oracle_positions(_ptr(t, ctypes.c_uint32), t.shape[0], _ptr(alpha, ctypes.c_uint8), t.shape[1],
                              int(start), PARTIAL if partial else 0, _ptr(fin, ctypes.c_uint8),
                              _ptr(x, ctypes.c_uint8), x.size, _ptr(out, ctypes.c_uint64), cap,
                              ctypes.byref(total), ctypes.byref(bad))
    if rc:
        err = OracleError(rc, "oracle_positions")
        err.bad_pos = int(bad.value)
        raise err
    return out[:min(cap, int(total.value))], int(total.value)


def positions_dfa(dfa, text, cap: int | None = None):
    return positions(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, cap,
                     partial=getattr(dfa, "partial", False))


@dataclass
class ParemResult:
    final_state: int
    accept: bool
    count: int
    runs: int
    entries: np.ndarray      # true entry state of each slice
    rsize: np.ndarray        # |R| of each slice
    traces: list | None      # [(slice, r, visited states)] when requested


def parem(table, alphabet, start, accepting, text, p: int, traces: bool = False, policy: int = POLICY_PAREM,
          partial: bool = False) -> ParemResult:
    """Algorithm 1 executed step by step with ``p`` slices (``policy``
    POLICY_ENUMERATE: every state speculated for every slice after the
    first)."""
    lib = _load()
    t, alpha, fin = _prep(table, alphabet, accepting, partial)
    x = _text(text)
    entries = np.zeros(p, dtype=np.uint32)
    rsize = np.zeros(p, dtype=np.uint32)
    fq = ctypes.c_uint32(0)
    cnt = ctypes.c_uint64(0)
    runs = ctypes.c_uint64(0)
    tl = ctypes.c_uint64(0)
    cap = 0
    tr = None
    if traces:
        cap = (3 + x.size) * t.shape[0] * max(p, 1) + 16
        tr = np.zeros(cap, dtype=np.uint32)
    rc = lib.oracle_parem(_ptr(t, ctypes.c_uint32), t.shape[0], _ptr(alpha, ctypes.c_uint8), t.shape[1],
                          int(start), PARTIAL if partial else 0, int(policy), _ptr(fin, ctypes.c_uint8),
                          _ptr(x, ctypes.c_uint8), x.size, p,
                          ctypes.byref(fq), ctypes.byref(cnt), ctypes.byref(runs),
                          _ptr(entries, ctypes.c_uint32), _ptr(rsize, ctypes.c_uint32),
                          _ptr(tr, ctypes.c_uint32), cap, ctypes.byref(tl))
    if rc:
        raise OracleError(rc, "oracle_parem")
    recs = None
    if traces:
        recs = []
        k = 0
        while k < tl.value:
            c, r, n = int(tr[k]), int(tr[k + 1]), int(tr[k + 2])
            recs.append((c, r, tr[k + 3:k + 3 + n].tolist()))
            k += 3 + n
    f = int(fq.value)
    return ParemResult(f, bool(f < t.shape[0] and fin[f]), int(cnt.value), int(runs.value), entries, rsize, recs)
