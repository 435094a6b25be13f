"""CPU oracle for the speculative chunked DFA walk.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library under
``paper_1412_1741_amd`` never does, and this package imports nothing from it.

The C part (``parem_oracle.c``) is a plain single-threaded DFA run plus a
step-by-step execution of the paper's Algorithm 1; this module loads it with
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
        lib.oracle_walk.argtypes = [u32p, ctypes.c_uint32, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                    u8p, u8p, ctypes.c_uint64, u32p, u64p, u64p]
        lib.oracle_states_at.restype = ctypes.c_int
        lib.oracle_states_at.argtypes = [u32p, ctypes.c_uint32, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                         u8p, u8p, ctypes.c_uint64, u64p, ctypes.c_uint64, u32p, u64p]
        lib.oracle_parem.restype = ctypes.c_int
        lib.oracle_parem.argtypes = [u32p, ctypes.c_uint32, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                     u8p, u8p, ctypes.c_uint64, ctypes.c_uint64, u32p, u64p, u64p,
                                     u32p, u32p, u32p, ctypes.c_uint64, u64p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _prep(table, alphabet, accepting, num_states=None):
    t = np.ascontiguousarray(np.asarray(table), dtype=np.uint32)
    if t.ndim != 2:
        raise ValueError("table must be 2-D [Q, A]")
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


def walk(table, alphabet, start, accepting, text) -> WalkResult:
    """Sequential DFA run: final state, accept flag, number of steps whose
    destination is final. Raises OracleError(-4) on a byte outside the
    alphabet (``.bad_pos`` holds its offset)."""
    lib = _load()
    t, alpha, fin = _prep(table, alphabet, accepting)
    x = _text(text)
    fq = ctypes.c_uint32(0)
    cnt = ctypes.c_uint64(0)
    bad = ctypes.c_uint64(0)
    rc = lib.oracle_walk(_ptr(t, ctypes.c_uint32), t.shape[0], _ptr(alpha, ctypes.c_uint8), t.shape[1],
                         int(start), _ptr(fin, ctypes.c_uint8), _ptr(x, ctypes.c_uint8), x.size,
                         ctypes.byref(fq), ctypes.byref(cnt), ctypes.byref(bad))
    if rc:
        err = OracleError(rc, "oracle_walk")
        err.bad_pos = int(bad.value)
        raise err
    return WalkResult(int(fq.value), bool(fin[fq.value]), int(cnt.value))


def walk_dfa(dfa, text) -> WalkResult:
    return walk(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text)


def states_at(table, alphabet, start, accepting, text, positions):
    """State (and running count) after each prefix length in ``positions``."""
    lib = _load()
    t, alpha, fin = _prep(table, alphabet, accepting)
    x = _text(text)
    pos = np.ascontiguousarray(positions, dtype=np.uint64).reshape(-1)
    st = np.zeros(pos.size, dtype=np.uint32)
    cn = np.zeros(pos.size, dtype=np.uint64)
    rc = lib.oracle_states_at(_ptr(t, ctypes.c_uint32), t.shape[0], _ptr(alpha, ctypes.c_uint8),
                              t.shape[1], int(start), _ptr(fin, ctypes.c_uint8),
                              _ptr(x, ctypes.c_uint8), x.size, _ptr(pos, ctypes.c_uint64), pos.size,
                              _ptr(st, ctypes.c_uint32), _ptr(cn, ctypes.c_uint64))
    if rc:
        raise OracleError(rc, "oracle_states_at")
    return st, cn


@dataclass
class ParemResult:
    final_state: int
    accept: bool
    count: int
    runs: int
    entries: np.ndarray      # true entry state of each slice
    rsize: np.ndarray        # |R| of each slice
    traces: list | None      # [(slice, r, visited states)] when requested


def parem(table, alphabet, start, accepting, text, p: int, traces: bool = False) -> ParemResult:
    """Algorithm 1 executed step by step with ``p`` slices."""
    lib = _load()
    t, alpha, fin = _prep(table, alphabet, accepting)
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
                          int(start), _ptr(fin, ctypes.c_uint8), _ptr(x, ctypes.c_uint8), x.size, p,
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
    return ParemResult(int(fq.value), bool(fin[fq.value]), int(cnt.value), int(runs.value),
                       entries, rsize, recs)
