"""Python binding of ``libparem.so``: the MI355X speculative chunked DFA walk.

Argument marshalling only. Every step of a match runs in the library's HIP
kernels; PyTorch is used for device memory and streams. The first call loads
the library and raises ImportError when it has not been built
(``python -m paper_1412_1741_amd.build``): there is no CPU fallback.

The functions carry the C names (``parem_compile``, ``parem_match``,
``parem_match_async``, ...); ``Matcher`` wraps a handle for convenience.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparem.so")

PAREM_OK = 0
PAREM_EINVAL = -1
PAREM_ENOMEM = -2
PAREM_EDEVICE = -3
PAREM_ESYMBOL = -4
PAREM_ESTATE = -5
PAREM_EUNSUPPORTED = -6
PAREM_ESYNTAX = -7

RE_ANCHORED = 0
RE_SEARCH = 1

LAYOUT_AUTO = 0
LAYOUT_BYTE_LDS = 1
LAYOUT_BYTE_GLOBAL = 2
LAYOUT_KGRAM_LDS = 3
LAYOUT_HOT_LDS = 4
LAYOUT_CLASS_LDS = 5
LAYOUT_SPARSE_LDS = 6

POLICY_PAREM = 0
POLICY_ENUMERATE = 1

RESULT_BYTES = 40
INVALID_STATE = 0xFFFFFFFF
DEAD_STATE = 0xFFFFFFFE


class ParemError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {parem_strerror(status)} ({status})")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("chunk_len", ctypes.c_uint32), ("layout", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("policy", ctypes.c_uint32), ("tile", ctypes.c_uint32), ("no_merge", ctypes.c_uint32),
                ("lookback", ctypes.c_uint32), ("partial", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("final_state", ctypes.c_uint32), ("accept", ctypes.c_uint32), ("count", ctypes.c_uint64),
                ("chunks", ctypes.c_uint64), ("spec_runs", ctypes.c_uint64), ("rerun_chunks", ctypes.c_uint64)]


assert ctypes.sizeof(Result) == RESULT_BYTES


class BatchInfo(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_uint32), ("walk_launches", ctypes.c_uint32), ("walk_items", ctypes.c_uint64),
                ("levels", ctypes.c_uint32), ("graph_nodes", ctypes.c_uint32), ("learned_pairs", ctypes.c_uint32),
                ("chunks", ctypes.c_uint64), ("text_bytes", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1412_1741_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.parem_compile.restype = i32
    lib.parem_compile.argtypes = [vp, i32, u32, vp, u32, u32, vp, u32, ctypes.POINTER(Options),
                                  ctypes.POINTER(vp)]
    lib.parem_regex_dfa.restype = i32
    lib.parem_regex_dfa.argtypes = [ctypes.c_char_p, u64, vp, u32, u32, u32, ctypes.POINTER(u32), vp, u64, vp, u64]
    lib.parem_compile_regex.restype = i32
    lib.parem_compile_regex.argtypes = [ctypes.c_char_p, u64, vp, u32, u32, ctypes.POINTER(Options),
                                        ctypes.POINTER(vp)]
    lib.parem_free.restype = None
    lib.parem_free.argtypes = [vp]
    lib.parem_strerror.restype = ctypes.c_char_p
    lib.parem_strerror.argtypes = [i32]
    lib.parem_describe.restype = i32
    lib.parem_describe.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32),
                                   ctypes.POINTER(u32)]
    lib.parem_workspace_size.restype = i32
    lib.parem_workspace_size.argtypes = [vp, u64, ctypes.POINTER(u64)]
    lib.parem_match_async.restype = i32
    lib.parem_match_async.argtypes = [vp, vp, u64, vp, u64, vp, vp]
    lib.parem_match_async_timed.restype = i32
    lib.parem_match_async_timed.argtypes = [vp, vp, u64, vp, u64, vp, vp, vp, vp]
    lib.parem_match_async_noalloc.restype = i32
    lib.parem_match_async_noalloc.argtypes = [vp, vp, u64, vp, vp]
    lib.parem_noalloc_scratch_bytes.restype = u64
    lib.parem_noalloc_scratch_bytes.argtypes = []
    lib.parem_read_sweep.restype = i32
    lib.parem_read_sweep.argtypes = [vp, u64, vp, vp]
    lib.parem_match.restype = i32
    lib.parem_match.argtypes = [vp, vp, u64, ctypes.POINTER(Result)]
    lib.parem_boundary_workspace_size.restype = i32
    lib.parem_boundary_workspace_size.argtypes = [vp, u64, u32, ctypes.POINTER(u64)]
    lib.parem_boundary_states.restype = i32
    lib.parem_boundary_states.argtypes = [vp, vp, u64, u32, vp, vp, u64, vp]
    lib.parem_positions_workspace_size.restype = i32
    lib.parem_positions_workspace_size.argtypes = [vp, u64, ctypes.POINTER(u64)]
    lib.parem_match_positions_async.restype = i32
    lib.parem_match_positions_async.argtypes = [vp, vp, u64, vp, u64, vp, u64, vp, vp]
    lib.parem_proposal_create.restype = i32
    lib.parem_proposal_create.argtypes = [vp, vp, u64, ctypes.POINTER(vp)]
    lib.parem_proposal_free.restype = None
    lib.parem_proposal_free.argtypes = [vp]
    lib.parem_proposal_params.restype = i32
    lib.parem_proposal_params.argtypes = [vp, vp, vp, u64]
    lib.parem_proposal_train_step.restype = i32
    lib.parem_proposal_train_step.argtypes = [vp, vp, u64, vp, vp, u32, ctypes.c_float, ctypes.c_float, vp, vp]
    lib.parem_proposal_logits.restype = i32
    lib.parem_proposal_logits.argtypes = [vp, vp, u64, vp, u32, vp, vp]
    lib.parem_proposal_apply_grad.restype = i32
    lib.parem_proposal_apply_grad.argtypes = [vp, vp, u64, ctypes.c_float, ctypes.c_float, vp]
    lib.parem_proposal_select_size.restype = i32
    lib.parem_proposal_select_size.argtypes = [vp, u64, u32, ctypes.POINTER(u64)]
    lib.parem_proposal_select.restype = i32
    lib.parem_proposal_select.argtypes = [vp, vp, u64, u32, u32, vp, vp, vp, u64, vp]
    lib.parem_learned_workspace_size.restype = i32
    lib.parem_learned_workspace_size.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
    lib.parem_match_learned_async.restype = i32
    lib.parem_match_learned_async.argtypes = [vp, vp, u32, vp, u64, vp, u64, vp, vp, vp, vp]
    lib.parem_batch_create.restype = i32
    lib.parem_batch_create.argtypes = [vp, vp, u32, vp, vp, vp, ctypes.POINTER(vp)]
    lib.parem_batch_run.restype = i32
    lib.parem_batch_run.argtypes = [vp, vp, vp, vp, i32]
    lib.parem_batch_describe.restype = i32
    lib.parem_batch_describe.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    lib.parem_batch_free.restype = None
    lib.parem_batch_free.argtypes = [vp]
    lib.parem_match_batch.restype = i32
    lib.parem_match_batch.argtypes = [vp, vp, vp, u32, vp, vp]
    lib.parem_tune.restype = i32
    lib.parem_tune.argtypes = [vp, vp, u64, u32, vp, u32, u32, vp, vp, ctypes.POINTER(u32)]
    return lib


_lib = None

# every symbol the header declares, for the export check
EXPORTED = ["parem_compile", "parem_regex_dfa", "parem_compile_regex", "parem_free", "parem_strerror", "parem_describe", "parem_workspace_size",
            "parem_match_async", "parem_match_async_timed", "parem_match_async_noalloc",
            "parem_noalloc_scratch_bytes", "parem_read_sweep", "parem_match", "parem_boundary_workspace_size",
            "parem_boundary_states", "parem_positions_workspace_size", "parem_match_positions_async",
            "parem_proposal_create", "parem_proposal_free", "parem_proposal_params",
            "parem_proposal_train_step", "parem_proposal_logits", "parem_proposal_apply_grad",
            "parem_proposal_select_size",
            "parem_proposal_select", "parem_learned_workspace_size",
            "parem_match_learned_async", "parem_batch_create", "parem_batch_run", "parem_batch_describe",
            "parem_batch_free", "parem_match_batch", "parem_tune"]


def lib() -> ctypes.CDLL:
    """The loaded library; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


# ---------------------------------------------------------------------------
# C names
# ---------------------------------------------------------------------------

def parem_strerror(status: int) -> str:
    return lib().parem_strerror(int(status)).decode()


def _check(status: int, where: str):
    if status != PAREM_OK:
        raise ParemError(status, where)


def parem_compile(table, alphabet, start: int, accepting, *, chunk_len: int = 0, layout: int = 0,
                  group: int = 0, tile: int = 0, no_merge: bool = False, lookback: int = 0,
                  policy: int = POLICY_PAREM, partial: bool = False) -> int:
    """Compile a DFA; returns the handle (an integer address). With
    ``partial`` the all-ones value of the table's unsigned type marks an
    undefined transition (a signed table's -1 is converted to it)."""
    t = np.ascontiguousarray(table)
    if t.ndim != 2:
        raise ValueError("table must be 2-D [num_states, alphabet_size]")
    if t.dtype not in (np.uint8, np.uint16, np.uint32):
        if partial and t.dtype.kind == "i":
            t = np.where(t < 0, 0xFFFFFFFF, t)
        t = np.ascontiguousarray(t, dtype=np.uint32)
    alpha = np.frombuffer(bytes(alphabet), dtype=np.uint8).copy()
    acc = np.ascontiguousarray(np.asarray(accepting, dtype=np.uint32).reshape(-1))
    opt = Options(chunk_len, layout, group, policy, tile, 1 if no_merge else 0, lookback, 1 if partial else 0)
    h = ctypes.c_void_p()
    st = lib().parem_compile(t.ctypes.data, t.dtype.itemsize, t.shape[0], alpha.ctypes.data, alpha.size,
                            int(start), acc.ctypes.data if acc.size else None, acc.size, ctypes.byref(opt),
                            ctypes.byref(h))
    _check(st, "parem_compile")
    return h.value


def parem_regex_dfa(pattern: bytes, alphabet, mode: int = RE_ANCHORED, partial: bool = False):
    """Host-side front-end: (table [Q, A] uint32 with 0xFFFFFFFF for undefined
    transitions, final flags [Q] uint8); start state 0."""
    pat = bytes(pattern)
    alpha = np.frombuffer(bytes(alphabet), dtype=np.uint8).copy()
    q = ctypes.c_uint32()
    _check(lib().parem_regex_dfa(pat, len(pat), alpha.ctypes.data, alpha.size, int(mode), 1 if partial else 0,
                                 ctypes.byref(q), None, 0, None, 0), "parem_regex_dfa")
    table = np.zeros((q.value, alpha.size), dtype=np.uint32)
    fin = np.zeros(q.value, dtype=np.uint8)
    _check(lib().parem_regex_dfa(pat, len(pat), alpha.ctypes.data, alpha.size, int(mode), 1 if partial else 0,
                                 ctypes.byref(q), table.ctypes.data, table.size, fin.ctypes.data, fin.size),
           "parem_regex_dfa")
    return table, fin


def parem_compile_regex(pattern: bytes, alphabet, mode: int = RE_ANCHORED, *, chunk_len: int = 0,
                        layout: int = 0, group: int = 0, tile: int = 0, no_merge: bool = False, lookback: int = 0,
                        policy: int = POLICY_PAREM, partial: bool = False) -> int:
    pat = bytes(pattern)
    alpha = np.frombuffer(bytes(alphabet), dtype=np.uint8).copy()
    opt = Options(chunk_len, layout, group, policy, tile, 1 if no_merge else 0, lookback, 1 if partial else 0)
    h = ctypes.c_void_p()
    _check(lib().parem_compile_regex(pat, len(pat), alpha.ctypes.data, alpha.size, int(mode), ctypes.byref(opt),
                                     ctypes.byref(h)), "parem_compile_regex")
    return h.value


def parem_free(handle: int) -> None:
    lib().parem_free(handle)


def parem_describe(handle: int) -> dict:
    a, b, c, d = (ctypes.c_uint32() for _ in range(4))
    _check(lib().parem_describe(handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)),
           "parem_describe")
    return {"layout": a.value, "max_spec": b.value, "lds_bytes": c.value, "kgram": d.value}


def parem_workspace_size(handle: int, length: int) -> int:
    n = ctypes.c_uint64()
    _check(lib().parem_workspace_size(handle, int(length), ctypes.byref(n)), "parem_workspace_size")
    return n.value


def parem_match_async(handle: int, d_text_ptr: int, length: int, d_workspace_ptr: int, workspace_bytes: int,
                      stream_ptr: int, d_out_ptr: int) -> None:
    """Enqueue a match; all pointers are device addresses (ints)."""
    _check(lib().parem_match_async(handle, d_text_ptr or None, int(length), d_workspace_ptr or None,
                                  int(workspace_bytes), stream_ptr or None, d_out_ptr), "parem_match_async")


def parem_match_async_timed(handle: int, d_text_ptr: int, length: int, d_workspace_ptr: int,
                            workspace_bytes: int, stream_ptr: int, d_out_ptr: int, ev_begin: int,
                            ev_end: int) -> None:
    """parem_match_async with hipEvent_t handles recorded around the walk kernel."""
    _check(lib().parem_match_async_timed(handle, d_text_ptr or None, int(length), d_workspace_ptr or None,
                                        int(workspace_bytes), stream_ptr or None, d_out_ptr, ev_begin or None,
                                        ev_end or None), "parem_match_async_timed")


def parem_match_async_noalloc(handle: int, d_text_ptr: int, length: int, stream_ptr: int, d_out_ptr: int) -> None:
    """parem_match_async with the library's own device scratch array (no
    workspace; allocates no device memory)."""
    _check(lib().parem_match_async_noalloc(handle, d_text_ptr or None, int(length), stream_ptr or None, d_out_ptr),
           "parem_match_async_noalloc")


def parem_read_sweep(d_buf_ptr: int, length: int, stream_ptr: int, d_sink_ptr: int) -> None:
    """One coalesced 16-byte-load read of a device buffer (the HBM read
    ceiling the walk is compared against; measurement helper)."""
    _check(lib().parem_read_sweep(d_buf_ptr, int(length), stream_ptr or None, d_sink_ptr), "parem_read_sweep")


def parem_noalloc_scratch_bytes() -> int:
    return int(lib().parem_noalloc_scratch_bytes())


def parem_boundary_workspace_size(handle: int, length: int, chunk_len: int) -> int:
    n = ctypes.c_uint64()
    _check(lib().parem_boundary_workspace_size(handle, int(length), int(chunk_len), ctypes.byref(n)),
           "parem_boundary_workspace_size")
    return n.value


def parem_boundary_states(handle: int, d_text_ptr: int, length: int, chunk_len: int, d_states_ptr: int,
                          d_workspace_ptr: int, workspace_bytes: int, stream_ptr: int) -> None:
    _check(lib().parem_boundary_states(handle, d_text_ptr or None, int(length), int(chunk_len), d_states_ptr or None,
                                       d_workspace_ptr or None, int(workspace_bytes), stream_ptr or None),
           "parem_boundary_states")


def parem_positions_workspace_size(handle: int, length: int) -> int:
    n = ctypes.c_uint64()
    _check(lib().parem_positions_workspace_size(handle, int(length), ctypes.byref(n)),
           "parem_positions_workspace_size")
    return n.value


def parem_match_positions_async(handle: int, d_text_ptr: int, length: int, d_pos_ptr: int, cap: int,
                                d_workspace_ptr: int, workspace_bytes: int, stream_ptr: int, d_out_ptr: int) -> None:
    _check(lib().parem_match_positions_async(handle, d_text_ptr or None, int(length), d_pos_ptr or None, int(cap),
                                             d_workspace_ptr or None, int(workspace_bytes), stream_ptr or None,
                                             d_out_ptr), "parem_match_positions_async")


def parem_proposal_create(handle: int, params: np.ndarray) -> int:
    w = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    out = ctypes.c_void_p()
    _check(lib().parem_proposal_create(handle, w.ctypes.data, w.size, ctypes.byref(out)), "parem_proposal_create")
    return out.value


def parem_proposal_free(proposal: int) -> None:
    lib().parem_proposal_free(proposal)


def parem_proposal_params(proposal: int, nparams: int, grad: bool = False) -> np.ndarray:
    out = np.empty(nparams, dtype=np.float32)
    if grad:
        _check(lib().parem_proposal_params(proposal, None, out.ctypes.data, nparams), "parem_proposal_params")
    else:
        _check(lib().parem_proposal_params(proposal, out.ctypes.data, None, nparams), "parem_proposal_params")
    return out


def parem_proposal_train_step(proposal: int, d_text_ptr: int, length: int, d_pos_ptr: int, d_labels_ptr: int,
                              batch: int, lr: float, weight_decay: float, stream_ptr: int, d_loss_ptr: int) -> None:
    _check(lib().parem_proposal_train_step(proposal, d_text_ptr, int(length), d_pos_ptr, d_labels_ptr, int(batch),
                                           float(lr), float(weight_decay), stream_ptr or None, d_loss_ptr or None),
           "parem_proposal_train_step")


def parem_proposal_logits(proposal: int, d_text_ptr: int, length: int, d_pos_ptr: int, batch: int,
                          d_logits_ptr: int, stream_ptr: int) -> None:
    _check(lib().parem_proposal_logits(proposal, d_text_ptr, int(length), d_pos_ptr, int(batch), d_logits_ptr,
                                       stream_ptr or None), "parem_proposal_logits")


def parem_proposal_apply_grad(proposal: int, d_grad_ptr: int, nparams: int, lr: float, weight_decay: float,
                              stream_ptr: int) -> None:
    _check(lib().parem_proposal_apply_grad(proposal, d_grad_ptr, int(nparams), float(lr), float(weight_decay),
                                           stream_ptr or None), "parem_proposal_apply_grad")


def parem_proposal_select_size(proposal: int, length: int, chunk_len: int) -> int:
    n = ctypes.c_uint64()
    _check(lib().parem_proposal_select_size(proposal, int(length), int(chunk_len), ctypes.byref(n)),
           "parem_proposal_select_size")
    return n.value


def parem_proposal_select(proposal: int, d_text_ptr: int, length: int, chunk_len: int, m: int, d_sel_ptr: int,
                          d_nsel_ptr: int, d_workspace_ptr: int, workspace_bytes: int, stream_ptr: int) -> None:
    _check(lib().parem_proposal_select(proposal, d_text_ptr, int(length), int(chunk_len), int(m), d_sel_ptr,
                                       d_nsel_ptr, d_workspace_ptr, int(workspace_bytes), stream_ptr or None),
           "parem_proposal_select")


def parem_learned_workspace_size(handle: int, proposal: int, length: int) -> int:
    n = ctypes.c_uint64()
    _check(lib().parem_learned_workspace_size(handle, proposal, int(length), ctypes.byref(n)),
           "parem_learned_workspace_size")
    return n.value


def parem_match_learned_async(handle: int, proposal: int, m: int, d_text_ptr: int, length: int,
                              d_workspace_ptr: int, workspace_bytes: int, stream_ptr: int, d_out_ptr: int,
                              ev_begin: int = 0, ev_end: int = 0) -> None:
    _check(lib().parem_match_learned_async(handle, proposal, int(m), d_text_ptr or None, int(length),
                                           d_workspace_ptr or None, int(workspace_bytes), stream_ptr or None,
                                           d_out_ptr, ev_begin or None, ev_end or None), "parem_match_learned_async")


def _options_array(opts):
    if opts is None:
        return None
    arr = (Options * len(opts))()
    for i, o in enumerate(opts):
        arr[i] = o if isinstance(o, Options) else Options(**o)
    return arr


def _u64_array(values):
    return np.ascontiguousarray(np.asarray(values, dtype=np.uint64).reshape(-1))


def parem_batch_create(handles, lens, opts=None, proposals=None, m=None) -> int:
    """Plan a batch; ``opts`` is None or one Options (or dict of its fields) per
    pair; ``proposals`` is None or one proposal handle (or 0: plain) per pair,
    with ``m`` the top-m of each learned pair."""
    n = len(handles)
    hs = (ctypes.c_void_p * max(n, 1))(*handles)
    ln = _u64_array(lens)
    if ln.size != n:
        raise ValueError("one length per pair")
    oa = _options_array(opts)
    pa = None
    ma = None
    if proposals is not None:
        pa = (ctypes.c_void_p * max(n, 1))(*[p or None for p in proposals])
        ma = np.ascontiguousarray(np.asarray(m if m is not None else [0] * n, dtype=np.uint32).reshape(-1))
    b = ctypes.c_void_p()
    _check(lib().parem_batch_create(hs, ln.ctypes.data, n, oa, pa, ma.ctypes.data if ma is not None else None,
                                    ctypes.byref(b)), "parem_batch_create")
    return b.value


def parem_batch_run(batch: int, d_text_ptrs, stream_ptr: int, d_out_ptr: int, use_graph: bool = True) -> None:
    ptrs = _u64_array(d_text_ptrs)
    _check(lib().parem_batch_run(batch, ptrs.ctypes.data, stream_ptr or None, d_out_ptr, 1 if use_graph else 0),
           "parem_batch_run")


def parem_batch_describe(batch: int) -> dict:
    info = BatchInfo()
    _check(lib().parem_batch_describe(batch, ctypes.byref(info)), "parem_batch_describe")
    return {f: int(getattr(info, f)) for f, _ in BatchInfo._fields_}


def parem_batch_free(batch: int) -> None:
    lib().parem_batch_free(batch)


def parem_match_batch(handles, d_text_ptrs, lens, stream_ptr: int, d_out_ptr: int) -> None:
    n = len(handles)
    hs = (ctypes.c_void_p * max(n, 1))(*handles)
    ptrs = _u64_array(d_text_ptrs)
    ln = _u64_array(lens)
    _check(lib().parem_match_batch(hs, ptrs.ctypes.data, ln.ctypes.data, n, stream_ptr or None, d_out_ptr),
           "parem_match_batch")


def parem_tune(handle: int, d_sample_ptr: int, sample_len: int, copies: int, cands, reps: int,
               stream_ptr: int):
    """Times candidate options (Options or dicts); returns (ms per copy list, best index)."""
    oa = _options_array(cands)
    ms = np.zeros(len(cands), dtype=np.float32)
    best = ctypes.c_uint32()
    _check(lib().parem_tune(handle, d_sample_ptr, int(sample_len), int(copies), oa, len(cands), int(reps),
                            stream_ptr or None, ms.ctypes.data, ctypes.byref(best)), "parem_tune")
    return [float(x) for x in ms], int(best.value)


def parem_match(handle: int, text_ptr: int, length: int) -> Result:
    """Synchronous match on a host or device address."""
    r = Result()
    _check(lib().parem_match(handle, text_ptr or None, int(length), ctypes.byref(r)), "parem_match")
    return r


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

@dataclass
class MatchResult:
    final_state: int
    accept: bool
    count: int
    chunks: int
    spec_runs: int
    rerun_chunks: int

    @classmethod
    def from_struct(cls, r: Result) -> "MatchResult":
        return cls(int(r.final_state), bool(r.accept), int(r.count), int(r.chunks), int(r.spec_runs),
                   int(r.rerun_chunks))

    @classmethod
    def from_bytes(cls, raw: bytes) -> "MatchResult":
        return cls.from_struct(Result.from_buffer_copy(raw))


class Matcher:
    """Owns a compiled handle; matches torch uint8 device tensors or host bytes."""

    def __init__(self, table, alphabet, start, accepting, **opts):
        self.handle = parem_compile(table, alphabet, start, accepting, **opts)
        self.num_states = int(np.asarray(table).shape[0])
        self._ws = {}
        self._lws = None

    @classmethod
    def from_regex(cls, pattern: bytes, alphabet, mode: int = RE_ANCHORED, **opts) -> "Matcher":
        """A matcher of a regular expression (Section III front-end)."""
        self = cls.__new__(cls)
        self.handle = parem_compile_regex(pattern, alphabet, mode, **opts)
        table, _ = parem_regex_dfa(pattern, alphabet, mode, opts.get("partial", False))
        self.num_states = int(table.shape[0])
        self._ws = {}
        self._lws = None
        return self

    def close(self):
        if self.handle:
            parem_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def describe(self) -> dict:
        return parem_describe(self.handle)

    def describe_states(self) -> int:
        return self.num_states

    def learned_workspace(self, proposal: "Proposal", length: int):
        import torch
        need = parem_learned_workspace_size(self.handle, proposal.handle, length)
        if self._lws is None or self._lws.numel() < need:
            self._lws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        return self._lws

    def match_learned_async(self, proposal: "Proposal", text, m: int, out=None, ev_begin=0, ev_end=0):
        import torch
        assert text.is_cuda and text.dtype == torch.uint8 and text.is_contiguous()
        ws = self.learned_workspace(proposal, text.numel())
        if out is None:
            out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=text.device)
        parem_match_learned_async(self.handle, proposal.handle, m, text.data_ptr(), text.numel(), ws.data_ptr(),
                                  ws.numel(), torch.cuda.current_stream().cuda_stream, out.data_ptr(), ev_begin,
                                  ev_end)
        return out

    def match_learned(self, proposal: "Proposal", text, m: int) -> MatchResult:
        out = self.match_learned_async(proposal, text, m)
        res = MatchResult.from_bytes(out.cpu().numpy().tobytes())
        if res.final_state == INVALID_STATE:
            raise ParemError(PAREM_ESYMBOL, "parem_match_learned_async")
        return res

    def workspace(self, length: int, stream=None):
        """Workspace for a match of ``length`` bytes on ``stream`` (default:
        torch's current stream). Each stream has its own, so that matches
        enqueued on different streams never share one. It is allocated on
        that stream, so when a larger one replaces it the caching allocator
        reuses its memory only in that stream's order."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        need = parem_workspace_size(self.handle, length)
        ws = self._ws.get(s.cuda_stream)
        if ws is None or ws.numel() < need:
            with torch.cuda.stream(s):
                ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
            self._ws[s.cuda_stream] = ws
        return ws

    def match_async(self, text, out=None, stream=None):
        """Enqueue on torch's current stream (or ``stream``); returns the
        40-byte device result tensor (allocated on that stream when not
        given; a caller's ``out`` is recorded on it)."""
        import torch
        assert text.is_cuda and text.dtype == torch.uint8 and text.is_contiguous()
        s = stream if stream is not None else torch.cuda.current_stream()
        ws = self.workspace(text.numel(), s)
        if out is None:
            with torch.cuda.stream(s):
                out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=text.device)
        elif s != torch.cuda.current_stream():
            out.record_stream(s)
        if s != torch.cuda.current_stream():
            text.record_stream(s)
        parem_match_async(self.handle, text.data_ptr(), text.numel(), ws.data_ptr(), ws.numel(), s.cuda_stream,
                          out.data_ptr())
        return out

    def positions(self, text, cap: int | None = None):
        """Offsets of the bytes whose step enters a final state (uint64
        device tensor, ascending) and the match result. With cap None a plain
        match first sizes the output to the count."""
        import torch
        assert text.is_cuda and text.dtype == torch.uint8 and text.is_contiguous()
        if cap is None:
            cap = self.match(text).count
        s = torch.cuda.current_stream()
        ws = torch.empty(max(parem_positions_workspace_size(self.handle, text.numel()), 256), dtype=torch.uint8,
                         device=text.device)
        pos = torch.empty(max(int(cap), 1), dtype=torch.int64, device=text.device)
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=text.device)
        parem_match_positions_async(self.handle, text.data_ptr(), text.numel(), pos.data_ptr(), int(cap),
                                    ws.data_ptr(), ws.numel(), s.cuda_stream, out.data_ptr())
        res = MatchResult.from_bytes(out.cpu().numpy().tobytes())
        if res.final_state == INVALID_STATE:
            raise ParemError(PAREM_ESYMBOL, "parem_match_positions_async")
        return pos[:min(int(cap), res.count)], res

    def match(self, text) -> MatchResult:
        try:
            import torch
            is_tensor = isinstance(text, torch.Tensor)
        except ImportError:
            is_tensor = False
        if is_tensor and text.is_cuda:
            out = self.match_async(text)
            raw = out.cpu().numpy().tobytes()
            res = MatchResult.from_bytes(raw)
            if res.final_state == INVALID_STATE:
                raise ParemError(PAREM_ESYMBOL, "parem_match_async")
            return res
        if is_tensor:
            text = text.numpy()
        arr = np.ascontiguousarray(np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray))
                                   else text, dtype=np.uint8).reshape(-1)
        return MatchResult.from_struct(parem_match(self.handle, arr.ctypes.data, arr.size))


class Batch:
    """A planned batch of (Matcher, text length) pairs; ``run`` matches one
    set of uint8 device tensors of those lengths (16-byte aligned)."""

    def __init__(self, matchers, lens, opts=None, proposals=None, m=None):
        self.handles = [m_.handle for m_ in matchers]
        self._matchers = list(matchers)  # the handles and proposals must outlive the plan
        self._proposals = list(proposals) if proposals is not None else None
        self.lens = [int(x) for x in lens]
        props = None if proposals is None else [p.handle if p is not None else 0 for p in proposals]
        self.handle = parem_batch_create(self.handles, self.lens, opts, props, m)

    def close(self):
        if self.handle:
            parem_batch_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def describe(self) -> dict:
        return parem_batch_describe(self.handle)

    def run_async(self, texts, out=None, use_graph: bool = True, stream=None):
        import torch
        if len(texts) != len(self.lens):
            raise ValueError("one text per pair")
        for t, n in zip(texts, self.lens):
            assert t.is_cuda and t.dtype == torch.uint8 and t.is_contiguous() and t.numel() == n
        if out is None:
            out = torch.empty(max(len(texts), 1) * RESULT_BYTES, dtype=torch.uint8, device="cuda")
        s = stream if stream is not None else torch.cuda.current_stream()
        parem_batch_run(self.handle, [t.data_ptr() for t in texts], s.cuda_stream, out.data_ptr(), use_graph)
        return out

    @staticmethod
    def results(out, n: int):
        raw = out[: n * RESULT_BYTES].cpu().numpy().tobytes()
        return [MatchResult.from_bytes(raw[i * RESULT_BYTES:(i + 1) * RESULT_BYTES]) for i in range(n)]

    def run(self, texts, use_graph: bool = True):
        out = self.run_async(texts, use_graph=use_graph)
        return self.results(out, len(texts))


# ---------------------------------------------------------------------------
# learned proposal
# ---------------------------------------------------------------------------

MLP_WINDOW = 32


def proposal_param_count(states: int) -> int:
    """4096 (embedding) + 131328 (layer 1) + 65792 (layer 2) + 257 per state."""
    return 256 * 16 + 256 * 512 + 256 + 256 * 256 + 256 + 257 * states


class Proposal:
    """Owns a proposal network on the device (fp32 master weights, bf16 copy)."""

    def __init__(self, matcher: "Matcher", params):
        self.matcher = matcher
        self.states = int(matcher.describe_states())
        self.nparams = proposal_param_count(self.states)
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if p.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {p.size}")
        self.handle = parem_proposal_create(matcher.handle, p)

    def close(self):
        if self.handle:
            parem_proposal_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        return parem_proposal_params(self.handle, self.nparams)

    def grad(self) -> np.ndarray:
        return parem_proposal_params(self.handle, self.nparams, grad=True)

    def logits(self, text, positions):
        import torch
        pos = torch.as_tensor(np.asarray(positions, dtype=np.uint64).view(np.int64), device=text.device)
        out = torch.empty((pos.numel(), self.states), dtype=torch.float32, device=text.device)
        parem_proposal_logits(self.handle, text.data_ptr(), text.numel(), pos.data_ptr(), pos.numel(),
                              out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        return out

    def apply_grad(self, grad, lr: float, weight_decay: float = 0.01):
        """One AdamW step with ``grad`` (float32 device tensor, nparams)."""
        import torch
        assert grad.is_cuda and grad.dtype == torch.float32 and grad.numel() == self.nparams
        g = grad.contiguous()
        parem_proposal_apply_grad(self.handle, g.data_ptr(), self.nparams, lr, weight_decay,
                                  torch.cuda.current_stream().cuda_stream)

    def select(self, text, chunk_len: int, m: int):
        """(positions [chunks, m] within each chunk's speculated list, counts)"""
        import torch
        n = text.numel()
        chunks = (n + chunk_len - 1) // chunk_len
        ws = torch.empty(parem_proposal_select_size(self.handle, n, chunk_len), dtype=torch.uint8,
                         device=text.device)
        sel = torch.zeros((chunks, m), dtype=torch.int16, device=text.device)
        nsel = torch.zeros(chunks, dtype=torch.uint8, device=text.device)
        parem_proposal_select(self.handle, text.data_ptr(), n, chunk_len, m, sel.data_ptr(), nsel.data_ptr(),
                              ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
        return sel, nsel

    def train_step(self, text, positions, labels, lr: float, weight_decay: float = 0.01):
        """positions / labels: int64 / int32 device tensors. Returns the loss
        as a device tensor (no synchronisation)."""
        import torch
        loss = torch.zeros(1, dtype=torch.float32, device=text.device)
        parem_proposal_train_step(self.handle, text.data_ptr(), text.numel(), positions.data_ptr(),
                                  labels.data_ptr(), positions.numel(), lr, weight_decay,
                                  torch.cuda.current_stream().cuda_stream, loss.data_ptr())
        return loss


def boundary_states(matcher: "Matcher", text, chunk_len: int):
    """True state at every multiple of chunk_len (device u32 tensor, one per
    chunk), computed by the HIP walk + composition + down-sweep."""
    import torch
    n = text.numel()
    chunks = (n + chunk_len - 1) // chunk_len
    need = parem_boundary_workspace_size(matcher.handle, n, chunk_len)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=text.device)
    out = torch.empty(max(chunks, 1), dtype=torch.int32, device=text.device)
    parem_boundary_states(matcher.handle, text.data_ptr(), n, chunk_len, out.data_ptr(), ws.data_ptr(), ws.numel(),
                          torch.cuda.current_stream().cuda_stream)
    return out[:chunks]


def train_proposal(matcher: "Matcher", text, params, *, steps: int, batch: int = 4096, lr: float = 1e-3,
                   weight_decay: float = 0.01, label_stride: int = 64, seed: int = 0, log_every: int = 0):
    """Train a proposal on the states at every label_stride bytes of `text`
    (a device uint8 tensor). Labels come from boundary_states (the HIP path).
    Returns (Proposal, list of (step, loss))."""
    import torch
    prop = Proposal(matcher, params)
    states = boundary_states(matcher, text, label_stride)
    n_lab = states.numel()
    pos_all = torch.arange(n_lab, dtype=torch.int64, device=text.device) * label_stride
    # the first boundary (q0, no window) teaches nothing; boundaries after a
    # byte outside the alphabet have no state (0xffffffff) and are dropped
    keep = (pos_all > 0) & (states != -1)
    pos_all, states = pos_all[keep], states[keep]
    if pos_all.numel() == 0:
        raise ValueError("no labelled boundary in the training text")
    g = torch.Generator(device="cpu").manual_seed(seed)
    history = []
    n = pos_all.numel()
    for step in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(text.device)
        loss = prop.train_step(text, pos_all[idx].contiguous(), states[idx].contiguous(), lr, weight_decay)
        if log_every and (step % log_every == 0 or step == steps - 1):
            history.append((step, float(loss.item())))
    return prop, history
