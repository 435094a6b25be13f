"""The allocation-free match entry point against parem_match_async.

parem_match_async_noalloc keeps its workspace in the library's device array;
its results must equal those of parem_match_async (caller workspace) bit for
bit, on two calls in a row, the second with a smaller input (the array keeps
the first call's contents), and a text whose workspace exceeds the array is
refused before anything runs.
"""
import sys

import numpy as np
import pytest

import workloads as W
from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_1412_1741_amd as P


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both(m, text):
    """(noalloc result bytes, async result bytes) for one device text."""
    s = torch.cuda.current_stream()
    out_a = torch.full((P.RESULT_BYTES,), 0xAB, dtype=torch.uint8, device="cuda")
    out_b = torch.full((P.RESULT_BYTES,), 0xCD, dtype=torch.uint8, device="cuda")
    P.parem_match_async_noalloc(m.handle, text.data_ptr(), text.numel(), s.cuda_stream, out_a.data_ptr())
    ws = torch.empty(max(P.parem_workspace_size(m.handle, text.numel()), 256), dtype=torch.uint8, device="cuda")
    P.parem_match_async(m.handle, text.data_ptr(), text.numel(), ws.data_ptr(), ws.numel(), s.cuda_stream,
                        out_b.data_ptr())
    torch.cuda.synchronize()
    return out_a.cpu().numpy().tobytes(), out_b.cpu().numpy().tobytes()


def test_noalloc_matches_async_twice():
    assert P.parem_noalloc_scratch_bytes() == 64 << 20
    dfa, text = W.dna_motif(n=(256 << 20) + 77, copies=20000)
    d = torch.from_numpy(text).cuda()
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    assert P.parem_workspace_size(m.handle, d.numel()) <= P.parem_noalloc_scratch_bytes()
    say(f"[case] noalloc: first call n={d.numel()}")
    a, b = both(m, d)
    assert a == b
    r = P.MatchResult.from_bytes(a)
    assert r.count > 0 and r.chunks > 0
    # a smaller second input: the array still holds the first call's maps
    small = d[: (3 << 20) + 5]
    say(f"[case] noalloc: second call n={small.numel()}")
    a2, b2 = both(m, small)
    assert a2 == b2 and a2 != a
    m.close()
    # other layouts and a partial table through the same array
    rng = np.random.default_rng(3)
    for lay in (P.LAYOUT_BYTE_LDS, P.LAYOUT_CLASS_LDS, P.LAYOUT_BYTE_GLOBAL):
        dd, tt = W.random_case(rng, max_states=100, max_alpha=8, max_len=2_000_000)
        mm = P.Matcher(dd.table, dd.alphabet, dd.start, dd.accepting, layout=lay, chunk_len=1024)
        a3, b3 = both(mm, torch.from_numpy(tt).cuda())
        assert a3 == b3, lay
        mm.close()
    t = rng.integers(0, 20, size=(20, 4)).astype(np.uint8)
    t[rng.random((20, 4)) < 0.02] = 255
    mp = P.Matcher(t, b"ACGT", 0, [3], partial=True, chunk_len=256)
    a4, b4 = both(mp, torch.from_numpy(W.uniform_text(rng, b"ACGT", 500_000)).cuda())
    assert a4 == b4
    mp.close()


def test_noalloc_refuses_oversized_and_empty_works():
    dfa, text = W.sparse4096(n=64 << 20)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    need = P.parem_workspace_size(m.handle, text.size)
    assert need > P.parem_noalloc_scratch_bytes()
    d = torch.from_numpy(text).cuda()
    out = torch.zeros(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.ParemError) as ei:
        P.parem_match_async_noalloc(m.handle, d.data_ptr(), d.numel(), torch.cuda.current_stream().cuda_stream,
                                    out.data_ptr())
    assert ei.value.status == P.PAREM_EUNSUPPORTED
    # an empty text needs no workspace
    P.parem_match_async_noalloc(m.handle, 0, 0, torch.cuda.current_stream().cuda_stream, out.data_ptr())
    r = P.MatchResult.from_bytes(out.cpu().numpy().tobytes())
    assert (r.final_state, r.count, r.chunks) == (dfa.start, 0, 0)
    m.close()
