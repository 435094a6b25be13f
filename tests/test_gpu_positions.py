"""GPU parity of match positions against the oracle, offset by offset.

The oracle lists the offset of every byte whose step enters a final state
(pinned in test_oracle_pins.py to word ends, Python's re and the motif's
sliding compare). The GPU path (walk, composition, down-sweep of entry
states, scan of per-chunk counts, second walk of the chunks with matches)
must give the same offsets, bit-exact, and the same count.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_1412_1741_amd as P


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


PAREL = b"parel"
TABLE1 = np.asarray([[1, 0, 0, 0, 0], [1, 2, 0, 0, 0], [1, 0, 3, 0, 0], [1, 4, 0, 0, 0], [1, 0, 0, 0, 5],
                     [1, 0, 0, 0, 6], [1, 0, 0, 7, 0], [1, 0, 0, 0, 8], [1, 0, 0, 0, 0]], dtype=np.uint8)


def pos_case(name, table, alphabet, start, accepting, text, offset=0, cap=None, partial=False, **opts):
    say(f"[case] positions {name}: Q={table.shape[0]} n={text.size} cap={cap} opts={opts} off={offset}")
    t = table
    if partial:
        t = np.where(table < 0, np.iinfo(np.uint16).max, table).astype(np.uint16)
    m = P.Matcher(t, alphabet, start, accepting, partial=partial, **opts)
    buf = torch.empty(text.size + offset + 16, dtype=torch.uint8, device="cuda")
    d = buf[offset:offset + text.size]
    if text.size:
        d.copy_(torch.from_numpy(text))
    want, total = oracle.positions(table, alphabet, start, accepting, text, cap=cap, partial=partial)
    got, res = m.positions(d, cap)
    assert res.count == total, (res.count, total)
    g = got.cpu().numpy().view(np.uint64)
    assert g.size == want.size and np.array_equal(g, want), name
    plain = m.match(d)
    assert (plain.final_state, plain.count) == (res.final_state, res.count)
    m.close()
    return total


def test_positions_parallel_words():
    rng = np.random.default_rng(1)
    text = np.frombuffer(PAREL, dtype=np.uint8)[rng.integers(0, 5, size=2_000_003)].copy()
    for o in rng.integers(0, text.size - 8, size=5000):
        text[o:o + 8] = np.frombuffer(b"parallel", dtype=np.uint8)
    for L in (64, 1024, 0):
        total = pos_case(f"words L={L}", TABLE1, PAREL, 0, [8], text, chunk_len=L)
        assert total > 4000
    pos_case("words, unaligned", TABLE1, PAREL, 0, [8], text, offset=3, chunk_len=256)
    pos_case("words, cap 100", TABLE1, PAREL, 0, [8], text, cap=100, chunk_len=256)
    pos_case("words, cap 0", TABLE1, PAREL, 0, [8], text, cap=0, chunk_len=256)


def test_positions_motif_4MiB_and_edges():
    dfa, text = W.dna_motif(n=(4 << 20) + 5, copies=3000)
    pos_case("motif 4 MiB", dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text)
    none = W.uniform_text(np.random.default_rng(3), b"AC", 100_000)  # the motif needs G/T
    assert pos_case("no matches", dfa.table, dfa.alphabet, dfa.start, dfa.accepting, none) == 0
    for n in (0, 1, 63, 65, 1000):
        pos_case(f"tiny n={n}", dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text[:n].copy())


def test_positions_motif_full_size():
    """The 1 GiB DNA workload (1e5 planted copies): every offset equals the
    oracle's."""
    dfa, text = W.dna_motif()
    total = pos_case("motif 1 GiB", dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text)
    assert total >= 99_000


def test_positions_random_layouts():
    rng = np.random.default_rng(7)
    for lay in (P.LAYOUT_AUTO, P.LAYOUT_BYTE_LDS, P.LAYOUT_CLASS_LDS, P.LAYOUT_BYTE_GLOBAL, P.LAYOUT_HOT_LDS,
                P.LAYOUT_SPARSE_LDS):
        for i in range(3):
            dfa, text = W.random_case(rng, max_states=200, max_alpha=20, max_len=500_000)
            pos_case(f"random layout={lay} {i}", dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text,
                     layout=lay, chunk_len=int(rng.choice([64, 512, 4096])))
    dfa, text = W.sparse4096(n=1 << 22)
    pos_case("sparse byte DFA", dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text)


def test_positions_partial():
    rng = np.random.default_rng(8)
    for i in range(4):
        q, a = 30 + 40 * i, 5
        alphabet = b"ACGTN"
        t = rng.integers(0, q, size=(q, a)).astype(np.int64)
        t[rng.random(q) < 0.5, a - 1] = -1
        text = W.uniform_text(rng, alphabet[:-1], 600_000)
        text[rng.integers(0, text.size, size=i)] = ord("N")
        pos_case(f"partial {i}", t, alphabet, 0, rng.choice(q, size=3, replace=False), text, partial=True,
                 chunk_len=512)


def test_positions_invalid_byte():
    dfa, text = W.dna_motif(n=1 << 20, copies=100)
    text = text.copy()
    text[70000] = ord("N")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    with pytest.raises(P.ParemError) as ei:
        m.positions(torch.from_numpy(text).cuda(), 10)
    assert ei.value.status == P.PAREM_ESYMBOL
    m.close()
