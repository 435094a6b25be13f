"""GPU parity of the Enumeration policy and of partial tables.

* Enumeration (every state speculated for every chunk after the first; the
  approach Section IV-A compares against): bit-exact (final, accept, count)
  against the oracle, and exactly 1 + (chunks - 1) * Q walks.
* Partial tables (undefined transitions; Algorithm 1's S set): bit-exact
  against the oracle's partial run (PAREM_DEAD_STATE where the run met an
  undefined transition), and as many walks as S intersect L holds over the
  chunks, counted here from the definition with numpy: L = destinations of
  the defined transitions on the byte before the chunk, S = states with a
  transition on its first byte.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


PAREL = b"parel"
TABLE1 = np.asarray([[1, 0, 0, 0, 0], [1, 2, 0, 0, 0], [1, 0, 3, 0, 0], [1, 4, 0, 0, 0], [1, 0, 0, 0, 5],
                     [1, 0, 0, 0, 6], [1, 0, 0, 7, 0], [1, 0, 0, 0, 8], [1, 0, 0, 0, 0]], dtype=np.uint8)


# ---------------------------------------------------------------------------
# Enumeration
# ---------------------------------------------------------------------------

def enum_case(name, dfa, text, **opts):
    say(f"[case] enumerate {name}: Q={dfa.num_states} n={text.size} opts={opts}")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, policy=P.POLICY_ENUMERATE, **opts)
    got = m.match(dev(text))
    want = oracle.walk_dfa(dfa, text)
    assert (got.final_state, got.accept, got.count) == (want.final_state, want.accept, want.count), name
    L = opts.get("chunk_len")
    if L:
        chunks = (text.size + L - 1) // L
        assert got.chunks == chunks
        assert got.spec_runs == 1 + (chunks - 1) * dfa.num_states
        if text.size % L == 0:
            # the oracle's balanced split is the same chunking here
            r = oracle.parem(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, p=chunks,
                             policy=oracle.POLICY_ENUMERATE)
            assert got.spec_runs == r.runs and (got.final_state, got.count) == (r.final_state, r.count)
    m.close()
    return got


def test_enumeration_parallel_automaton():
    """The 9-state automaton of Table I over {p,a,r,e,l}: 28 walks on four
    chunks (Section II-C's count), and long texts on every layout."""
    dfa = W.Dfa(TABLE1, PAREL, 0, np.asarray([8], dtype=np.uint32))
    rng = np.random.default_rng(1)
    text = np.frombuffer(PAREL, dtype=np.uint8)[rng.integers(0, 5, size=256)].copy()
    got = enum_case("four chunks", dfa, text, chunk_len=64)
    assert got.spec_runs == 28
    text = np.frombuffer(PAREL, dtype=np.uint8)[rng.integers(0, 5, size=3_000_017)].copy()
    for o in range(0, text.size - 8, 997):
        text[o:o + 8] = np.frombuffer(b"parallel", dtype=np.uint8)
    for lay in (P.LAYOUT_AUTO, P.LAYOUT_BYTE_LDS, P.LAYOUT_CLASS_LDS, P.LAYOUT_BYTE_GLOBAL):
        for nm in (False, True):
            enum_case(f"layout={lay} no_merge={nm}", dfa, text, chunk_len=1024, layout=lay, no_merge=nm)


def test_enumeration_motif_and_random():
    dfa, text = W.dna_motif(n=4 << 20)
    enum_case("motif", dfa, text, chunk_len=4096)
    enum_case("motif, paper scheme", dfa, text, chunk_len=4096, no_merge=True, group=16)
    rng = np.random.default_rng(5)
    for i in range(10):
        d, t = W.random_case(rng, max_states=60, max_alpha=8, max_len=200_000)
        if t.size == 0:
            continue
        enum_case(f"random {i}", d, t, chunk_len=int(rng.choice([64, 256, 2048])))


def test_enumeration_gives_plain_results_with_more_walks():
    dfa, text = W.dna_motif(n=1 << 20)
    plain = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=1024)
    enum = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=1024, policy=P.POLICY_ENUMERATE)
    a, b = plain.match(dev(text)), enum.match(dev(text))
    assert (a.final_state, a.count) == (b.final_state, b.count)
    say(f"[enum] walks: PaREM {a.spec_runs}, Enumeration {b.spec_runs}")
    assert b.spec_runs > 2 * a.spec_runs
    plain.close()
    enum.close()


# ---------------------------------------------------------------------------
# partial tables
# ---------------------------------------------------------------------------

def partial_runs(table, alphabet, text, L):
    """1 + sum over chunks c >= 1 of |S intersect L| (undefined entries < 0)."""
    n = text.size
    chunks = (n + L - 1) // L
    col = np.full(256, -1, dtype=np.int64)
    col[np.frombuffer(alphabet, dtype=np.uint8)] = np.arange(len(alphabet))
    cache = {}
    runs = 1
    for c in range(1, chunks):
        key = (int(col[text[c * L - 1]]), int(col[text[c * L]]))
        if key not in cache:
            prev, first = key
            dest = table[:, prev]
            lset = np.zeros(table.shape[0], dtype=bool)
            lset[dest[dest >= 0]] = True
            cache[key] = int(np.count_nonzero(lset & (table[:, first] >= 0)))
        runs += cache[key]
    return runs, cache


def partial_case(name, table, alphabet, start, accepting, text, chunk_len, dtype=np.uint16, **opts):
    """table: int64 with -1 for undefined entries; compiled as `dtype` with
    the all-ones value marking them."""
    say(f"[case] partial {name}: Q={table.shape[0]} A={table.shape[1]} n={text.size} L={chunk_len} {opts}")
    t = np.where(table < 0, np.iinfo(dtype).max, table).astype(dtype)
    m = P.Matcher(t, alphabet, start, accepting, chunk_len=chunk_len, partial=True, **opts)
    got = m.match(dev(text))
    want = oracle.walk(table, alphabet, start, accepting, text, partial=True)
    wf = P.DEAD_STATE if want.final_state == oracle.DEAD else want.final_state
    assert (got.final_state, got.accept, got.count) == (wf, want.accept, want.count), name
    runs, cache = partial_runs(table, alphabet, text, chunk_len)
    assert got.spec_runs == runs, (got.spec_runs, runs)
    m.close()
    return got, cache


def rare_column_dfa(rng, q, a, undef_share=0.5):
    """Dense random table over `a` symbols whose last column (a rare symbol in
    the texts) is undefined for about `undef_share` of the states."""
    t = rng.integers(0, q, size=(q, a)).astype(np.int64)
    t[rng.random(q) < undef_share, a - 1] = -1
    return t


def rare_text(rng, alphabet, n, plants):
    text = W.uniform_text(rng, alphabet[:-1], n)
    text[rng.integers(0, n, size=plants)] = alphabet[-1]
    return text


def test_partial_parallel_automaton():
    """Table I with its restart entries undefined: texts built of whole words
    survive until the first broken one; every chunk boundary exercises S."""
    t = TABLE1.astype(np.int64)
    t[t == 0] = -1
    rng = np.random.default_rng(2)
    words = [b"parallel", b"para", b"p", b"paral"]
    for i in range(6):
        parts = [words[int(k)] for k in rng.integers(0, 4, size=40000)]
        if i % 2:
            parts[int(rng.integers(100, 39000))] = b"pl"  # 'l' after 'p' is undefined
        text = np.frombuffer(b"".join(parts), dtype=np.uint8).copy()
        for L in (64, 1024):
            got, _ = partial_case(f"words {i}", t, PAREL, 0, [8], text, L, dtype=np.uint8)
            assert (got.final_state == P.DEAD_STATE) == bool(i % 2)


def test_partial_first_symbol_empties_s():
    """Symbol 'x' is defined only for state 0 and 'y' never leads to 0, so a
    chunk that follows 'y' and starts with 'x' has S intersect L empty: the
    run dies on that chunk's first byte unless it was dead before."""
    q = 6
    t = np.full((q, 3), -1, dtype=np.int64)
    t[:, 0] = (np.arange(q) + 1) % q          # 'a': a cycle
    t[:, 1] = np.where(np.arange(q) == 0, 1, np.arange(q))  # 'y': never to 0
    t[:, 1][t[:, 1] == 0] = 1
    t[0, 2] = 3                                 # 'x': only from 0
    alphabet = b"ayx"
    L = 64
    rng = np.random.default_rng(4)
    text = W.uniform_text(rng, b"a", 64 * 300)
    text[5 * L - 1] = ord("y")
    text[5 * L] = ord("x")
    got, cache = partial_case("empty S", t, alphabet, 0, [2, 3], text, L, dtype=np.uint8)
    assert cache[(1, 2)] == 0
    assert got.final_state == P.DEAD_STATE
    # the same pair inside a chunk (not at a boundary) kills it too
    text2 = W.uniform_text(rng, b"a", 64 * 300)
    text2[5 * L + 9] = ord("y")
    text2[5 * L + 10] = ord("x")
    got, _ = partial_case("y x inside a chunk", t, alphabet, 0, [2, 3], text2, L, dtype=np.uint8)
    assert got.final_state == P.DEAD_STATE
    # 'x' right after 'a' steps from 0 when the cycle is there
    text3 = np.frombuffer(b"a" * 6 * 50 + b"x" + b"a" * 200, dtype=np.uint8).copy()
    partial_case("x from state 0", t, alphabet, 0, [2, 3], text3, 64, dtype=np.uint8)


@pytest.mark.parametrize("layout", ["auto", "byte_lds", "class", "byte_global", "hot"])
def test_partial_random_tables(layout):
    lay = {"auto": P.LAYOUT_AUTO, "byte_lds": P.LAYOUT_BYTE_LDS, "class": P.LAYOUT_CLASS_LDS,
           "byte_global": P.LAYOUT_BYTE_GLOBAL, "hot": P.LAYOUT_HOT_LDS}[layout]
    rng = np.random.default_rng(hash(layout) % 1000)
    dead = 0
    for i, (q, a, n, L) in enumerate([(7, 4, 300_000, 64), (60, 4, 1_000_000, 1024), (100, 20, 500_003, 256),
                                      (900, 20, 2_000_000, 2048), (3000, 4, 1_000_000, 4096), (40, 256, 400_000, 128)]):
        alphabet = bytes(rng.choice(256, size=a, replace=False).astype(np.uint8))
        t = rare_column_dfa(rng, q, a)
        acc = rng.choice(q, size=max(1, q // 8), replace=False)
        text = rare_text(rng, alphabet, n, plants=int(rng.integers(1, 4)))
        got, _ = partial_case(f"{layout} {i}", t, alphabet, int(rng.integers(0, q)), acc, text, L, layout=lay,
                              group=int(rng.choice([4, 8, 16])))
        dead += got.final_state == P.DEAD_STATE
    say(f"[partial] {layout}: {dead} of 6 runs died")


def test_partial_sparse_rows():
    """Partial byte tables in the sparse layout (every byte valid, so the
    keys are the bytes themselves): per state a default of 0, two explicit
    transitions on bytes of a 64-symbol set, and byte 255 undefined for about
    half the states (an exception to the dead state); Zipf text over the 64
    symbols with a few 255s planted. Up to 4095 states (4096 with the dead
    state)."""
    rng = np.random.default_rng(4096)
    symbols = np.sort(rng.choice(255, size=64, replace=False)).astype(np.uint8)
    alphabet = bytes(range(256))
    for q, n, L in [(300, 700_000, 1024), (2000, 2_000_003, 4096), (4095, 4_000_000, 8192)]:
        t = np.zeros((q, 256), dtype=np.int64)
        for s_ in range(q):
            cols = rng.choice(symbols, size=2, replace=False)
            t[s_, cols] = rng.integers(0, q, size=2)
        t[rng.random(q) < 0.5, 255] = -1
        acc = rng.choice(q, size=16, replace=False)
        text = symbols[np.minimum(rng.zipf(1.1, size=n) - 1, 63)].astype(np.uint8)
        text[rng.integers(0, n, size=3)] = 255
        tt = np.where(t < 0, 0xFFFF, t).astype(np.uint16)
        m = P.Matcher(tt, alphabet, 0, acc, partial=True, layout=P.LAYOUT_SPARSE_LDS)
        assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
        m.close()
        for g in (4, 16):
            partial_case(f"sparse rows Q={q} G={g}", t, alphabet, 0, acc, text, L, layout=P.LAYOUT_SPARSE_LDS,
                         group=g)


def test_partial_regex_example():
    """(a|b)?c*[0-3]b+ without its dead state: accepted texts stay alive to
    the end, others die where the total automaton would enter its dead state."""
    t = np.full((4, 7), -1, dtype=np.int64)
    col = {c: i for i, c in enumerate(b"abc0123")}
    t[0, col[ord("a")]] = 1
    t[0, col[ord("b")]] = 1
    for s in (0, 1):
        t[s, col[ord("c")]] = 1
        for d in b"0123":
            t[s, col[d]] = 2
    t[2, col[ord("b")]] = 3
    t[3, col[ord("b")]] = 3
    for text in (b"a" + b"c" * 100000 + b"2" + b"b" * 300000, b"c" * 5000 + b"1" + b"b" * 70000 + b"a",
                 b"b" * 100 + b"c" * 100000):
        arr = np.frombuffer(text, dtype=np.uint8).copy()
        got, _ = partial_case("regex", t, b"abc0123", 0, [3], arr, 1024, dtype=np.uint8)


def test_partial_invalid_byte_after_death():
    t = np.array([[1, -1], [0, 1]], dtype=np.int64)
    text = np.frombuffer(b"ab" * 5000 + b"abab" + b"b" * 3000 + b"z" + b"a" * 100, dtype=np.uint8).copy()
    tt = np.where(t < 0, 255, t).astype(np.uint8)
    m = P.Matcher(tt, b"ab", 0, [1], chunk_len=64, partial=True)
    with pytest.raises(P.ParemError) as ei:
        m.match(dev(text))
    assert ei.value.status == P.PAREM_ESYMBOL
    m.close()


def test_partial_boundary_states():
    rng = np.random.default_rng(9)
    alphabet = b"ACGTN"
    t = rare_column_dfa(rng, 50, 5)
    text = rare_text(rng, alphabet, 400_000, plants=2)
    tt = np.where(t < 0, 0xFFFF, t).astype(np.uint16)
    m = P.Matcher(tt, alphabet, 0, [3, 7], partial=True)
    for L in (64, 1024):
        got = P.boundary_states(m, dev(text), L).cpu().numpy().view(np.uint32)
        pos = np.arange(0, text.size, L, dtype=np.uint64)
        want, _ = oracle.states_at(t, alphabet, 0, [3, 7], text, pos, partial=True)
        want = np.where(want == oracle.DEAD, P.DEAD_STATE, want).astype(np.uint32)
        assert np.array_equal(got, want)
    m.close()


def test_policy_errors():
    t = np.array([[1, 255], [0, 1]], dtype=np.uint8)
    with pytest.raises(P.ParemError) as ei:
        P.Matcher(t, b"ab", 0, [1])  # 255 is not a state of a total table
    assert ei.value.status == P.PAREM_ESTATE
    for kw in ({"partial": True, "policy": P.POLICY_ENUMERATE}, {"partial": True, "lookback": 8},
               {"policy": P.POLICY_ENUMERATE, "lookback": 8}, {"policy": 2}):
        with pytest.raises(P.ParemError) as ei:
            P.Matcher(t if kw.get("partial") else np.array([[1, 0], [0, 1]], dtype=np.uint8), b"ab", 0, [1], **kw)
        assert ei.value.status == P.PAREM_EINVAL, kw
    m = P.Matcher(t, b"ab", 0, [1], partial=True)
    with pytest.raises(P.ParemError) as ei:
        P.Proposal(m, np.zeros(P.proposal_param_count(2), dtype=np.float32))
    assert ei.value.status == P.PAREM_EUNSUPPORTED
    with pytest.raises(P.ParemError) as ei:
        P.Batch([m], [128])
    assert ei.value.status == P.PAREM_EUNSUPPORTED
    m.close()
