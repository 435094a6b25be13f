"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's loop: each compares it with something
independent of it (values printed in the paper, a textbook construction,
Python's regular-expression engine, a sliding-window brute force, the
matrix-product formulation of a DFA run, or Algorithm 1's own invariants).
"""
import itertools
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W


# ---------------------------------------------------------------------------
# the worked example of Section II-C
# ---------------------------------------------------------------------------

PAREL = b"parel"
EXAMPLE = b"plaraparallelapareparapl"


def load_table1(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "table1_parallel.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.asarray(rows, dtype=np.uint32)


def kmp_automaton(pattern: bytes, alphabet: bytes) -> np.ndarray:
    """Textbook string-matching automaton (Knuth-Morris-Pratt failure
    function): state j = length of the longest prefix of the pattern that is
    a suffix of the text read; after a full match, continue from the failure
    of the whole pattern."""
    m = len(pattern)
    fail = [0] * (m + 1)
    k = 0
    for i in range(1, m):
        while k and pattern[i] != pattern[k]:
            k = fail[k]
        if pattern[i] == pattern[k]:
            k += 1
        fail[i + 1] = k
    table = np.zeros((m + 1, len(alphabet)), dtype=np.uint32)
    for j in range(m + 1):
        for ci, c in enumerate(alphabet):
            k = j
            if k == m:
                k = fail[m]
            while k and pattern[k] != c:
                k = fail[k]
            table[j, ci] = k + 1 if pattern[k] == c else 0
    return table


def test_table1_is_the_kmp_automaton(golden_dir):
    t1 = load_table1(golden_dir)
    assert t1.shape == (9, 5)
    assert np.array_equal(t1, kmp_automaton(b"parallel", PAREL))


def test_example_sequential_run(golden_dir):
    t1 = load_table1(golden_dir)
    r = oracle.walk(t1, PAREL, 0, [8], EXAMPLE)
    # one occurrence of the word, ending at offset 12; the text ends in
    # "...parapl": last symbol 'l' from state 1 goes to 0
    assert r.count == EXAMPLE.count(b"parallel") == 1
    assert r.final_state == 0 and not r.accept


def load_table2(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "table2_visits.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                head, vis = line.split(":")
                unit, start = (int(v) for v in head.split())
                rows.append((unit, start, [int(v) for v in vis.split()]))
    return rows


def test_example_table2_visits(golden_dir):
    t1 = load_table1(golden_dir)
    res = oracle.parem(t1, PAREL, 0, [8], EXAMPLE, p=4, traces=True)
    walks = {(c, r): v for c, r, v in res.traces}
    for unit, start, visits in load_table2(golden_dir):
        assert walks[(unit, start)] == visits, (unit, start)
    # the stated rule speculates {0, 7} for the fourth unit (previous slice
    # "lapare" ends in 'e'); Table II prints only 0. Both walks coincide.
    assert sorted(r for c, r in walks if c == 3) == [0, 7]
    assert walks[(3, 0)] == walks[(3, 7)]
    # speculated sets of units 1..3: L('p') = {1}, L('e') = {0, 7}, L('e')
    assert res.rsize.tolist() == [1, 1, 2, 2]
    assert res.runs == 6  # five distinct walks once the two identical ones merge
    assert res.entries.tolist() == [0, 1, 7, 0]
    assert (res.final_state, res.count) == (0, 1)


def test_example_candidate_images(golden_dir):
    """Per-symbol images quoted in Section II-C: the destinations on 'l' are
    {0, 5, 6, 8} (four), on 'e' {0, 7}; S is every state (total table)."""
    t1 = load_table1(golden_dir)
    images = {chr(PAREL[j]): sorted(set(t1[:, j].tolist())) for j in range(5)}
    assert images == {"p": [1], "a": [0, 2, 4], "r": [0, 3], "e": [0, 7], "l": [0, 5, 6, 8]}
    # the oracle's |R| for a slice after each symbol
    for sym, img in images.items():
        text = (b"p" * 5 + sym.encode()) + b"pppppp"
        res = oracle.parem(t1, PAREL, 0, [8], text, p=2)
        assert res.rsize[1] == len(img)


def test_example_worst_case_counts(golden_dir):
    """Every slice's predecessor ending in 'l': 3*4+1 = 13 walks versus
    3*9+1 = 28 for enumeration of all states, ratio 2.15."""
    t1 = load_table1(golden_dir)
    text = b"paral" + b"l" + b"parall" + b"eparal" + b"pppppp"
    assert len(text) == 24
    res = oracle.parem(t1, PAREL, 0, [8], text, p=4)
    assert res.runs == 13
    enum = 3 * t1.shape[0] + 1
    assert enum == 28
    assert round(enum / res.runs, 2) == 2.15
    seq = oracle.walk(t1, PAREL, 0, [8], text)
    assert (res.final_state, res.count) == (seq.final_state, seq.count)


# ---------------------------------------------------------------------------
# the second example expression of Section III: (a|b)?c*[0..3]b+
# ---------------------------------------------------------------------------

RE_ALPHA = b"abc0123"


def regex_dfa():
    """Hand-built minimal DFA for (a|b)?c*[0-3]b+ over a,b,c,0..3.
    States: 0 start, 1 after the optional a|b or inside c*, 2 after the
    digit, 3 inside b+ (final), 4 dead."""
    t = np.full((5, 7), 4, dtype=np.uint32)
    col = {c: i for i, c in enumerate(RE_ALPHA)}
    for s in (0,):
        t[s, col[ord("a")]] = 1
        t[s, col[ord("b")]] = 1
    for s in (0, 1):
        t[s, col[ord("c")]] = 1
        for d in b"0123":
            t[s, col[d]] = 2
    t[2, col[ord("b")]] = 3
    t[3, col[ord("b")]] = 3
    return t


def test_regex_example_against_python_re():
    t = regex_dfa()
    pat = re.compile(r"(a|b)?c*[0-3]b+")
    syms = [bytes([c]) for c in RE_ALPHA]
    n = 0
    for length in range(0, 6):
        for tup in itertools.product(syms, repeat=length):
            s = b"".join(tup)
            r = oracle.walk(t, RE_ALPHA, 0, [3], s)
            assert r.accept == bool(pat.fullmatch(s.decode())), s
            want = sum(1 for i in range(1, len(s) + 1) if pat.fullmatch(s[:i].decode()))
            assert r.count == want, s
            n += 1
    assert n == sum(7 ** k for k in range(6))


def test_regex_example_random_long():
    t = regex_dfa()
    pat = re.compile(r"(a|b)?c*[0-3]b+")
    rng = np.random.default_rng(11)
    alpha = np.frombuffer(RE_ALPHA, dtype=np.uint8)
    for _ in range(300):
        # bias towards the language's shape so that accepts occur
        parts = [b"" if rng.random() < 0.5 else bytes([RE_ALPHA[rng.integers(0, 2)]]),
                 b"c" * int(rng.integers(0, 4)),
                 bytes([RE_ALPHA[3 + rng.integers(0, 4)]]),
                 b"b" * int(rng.integers(0, 5))]
        s = b"".join(parts)
        if rng.random() < 0.3:
            k = int(rng.integers(0, len(s)))
            s = s[:k] + bytes([alpha[rng.integers(0, 7)]]) + s[k + 1:]
        r = oracle.walk(t, RE_ALPHA, 0, [3], s)
        assert r.accept == bool(pat.fullmatch(s.decode())), s


# ---------------------------------------------------------------------------
# the DNA motif workload: Sigma*.P search automaton
# ---------------------------------------------------------------------------

def brute_force_motif_count(text: np.ndarray, motif: bytes, wild: np.ndarray) -> int:
    m = len(motif)
    n = text.size - m + 1
    if n <= 0:
        return 0
    ok = np.ones(n, dtype=bool)
    for k in range(m):
        if not wild[k]:
            ok &= text[k:k + n] == motif[k]
    return int(ok.sum())


@pytest.mark.parametrize("seed", [2, 7, 19, 23])
def test_motif_count_equals_sliding_compare(seed):
    dfa, text = W.config2(seed, n=1 << 21, copies=2000)
    motif, wild = dfa.meta["motif"], dfa.meta["wild"]
    r = oracle.walk_dfa(dfa, text)
    want = brute_force_motif_count(text, motif, wild)
    assert want >= 1000
    assert r.count == want
    assert 17 <= dfa.num_states <= 64


def test_motif_dfa_final_state_tracks_suffix():
    """The motif automaton's state depends only on the last 16 symbols: two
    texts with the same 16-symbol suffix end in the same state."""
    dfa = W.config2_dfa(2)
    rng = np.random.default_rng(5)
    suffix = W.uniform_text(rng, W.ACGT, 16)
    ends = set()
    for _ in range(20):
        pre = W.uniform_text(rng, W.ACGT, int(rng.integers(0, 200)))
        ends.add(oracle.walk_dfa(dfa, np.concatenate([pre, suffix])).final_state)
    assert len(ends) == 1


# ---------------------------------------------------------------------------
# matrix-product formulation (a DFA run as products of 0/1 matrices)
# ---------------------------------------------------------------------------

def test_matrix_product_formulation():
    rng = np.random.default_rng(3)
    for _ in range(60):
        dfa, text = W.random_case(rng, max_states=12, max_alpha=5, max_len=64)
        q, a = dfa.table.shape
        mats = np.zeros((a, q, q), dtype=np.int64)
        for s in range(q):
            for j in range(a):
                mats[j, s, dfa.table[s, j]] = 1
        col = {c: j for j, c in enumerate(dfa.alphabet)}
        f = dfa.final_mask().astype(np.int64)
        v = np.zeros(q, dtype=np.int64)
        v[dfa.start] = 1
        count = 0
        for byte in text.tolist():
            v = v @ mats[col[byte]]
            count += int(v @ f)
        r = oracle.walk_dfa(dfa, text)
        assert v.sum() == 1
        assert r.final_state == int(np.argmax(v))
        assert r.count == count
        assert r.accept == bool(f[r.final_state])


# ---------------------------------------------------------------------------
# Algorithm 1 invariants and edge cases
# ---------------------------------------------------------------------------

def test_parem_independent_of_slice_count():
    rng = np.random.default_rng(9)
    for _ in range(40):
        dfa, text = W.random_case(rng, max_states=20, max_alpha=6, max_len=200)
        seq = oracle.walk_dfa(dfa, text)
        for p in sorted({1, 2, 3, 7, max(1, text.size), text.size + 3}):
            res = oracle.parem(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, p)
            assert (res.final_state, res.count) == (seq.final_state, seq.count)
            # each slice's true entry was among its speculated states (no
            # join failure), and |R| never exceeds the column image size
            assert res.rsize[0] == 1
            assert np.all(res.rsize <= dfa.num_states)


def test_states_at_matches_prefix_runs():
    rng = np.random.default_rng(4)
    dfa, text = W.random_case(rng, max_states=30, max_alpha=4, max_len=500)
    pos = np.sort(rng.integers(0, text.size + 1, size=20))
    st, cn = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, pos)
    for k, p in enumerate(pos):
        r = oracle.walk_dfa(dfa, text[:p])
        assert (st[k], cn[k]) == (r.final_state, r.count)


def test_edge_cases():
    t = np.asarray([[1, 0], [1, 1]], dtype=np.uint32)
    # empty text: start state, its membership in F, count 0
    r = oracle.walk(t, b"xy", 1, [1], b"")
    assert (r.final_state, r.accept, r.count) == (1, True, 0)
    # start state final but never counted itself
    r = oracle.walk(t, b"xy", 1, [1], b"x")
    assert (r.final_state, r.count) == (1, 1)
    r = oracle.walk(t, b"xy", 0, [1], b"y")
    assert (r.final_state, r.accept, r.count) == (0, False, 0)
    # a byte outside the alphabet
    with pytest.raises(oracle.OracleError) as ei:
        oracle.walk(t, b"xy", 0, [1], b"xxyzx")
    assert ei.value.code == oracle.ESYMBOL and ei.value.bad_pos == 3
    # an entry outside [0, Q)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.walk(np.asarray([[0, 2], [1, 1]]), b"xy", 0, [1], b"x")
    assert ei.value.code == oracle.ESTATE
    # start outside [0, Q)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.walk(t, b"xy", 2, [1], b"x")
    assert ei.value.code == oracle.ESTATE
    # the same byte named twice in the alphabet
    with pytest.raises(oracle.OracleError) as ei:
        oracle.walk(t, b"xx", 0, [1], b"x")
    assert ei.value.code == oracle.EINVAL
    # a one-state automaton with every step final
    r = oracle.walk(np.zeros((1, 3), dtype=np.uint32), b"abc", 0, [0], b"abcabc")
    assert (r.final_state, r.accept, r.count) == (0, True, 6)


def test_count_is_u64_wide():
    """A count of 2^32 + 17: a one-state automaton whose state is final makes
    every step count, so the count equals the text length by arithmetic
    alone; the oracle must not wrap it at 32 bits."""
    n = (1 << 32) + 17
    t = np.zeros((1, 1), dtype=np.uint32)
    text = np.full(n, ord("a"), dtype=np.uint8)
    r = oracle.walk(t, b"a", 0, [0], text)
    assert (r.final_state, r.accept, r.count) == (0, True, n)
    del text
    short = np.full(1 << 20, ord("a"), dtype=np.uint8)
    st, cn = oracle.states_at(t, b"a", 0, [0], short, [0, 1 << 19, 1 << 20])
    assert cn.dtype == np.uint64 and cn.tolist() == [0, 1 << 19, 1 << 20]


def test_permutation_automaton_closed_form():
    """delta(s, k-th symbol) = (s + k + 1) mod 7 never synchronises; its
    final state is the start plus the sum of (k + 1) over the text, mod 7,
    and with every state final the count is the length."""
    q = 7
    table = np.stack([(np.arange(q) + k + 1) % q for k in range(3)], axis=1).astype(np.uint32)
    rng = np.random.default_rng(5)
    text = W.uniform_text(rng, b"abc", 1_000_003)
    k = np.frombuffer(b"abc", dtype=np.uint8)
    total = sum((j + 1) * int(np.count_nonzero(text == k[j])) for j in range(3))
    r = oracle.walk(table, b"abc", 2, np.arange(q), text)
    assert (r.final_state, r.accept, r.count) == ((2 + total) % q, True, text.size)
    r = oracle.walk(table, b"abc", 2, [4], text)
    assert r.final_state == (2 + total) % q


def test_motif_count_full_size_equals_sliding_compare():
    """The benchmarked 1 GiB DNA text (default seed, 1e5 planted copies):
    the oracle's count equals the sliding-window compare at the motif's 12
    fixed positions over the whole text, taken in 64 MiB blocks that overlap
    by the motif length minus one."""
    dfa, text = W.config2()
    assert text.size == 1 << 30
    motif, wild = dfa.meta["motif"], dfa.meta["wild"]
    m = len(motif)
    block = 1 << 26
    want = 0
    for lo in range(0, text.size, block):
        want += brute_force_motif_count(text[lo:min(text.size, lo + block + m - 1)], motif, wild)
    assert want >= 100000 - 100
    r = oracle.walk_dfa(dfa, text)
    assert r.count == want
