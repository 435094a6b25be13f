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
    dfa, text = W.dna_motif(seed, n=1 << 21, copies=2000)
    motif, wild = dfa.meta["motif"], dfa.meta["wild"]
    r = oracle.walk_dfa(dfa, text)
    want = brute_force_motif_count(text, motif, wild)
    assert want >= 1000
    assert r.count == want
    assert 17 <= dfa.num_states <= 64


def test_motif_dfa_final_state_tracks_suffix():
    """The motif automaton's state depends only on the last 16 symbols: two
    texts with the same 16-symbol suffix end in the same state."""
    dfa = W.dna_motif_dfa(2)
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
    dfa, text = W.dna_motif()
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


# ---------------------------------------------------------------------------
# the Enumeration policy (Section II-C's run counts, Section IV-A)
# ---------------------------------------------------------------------------

def test_enumeration_runs_on_the_example(golden_dir):
    """Enumeration speculates all nine states for each unit after the first:
    3 * 9 + 1 = 28 walks on the worked example (Section II-C), against the
    six of Algorithm 1's rule; both reach the sequential result."""
    t1 = load_table1(golden_dir)
    enum = oracle.parem(t1, PAREL, 0, [8], EXAMPLE, p=4, policy=oracle.POLICY_ENUMERATE, traces=True)
    assert enum.runs == 28
    assert enum.rsize.tolist() == [1, 9, 9, 9]
    plain = oracle.parem(t1, PAREL, 0, [8], EXAMPLE, p=4)
    assert plain.runs == 6
    seq = oracle.walk(t1, PAREL, 0, [8], EXAMPLE)
    for r in (enum, plain):
        assert (r.final_state, r.count) == (seq.final_state, seq.count) == (0, 1)
    # the enumeration's walks of Table II's starts visit the printed states
    walks = {(c, r): v for c, r, v in enum.traces}
    for unit, start, visits in load_table2(golden_dir):
        assert walks[(unit, start)] == visits, (unit, start)


def test_enumeration_vs_parem_worst_case(golden_dir):
    """Every unit's predecessor ending in 'l' (four destinations): 13 walks
    against Enumeration's 28, the 2.15x of Section II-C, from two runs."""
    t1 = load_table1(golden_dir)
    text = b"paral" + b"l" + b"parall" + b"eparal" + b"pppppp"
    plain = oracle.parem(t1, PAREL, 0, [8], text, p=4)
    enum = oracle.parem(t1, PAREL, 0, [8], text, p=4, policy=oracle.POLICY_ENUMERATE)
    assert (plain.runs, enum.runs) == (13, 28)
    assert round(enum.runs / plain.runs, 2) == 2.15
    assert (plain.final_state, plain.count) == (enum.final_state, enum.count)


def test_enumeration_equals_sequential_for_any_split():
    rng = np.random.default_rng(41)
    for _ in range(20):
        dfa, text = W.random_case(rng, max_states=20, max_alpha=5, max_len=400)
        seq = oracle.walk_dfa(dfa, text)
        for p in (1, 2, 3, 7, max(1, text.size)):
            r = oracle.parem(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, p=p,
                             policy=oracle.POLICY_ENUMERATE)
            assert (r.final_state, r.count) == (seq.final_state, seq.count)
            # every slice after the first walks every state
            slices = [int((c + 1) * text.size // p) - int(c * text.size // p) for c in range(p)]
            assert r.runs == 1 + (p - 1) * dfa.num_states, slices


# ---------------------------------------------------------------------------
# partial DFAs: undefined transitions, the S set, the DEAD result
# ---------------------------------------------------------------------------

def partial_table1(golden_dir):
    """Table I with its restart entries (state 0) left undefined: a run dies
    on any symbol that does not extend the word or start it again."""
    t1 = load_table1(golden_dir).astype(np.int64)
    t1[t1 == 0] = -1
    return t1


def test_partial_example_dies_early(golden_dir):
    """Worked by hand from Table I: the run reads 'p' (state 1) and dies on
    'l'. Algorithm 1 with four units: unit 1 follows 'p' (L = {1}) and starts
    with 'a' (S = {1, 3}): R = {1}; unit 2 follows 'e' (L = {7}) and starts
    with 'l' (S = {4, 5, 7}): R = {7}, whose walk reaches 8 (one count) and
    dies on 'a'; unit 3: L = {7}, S = every state ('p'): R = {7}."""
    t = partial_table1(golden_dir)
    seq = oracle.walk(t, PAREL, 0, [8], EXAMPLE, partial=True)
    assert (seq.final_state, seq.accept, seq.count) == (oracle.DEAD, False, 0)
    r = oracle.parem(t, PAREL, 0, [8], EXAMPLE, p=4, partial=True, traces=True)
    assert (r.final_state, r.accept, r.count) == (oracle.DEAD, False, 0)
    assert r.rsize.tolist() == [1, 1, 1, 1]
    assert r.entries.tolist() == [0, oracle.DEAD, oracle.DEAD, oracle.DEAD]
    walks = {(c, s): v for c, s, v in r.traces}
    D = oracle.DEAD
    assert walks[(0, 0)] == [1, D, D, D, D, D]
    assert walks[(1, 1)] == [2, 3, 4, 5, 6, 7]
    assert walks[(2, 7)] == [8, D, D, D, D, D]
    assert walks[(3, 7)] == [1, 2, 3, 4, 1, D]


def test_partial_first_symbol_empties_s(golden_dir):
    """"parall" then "aaaaaa", two units: unit 1 follows 'l' (L = {5, 6, 8})
    and starts with 'a' (S = {1, 3}): R is empty, and the route (state 6)
    dies on the unit's first symbol. "para" then "llel": R = {4}, whose walk
    ends the word (accept, one count)."""
    t = partial_table1(golden_dir)
    r = oracle.parem(t, PAREL, 0, [8], b"paralla" + b"aaaaa", p=2, partial=True)
    assert r.rsize.tolist() == [1, 0]
    assert (r.final_state, r.count, r.runs) == (oracle.DEAD, 0, 1)
    assert r.entries.tolist() == [0, 6]
    r = oracle.parem(t, PAREL, 0, [8], b"parallel", p=2, partial=True)
    assert r.rsize.tolist() == [1, 1]
    assert (r.final_state, r.accept, r.count, r.runs) == (8, True, 1, 2)


def test_partial_equals_total_with_a_dead_state():
    """The regular-expression example without its dead state 4: undefined
    transitions give DEAD exactly where the total automaton enters state 4,
    the same count, and acceptance equals Python's re.fullmatch on every
    string of up to five symbols; Algorithm 1 on the partial table agrees for
    every split."""
    t = regex_dfa()
    part = t[:4].astype(np.int64)
    part[part == 4] = -1
    pat = re.compile(r"(a|b)?c*[0-3]b+")
    syms = [bytes([c]) for c in RE_ALPHA]
    for length in range(0, 6):
        for tup in itertools.product(syms, repeat=length):
            s = b"".join(tup)
            full = oracle.walk(t, RE_ALPHA, 0, [3], s)
            r = oracle.walk(part, RE_ALPHA, 0, [3], s, partial=True)
            assert r.count == full.count, s
            assert (r.final_state == oracle.DEAD) == (full.final_state == 4), s
            assert r.accept == bool(pat.fullmatch(s.decode())), s
            if 0 < length and length % 2:
                for p in range(1, length + 1):
                    a = oracle.parem(part, RE_ALPHA, 0, [3], s, p=p, partial=True)
                    assert (a.final_state, a.count) == (r.final_state, r.count), (s, p)


def test_partial_random_any_split():
    """Random partial tables (a quarter of the transitions undefined): the
    result of Algorithm 1 with the S filter equals the sequential run for
    every split, and never walks more states than its total completion (an
    absorbing non-final state for every undefined entry) would."""
    rng = np.random.default_rng(5)
    for _ in range(40):
        q = int(rng.integers(1, 12))
        a = int(rng.integers(1, 5))
        alpha = bytes(rng.choice(np.arange(97, 123), size=a, replace=False).astype(np.uint8))
        t = rng.integers(0, q, size=(q, a)).astype(np.int64)
        t[rng.random((q, a)) < 0.25] = -1
        acc = rng.choice(q, size=int(rng.integers(0, q + 1)), replace=False)
        text = np.frombuffer(alpha, dtype=np.uint8)[rng.integers(0, a, size=int(rng.integers(0, 60)))]
        comp = np.where(t < 0, q, t)
        comp = np.vstack([comp, np.full((1, a), q)])
        seq = oracle.walk(t, alpha, 0, acc, text, partial=True)
        tot = oracle.walk(comp, alpha, 0, acc, text)
        assert seq.count == tot.count
        assert (seq.final_state == oracle.DEAD) == (tot.final_state == q)
        for p in (1, 2, 3, 5, max(1, text.size)):
            r = oracle.parem(t, alpha, 0, acc, text, p=p, partial=True)
            assert (r.final_state, r.count) == (seq.final_state, seq.count)
            rc = oracle.parem(comp, alpha, 0, acc, text, p=p)
            assert r.runs <= rc.runs


def test_partial_errors():
    t = np.array([[1, -1], [0, 1]], dtype=np.int64)
    # undefined entries need the flag
    with pytest.raises(oracle.OracleError) as ei:
        oracle.walk(t, b"ab", 0, [1], b"ab")
    assert ei.value.code == oracle.ESTATE
    # a byte outside the alphabet is reported even after the run died
    with pytest.raises(oracle.OracleError) as ei:
        oracle.walk(t, b"ab", 0, [1], b"abbbxa", partial=True)
    assert ei.value.code == oracle.ESYMBOL and ei.value.bad_pos == 4
    r = oracle.walk(t, b"ab", 0, [1], b"abab", partial=True)  # 0 -a-> 1 -b-> 1 -a-> 0 -b-> dead
    assert (r.final_state, r.count) == (oracle.DEAD, 2)
    st, cn = oracle.states_at(t, b"ab", 0, [1], b"abab", [0, 1, 3, 4], partial=True)
    assert st.tolist() == [0, 1, 0, oracle.DEAD] and cn.tolist() == [0, 1, 2, 2]


# ---------------------------------------------------------------------------
# match positions (the steps that enter a final state)
# ---------------------------------------------------------------------------

def test_positions_of_the_example(golden_dir):
    t1 = load_table1(golden_dir)
    pos, total = oracle.positions(t1, PAREL, 0, [8], EXAMPLE)
    assert total == 1 and pos.tolist() == [EXAMPLE.index(b"parallel") + 7] == [12]


def test_positions_are_word_ends():
    """The KMP automaton enters state 8 exactly at the last symbol of every
    occurrence of "parallel" (overlaps included); random texts with planted
    copies; the cap keeps the first offsets and the total."""
    t1 = kmp_automaton(b"parallel", PAREL)
    rng = np.random.default_rng(9)
    for _ in range(10):
        text = bytearray(np.frombuffer(PAREL, dtype=np.uint8)[rng.integers(0, 5, size=5000)].tobytes())
        for o in rng.integers(0, 5000 - 8, size=30):
            text[o:o + 8] = b"parallel"
        text = bytes(text)
        want = [i + 7 for i in range(len(text) - 7) if text[i:i + 8] == b"parallel"]
        pos, total = oracle.positions(t1, PAREL, 0, [8], text)
        assert pos.tolist() == want and total == len(want)
        pos, total = oracle.positions(t1, PAREL, 0, [8], text, cap=5)
        assert pos.tolist() == want[:5] and total == len(want)


def test_positions_of_the_regex_example():
    """Offsets i whose prefix t[0..i] is in the language of
    (a|b)?c*[0-3]b+ (Python's re.fullmatch), partial and total forms."""
    t = regex_dfa()
    part = t[:4].astype(np.int64)
    part[part == 4] = -1
    pat = re.compile(r"(a|b)?c*[0-3]b+")
    rng = np.random.default_rng(3)
    for _ in range(200):
        s = bytes(np.frombuffer(RE_ALPHA, dtype=np.uint8)[rng.choice(7, size=int(rng.integers(0, 12)),
                                                                       p=[.1, .1, .2, .1, .1, .1, .3])])
        want = [i for i in range(len(s)) if pat.fullmatch(s[:i + 1].decode())]
        assert oracle.positions(t, RE_ALPHA, 0, [3], s)[0].tolist() == want
        assert oracle.positions(part, RE_ALPHA, 0, [3], s, partial=True)[0].tolist() == want


def test_positions_of_the_motif_automaton():
    dfa, text = W.dna_motif(seed=7, n=1 << 20, copies=300)
    motif, wild = dfa.meta["motif"], dfa.meta["wild"]
    m = len(motif)
    n = text.size - m + 1
    ok = np.ones(n, dtype=bool)
    for k in range(m):
        if not wild[k]:
            ok &= text[k:k + n] == motif[k]
    want = np.flatnonzero(ok) + m - 1
    pos, total = oracle.positions_dfa(dfa, text)
    assert total == want.size and np.array_equal(pos, want.astype(np.uint64))
