"""GPU parity of the plain speculative walk against the CPU oracle.

Bit-exact on (final state, accept flag, count) for every case, plus the
number of speculated walks, which the test derives from the definition of
the speculated set (the image of the column of the byte before each chunk;
{q0} for the first chunk).
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


def expected_spec_runs(dfa, text, L):
    n = text.size
    if n == 0:
        return 0
    chunks = (n + L - 1) // L
    col = np.full(256, -1, dtype=np.int64)
    col[np.frombuffer(dfa.alphabet, dtype=np.uint8)] = np.arange(dfa.alphabet_size)
    img = np.asarray([np.unique(dfa.table[:, j]).size for j in range(dfa.alphabet_size)], dtype=np.int64)
    prev = text[np.arange(1, chunks, dtype=np.int64) * L - 1]
    cols = col[prev]
    sizes = np.where(cols >= 0, img[np.maximum(cols, 0)], 1)
    return 1 + int(sizes.sum())


def run_case(name, dfa, text, offset=0, check_spec=True, **opts):
    say(f"[case] {name}: Q={dfa.num_states} A={dfa.alphabet_size} n={text.size} opts={opts} off={offset}")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, **opts)
    try:
        buf = torch.empty(text.size + offset + 16, dtype=torch.uint8, device="cuda")
        dev = buf[offset:offset + text.size]
        if text.size:
            dev.copy_(torch.from_numpy(text))
        want = oracle.walk_dfa(dfa, text)
        got = m.match(dev)
        assert (got.final_state, got.accept, got.count) == (want.final_state, want.accept, want.count), name
        L = opts.get("chunk_len") or None
        if L is not None and check_spec:
            assert got.chunks == (text.size + L - 1) // L
            assert got.spec_runs == expected_spec_runs(dfa, text, L)
        assert got.rerun_chunks == 0
        return got
    finally:
        m.close()


def test_worked_example():
    t1 = np.asarray([[1, 0, 0, 0, 0], [1, 2, 0, 0, 0], [1, 0, 3, 0, 0], [1, 4, 0, 0, 0], [1, 0, 0, 0, 5],
                     [1, 0, 0, 0, 6], [1, 0, 0, 7, 0], [1, 0, 0, 0, 8], [1, 0, 0, 0, 0]], dtype=np.uint8)
    dfa = W.Dfa(t1, b"parel", 0, np.asarray([8], dtype=np.uint32))
    text = np.frombuffer(b"plaraparallelapareparapl" * 1000, dtype=np.uint8).copy()
    for L in (64, 128, 4096):
        run_case(f"example L={L}", dfa, text, chunk_len=L)


def test_random8_full():
    dfa, text, chunks = W.random8()
    got = run_case("random8", dfa, text, chunk_len=text.size // chunks)
    assert got.chunks == 1024
    ref = oracle.parem(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, chunks)
    assert got.spec_runs == ref.runs


@pytest.mark.parametrize("group", [2, 4, 8, 16])
def test_dna_motif_small_groups(group):
    dfa, text = W.dna_motif(n=4 << 20)
    run_case(f"dna_motif 4MiB G={group}", dfa, text, chunk_len=1024, group=group)



def all_layouts():
    return [P.LAYOUT_AUTO, P.LAYOUT_KGRAM_LDS, P.LAYOUT_BYTE_LDS, P.LAYOUT_BYTE_GLOBAL, P.LAYOUT_HOT_LDS,
            P.LAYOUT_CLASS_LDS]


def test_dna_motif_layouts():
    dfa, text = W.dna_motif(n=1 << 22)
    for lay in all_layouts():
        for g in (4, 16):
            run_case(f"dna_motif layout={lay} G={g}", dfa, text, chunk_len=2048, layout=lay, group=g)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    assert m.describe()["layout"] == P.LAYOUT_KGRAM_LDS and m.describe()["kgram"] == 4
    m.close()


@pytest.mark.parametrize("alphabet,kgram", [(b"ab", 4), (b"AC", 4), (b"ACG", 4), (b"01234", 2),
                                             (b"01234567", 2), (b"@ABCDEFG", 2), (b"xyz", 4)])
def test_kgram_code_widths(alphabet, kgram):
    rng = np.random.default_rng(len(alphabet) * 7 + alphabet[0])
    dfa = W.random_dense_dfa(rng, 23, alphabet, num_accepting=5)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, layout=P.LAYOUT_KGRAM_LDS)
    d = m.describe()
    m.close()
    assert d["layout"] == P.LAYOUT_KGRAM_LDS and d["kgram"] == kgram, d
    for n in (0, 5, 64, 1000, 65536 + 13):
        text = W.uniform_text(rng, alphabet, n)
        for off in (0, 5):
            run_case(f"kgram {alphabet} n={n}", dfa, text, offset=off, chunk_len=128,
                     layout=P.LAYOUT_KGRAM_LDS, group=4)


def test_kgram_invalid_bytes():
    rng = np.random.default_rng(8)
    dfa = W.random_dense_dfa(rng, 9, b"ACGT", num_accepting=2)
    base = W.uniform_text(rng, b"ACGT", 8192 + 5)
    # bytes that share a symbol code with a valid byte must still be rejected
    for pos, bad in ((0, ord("a")), (100, ord("E")), (4095, ord("V")), (8192 + 4, ord("c")), (4096, 0)):
        text = base.copy()
        text[pos] = bad
        m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=64,
                      layout=P.LAYOUT_KGRAM_LDS)
        say(f"[case] kgram invalid byte {bad} at {pos}")
        with pytest.raises(P.ParemError) as ei:
            m.match(torch.from_numpy(text).cuda())
        assert ei.value.status == P.PAREM_ESYMBOL
        m.close()


@pytest.mark.parametrize("tile", [64, 128])
def test_dna_motif_no_merge(tile):
    """The paper's plain scheme: every speculated run walks its whole chunk."""
    dfa, text = W.dna_motif(n=1 << 22)
    for g in (4, 16):
        run_case(f"dna_motif no-merge G={g} tile={tile}", dfa, text, chunk_len=4096, group=g, no_merge=True,
                 tile=tile)


def test_dna_motif_full_size():
    dfa, text = W.dna_motif()
    got = run_case("dna_motif 1GiB", dfa, text)
    assert got.chunks >= 1024


@pytest.mark.parametrize("n", [0, 1, 2, 15, 16, 17, 63, 64, 65, 127, 1000, 4095, 4097, 65536 + 7])
def test_ragged_and_tiny(n):
    rng = np.random.default_rng(n)
    dfa = W.random_dense_dfa(rng, 13, b"xyz", num_accepting=4)
    text = W.uniform_text(rng, b"xyz", n)
    for off in (0, 3):
        run_case(f"tiny n={n}", dfa, text, offset=off, chunk_len=64)


def test_start_final_and_empty():
    t = np.asarray([[1, 0], [1, 1]], dtype=np.uint8)
    dfa = W.Dfa(t, b"ab", 1, np.asarray([1], dtype=np.uint32))
    run_case("start-final empty", dfa, np.zeros(0, dtype=np.uint8))
    run_case("start-final", dfa, np.frombuffer(b"ab" * 100, dtype=np.uint8).copy(), chunk_len=64)


def test_random_fuzz():
    rng = np.random.default_rng(1234)
    for i in range(60):
        dfa, text = W.random_case(rng, max_states=100, max_alpha=12, max_len=20000)
        L = int(rng.choice([64, 128, 256, 1024]))
        g = int(rng.choice([2, 4, 8, 16]))
        off = int(rng.integers(0, 16))
        lay = int(rng.choice(all_layouts()))
        nm = bool(rng.integers(0, 2))
        tile = int(rng.choice([0, 64, 128]))
        run_case(f"fuzz {i}", dfa, text, offset=off, chunk_len=L, group=g, layout=lay, no_merge=nm, tile=tile)


def test_large_state_counts():
    rng = np.random.default_rng(77)
    for q in (128, 300, 1000, 4096):
        dfa = W.random_dense_dfa(rng, q, bytes(range(0, 256, 16)), num_accepting=q // 8)
        text = W.uniform_text(rng, dfa.alphabet, 1 << 18)
        for lay in (P.LAYOUT_BYTE_GLOBAL, P.LAYOUT_HOT_LDS, P.LAYOUT_CLASS_LDS):
            run_case(f"dense Q={q} layout={lay}", dfa, text, chunk_len=4096, layout=lay)


@pytest.mark.parametrize("q,a", [(3000, 4), (1000, 20), (90, 255), (5000, 4)])
def test_class_table(q, a):
    """Column-indexed LDS table: chosen automatically when it fits in 48 KiB
    (and no k-gram code or LDS byte table applies); invalid bytes included."""
    rng = np.random.default_rng(q + a)
    alphabet = bytes(rng.choice(256, size=a, replace=False).astype(np.uint8))
    dfa = W.random_dense_dfa(rng, q, alphabet, num_accepting=max(1, q // 10))
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, layout=P.LAYOUT_CLASS_LDS)
    fits = 256 + (q + 1) * (a + 1) * 2 <= 48 * 1024
    assert (m.describe()["layout"] == P.LAYOUT_CLASS_LDS) == fits
    m.close()
    text = W.uniform_text(rng, alphabet, (1 << 18) + 5)
    for G in (4, 16):
        run_case(f"class Q={q} A={a} G={G}", dfa, text, chunk_len=1024, group=G, layout=P.LAYOUT_CLASS_LDS)
        run_case(f"class lookback Q={q} A={a} G={G}", dfa, text, chunk_len=1024, group=G,
                 layout=P.LAYOUT_CLASS_LDS, lookback=128, check_spec=False)
    bad = text.copy()
    bad[5000] = next(x for x in range(256) if x not in alphabet)
    say(f"[case] class invalid byte Q={q} A={a}")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, layout=P.LAYOUT_CLASS_LDS, chunk_len=1024)
    with pytest.raises(P.ParemError) as e:
        m.match(torch.from_numpy(bad).cuda())
    assert e.value.status == P.PAREM_ESYMBOL
    m.close()


@pytest.mark.parametrize("group", [2, 4, 8, 16])
def test_hot_rows_sparse_and_dense(group):
    """Hot-row layout: a sparse byte DFA whose walk stays in a few hot rows,
    a dense one whose walk mostly leaves them (every piece stepped twice),
    and one with fewer states than hot rows."""
    rng = np.random.default_rng(500 + group)
    sym = rng.choice(256, size=64, replace=False).astype(np.uint8)
    acc = rng.choice(np.arange(1, 3000), size=16, replace=False)
    sparse = W.sparse_dfa(rng, 3000, bytes(range(256)), 4, 4, acc, explicit_cols=sym)
    text = W.zipf_text(rng, sym, (1 << 20) + 77)
    m = P.Matcher(sparse.table, sparse.alphabet, sparse.start, sparse.accepting, layout=P.LAYOUT_HOT_LDS)
    assert m.describe()["layout"] == P.LAYOUT_HOT_LDS
    m.close()
    run_case(f"hot sparse G={group}", sparse, text, chunk_len=1024, group=group, layout=P.LAYOUT_HOT_LDS)
    run_case(f"hot sparse tiny G={group}", sparse, text[:1000], chunk_len=64, group=group, offset=3,
             layout=P.LAYOUT_HOT_LDS)
    dense = W.random_dense_dfa(rng, 700, bytes(rng.choice(256, size=4, replace=False).astype(np.uint8)),
                               num_accepting=70)
    run_case(f"hot dense G={group}", dense, W.uniform_text(rng, dense.alphabet, 1 << 18), chunk_len=2048,
             group=group, layout=P.LAYOUT_HOT_LDS)
    small = W.random_dense_dfa(rng, 20, bytes(rng.choice(256, size=30, replace=False).astype(np.uint8)),
                               num_accepting=3)
    run_case(f"hot small G={group}", small, W.uniform_text(rng, small.alphabet, 100_000), chunk_len=512,
             group=group, layout=P.LAYOUT_HOT_LDS)


@pytest.mark.parametrize("group", [2, 4, 8, 16])
def test_sparse_rows(group):
    """Sparse layout (rows of a default and a few exceptions displaced into
    one vector of slots): a byte DFA with explicit columns among 64 Zipf
    symbols (one default for every row: the uniform form), the same table
    with a default per state other than state 0 (per-row defaults: the
    general form), a 200-byte alphabet with per-row defaults (general form
    keyed by columns, with the invalid column), a 20-symbol alphabet whose
    invalid column is one of the exceptions (and a text with a byte outside
    it), lookback sets, a table with five exceptions in every row, and one
    whose slots do not fit LDS, which falls back to another layout."""
    rng = np.random.default_rng(900 + group)
    sym = rng.choice(256, size=64, replace=False).astype(np.uint8)
    acc = rng.choice(np.arange(1, 3000), size=16, replace=False)
    sp = W.sparse_dfa(rng, 3000, bytes(range(256)), 1, 4, acc, explicit_cols=sym)
    m = P.Matcher(sp.table, sp.alphabet, sp.start, sp.accepting, layout=P.LAYOUT_SPARSE_LDS)
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    m.close()
    m = P.Matcher(sp.table, sp.alphabet, sp.start, sp.accepting)  # no dense LDS table fits: AUTO takes it
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    m.close()
    text = W.zipf_text(rng, sym, (1 << 20) + 77)
    run_case(f"sparse G={group}", sp, text, chunk_len=1024, group=group, layout=P.LAYOUT_SPARSE_LDS)
    run_case(f"sparse tiny G={group}", sp, text[:1000], chunk_len=64, group=group, offset=3,
             layout=P.LAYOUT_SPARSE_LDS)
    run_case(f"sparse lookback G={group}", sp, text, chunk_len=2048, group=group, layout=P.LAYOUT_SPARSE_LDS,
             lookback=64, check_spec=False)
    # windows of 2..16 bytes: lookback sets read from the slot image, one lane a chunk
    full = expected_spec_runs(sp, text, 2048)
    for k in (2, 4, 16):
        got = run_case(f"sparse slot lookback K={k} G={group}", sp, text, chunk_len=2048, group=group,
                       layout=P.LAYOUT_SPARSE_LDS, lookback=k, check_spec=False)
        assert got.spec_runs < full / 4, (got.spec_runs, full)
    run_case(f"sparse slot lookback tiny G={group}", sp, text[:5000], chunk_len=64, group=group, offset=3,
             layout=P.LAYOUT_SPARSE_LDS, lookback=16, check_spec=False)
    dflt = (np.arange(3000, dtype=np.uint32) % 97 + 1)[:, None]
    shifted = W.Dfa(np.where(sp.table == 0, dflt, sp.table).astype(np.uint32), sp.alphabet, 5, sp.accepting)
    m = P.Matcher(shifted.table, shifted.alphabet, shifted.start, shifted.accepting, layout=P.LAYOUT_SPARSE_LDS)
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    m.close()
    run_case(f"sparse defaults G={group}", shifted, text, chunk_len=512, group=group, layout=P.LAYOUT_SPARSE_LDS)
    a200 = bytes(np.sort(rng.choice(256, size=200, replace=False)).astype(np.uint8))
    cols = W.sparse_dfa(rng, 1500, a200, 1, 3, acc[:5] % 1500)
    cdef = (np.arange(1500, dtype=np.uint32) % 89 + 2)[:, None]
    cols = W.Dfa(np.where(cols.table == 0, cdef, cols.table).astype(np.uint32), a200, 3, cols.accepting)
    m = P.Matcher(cols.table, cols.alphabet, cols.start, cols.accepting, layout=P.LAYOUT_SPARSE_LDS)
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    m.close()
    ctext = W.uniform_text(rng, a200, 400_003)
    run_case(f"sparse column defaults G={group}", cols, ctext, chunk_len=512, group=group,
             layout=P.LAYOUT_SPARSE_LDS)
    a20 = bytes(rng.choice(256, size=20, replace=False).astype(np.uint8))
    small = W.sparse_dfa(rng, 400, a20, 0, 3, rng.choice(np.arange(1, 400), size=9, replace=False))
    m = P.Matcher(small.table, small.alphabet, small.start, small.accepting, layout=P.LAYOUT_SPARSE_LDS,
                  chunk_len=1024, group=group)
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    stext = W.uniform_text(rng, a20, 300_001)
    want = oracle.walk_dfa(small, stext)
    got = m.match(torch.from_numpy(stext).cuda())
    assert (got.final_state, got.accept, got.count) == (want.final_state, want.accept, want.count)
    bad = stext.copy()
    bad[123_456] = next(x for x in range(256) if x not in a20)
    with pytest.raises(P.ParemError) as e:
        m.match(torch.from_numpy(bad).cuda())
    assert e.value.status == P.PAREM_ESYMBOL
    m.close()
    five = W.sparse_dfa(rng, 300, bytes(range(256)), 5, 5, acc[:3] % 300)
    m = P.Matcher(five.table, five.alphabet, five.start, five.accepting, layout=P.LAYOUT_SPARSE_LDS)
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    m.close()
    run_case(f"sparse five G={group}", five, W.uniform_text(rng, five.alphabet, 200_000), chunk_len=1024,
             group=group, layout=P.LAYOUT_SPARSE_LDS)
    # 2000 rows of 8-16 exceptions need about 26000 slots: more than LDS holds
    wide = W.sparse_dfa(rng, 2000, bytes(range(256)), 8, 16, acc[:3] % 2000)
    m = P.Matcher(wide.table, wide.alphabet, wide.start, wide.accepting, layout=P.LAYOUT_SPARSE_LDS)
    assert m.describe()["layout"] != P.LAYOUT_SPARSE_LDS
    m.close()
    run_case(f"sparse fallback G={group}", wide, W.uniform_text(rng, wide.alphabet, 200_000), chunk_len=1024,
             group=group, layout=P.LAYOUT_SPARSE_LDS)


def test_invalid_bytes():
    rng = np.random.default_rng(5)
    dfa = W.random_dense_dfa(rng, 9, b"ACGT", num_accepting=2)
    base = W.uniform_text(rng, b"ACGT", 8192)
    for pos in (0, 63, 64, 1000, 4095, 8191):
        text = base.copy()
        text[pos] = ord("N")
        m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=64)
        say(f"[case] invalid byte at {pos}")
        dev = torch.from_numpy(text).cuda()
        with pytest.raises(P.ParemError) as ei:
            m.match(dev)
        assert ei.value.status == P.PAREM_ESYMBOL
        with pytest.raises(P.ParemError) as ei:
            m.match(text)  # host path
        assert ei.value.status == P.PAREM_ESYMBOL
        m.close()


def test_host_text_path():
    dfa, text = W.dna_motif(n=1 << 20)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    got = m.match(text)
    want = oracle.walk_dfa(dfa, text)
    assert (got.final_state, got.accept, got.count) == (want.final_state, want.accept, want.count)
    m.close()


def test_compile_errors():
    with pytest.raises(P.ParemError) as ei:
        P.parem_compile(np.asarray([[0, 2], [1, 1]], dtype=np.uint8), b"ab", 0, [1])
    assert ei.value.status == P.PAREM_ESTATE
    with pytest.raises(P.ParemError) as ei:
        P.parem_compile(np.asarray([[0, 1], [1, 1]], dtype=np.uint8), b"aa", 0, [1])
    assert ei.value.status == P.PAREM_EINVAL
    with pytest.raises(P.ParemError) as ei:
        P.parem_compile(np.asarray([[0, 1], [1, 1]], dtype=np.uint8), b"ab", 2, [1])
    assert ei.value.status == P.PAREM_ESTATE
    with pytest.raises(P.ParemError) as ei:
        P.parem_compile(np.asarray([[0, 1], [1, 1]], dtype=np.uint8), b"ab", 0, [5])
    assert ei.value.status == P.PAREM_ESTATE
    with pytest.raises(P.ParemError) as ei:
        P.parem_compile(np.asarray([[0, 1], [1, 1]], dtype=np.uint8), b"ab", 0, [1], chunk_len=100)
    assert ei.value.status == P.PAREM_EINVAL


def test_sparse4096_reduced():
    dfa, text = W.sparse4096(n=64 << 20)
    run_case("sparse4096 64MiB", dfa, text)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    m.close()
    run_case("sparse4096 64MiB hot rows", dfa, text, layout=P.LAYOUT_HOT_LDS)
    got = run_case("sparse4096 64MiB lookback 4", dfa, text, lookback=4, check_spec=False)
    assert got.spec_runs < 2 * got.chunks, (got.spec_runs, got.chunks)


def test_batch_sample_pairs():
    specs = W.batch_specs()
    rng = np.random.default_rng(0)
    picks = sorted(rng.choice(len(specs), size=12, replace=False).tolist())
    for i in picks:
        s = specs[i]
        if s.text_len > (8 << 20):
            s = W.PairSpec(s.index, s.num_states, s.alphabet_size, 8 << 20)
        dfa, text = W.batch_pair(s)
        run_case(f"batch_pairs pair {i}", dfa, text)


def test_repeat_determinism():
    dfa, text = W.dna_motif(n=1 << 22)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    dev = torch.from_numpy(text).cuda()
    outs = set()
    for _ in range(5):
        r = m.match(dev)
        outs.add((r.final_state, r.count, r.spec_runs))
    assert len(outs) == 1
    m.close()


def test_nonsynchronizing_dfa():
    """Permutation columns: speculated runs never meet, so every chunk map is
    non-uniform and the general composition path runs."""
    q = 7
    alphabet = b"abc"
    table = np.stack([(np.arange(q) + k + 1) % q for k in range(3)], axis=1).astype(np.uint8)
    dfa = W.Dfa(table, alphabet, 2, np.asarray([0, 3], dtype=np.uint32))
    rng = np.random.default_rng(17)
    for n in (1, 100, 4096, 200003):
        text = W.uniform_text(rng, alphabet, n)
        for lay in all_layouts():
            run_case(f"permutation n={n} layout={lay}", dfa, text, chunk_len=64, layout=lay, group=4)
    # mixed: a synchronizing symbol 'r' resets to state 0
    table2 = np.concatenate([table, np.zeros((q, 1), dtype=np.uint8)], axis=1)
    dfa2 = W.Dfa(table2, b"abcr", 0, np.asarray([1, 5], dtype=np.uint32))
    probs = np.asarray([0.33, 0.33, 0.33, 0.01])
    text = np.frombuffer(b"abcr", dtype=np.uint8)[rng.choice(4, size=300000, p=probs)]
    for lay in all_layouts():
        run_case(f"mixed layout={lay}", dfa2, text, chunk_len=128, layout=lay, group=8)
    # more than 256 x 256 chunks: the second composition level takes more maps
    # than a workgroup has threads, all non-uniform (general tree)
    text = W.uniform_text(rng, alphabet, 64 * 70_001 + 5)
    run_case("permutation, two wide levels", dfa, text, chunk_len=64, group=4)
    run_case("mixed, two wide levels", dfa2,
             np.frombuffer(b"abcr", dtype=np.uint8)[rng.choice(4, size=64 * 90_000, p=probs)], chunk_len=64, group=8)
    # wide maps (100-state permutations: every set holds all 100 states, so a
    # first-level workgroup composes at most 64 maps): groups with a
    # synchronizing byte in every chunk compose one wave each, the others go
    # through the LDS tree
    q = 100
    wide = np.stack([rng.permutation(q) for _ in range(3)] + [np.zeros(q, dtype=np.int64)], axis=1)
    dfa3 = W.Dfa(wide.astype(np.uint8), b"abcr", 0, np.asarray([1, 50, 99], dtype=np.uint32))
    for pr, n in ((0.01, 400_000), (0.2, 400_000), (0.0005, 2_000_003)):
        p3 = np.asarray([(1 - pr) / 3] * 3 + [pr])
        text = np.frombuffer(b"abcr", dtype=np.uint8)[rng.choice(4, size=n, p=p3)]
        for lay in (P.LAYOUT_AUTO, P.LAYOUT_BYTE_LDS, P.LAYOUT_CLASS_LDS):
            run_case(f"wide permutation r={pr} n={n} layout={lay}", dfa3, text, chunk_len=64, layout=lay, group=8)


def lookback_runs(dfa, text, L, K, cap=64, kmax=4096):
    """Walks started with lookback sets: |B_c| when at most cap, else |R_c|.
    B_c is the image of every state under the K bytes before chunk c; the
    window grows fourfold (up to kmax) while |B_c| > cap, and a window that
    reaches the text start maps {q0} instead."""
    col = np.full(256, -1, dtype=np.int64)
    col[np.frombuffer(dfa.alphabet, dtype=np.uint8)] = np.arange(dfa.alphabet_size)
    T = dfa.table.astype(np.int64)
    chunks = (text.size + L - 1) // L
    runs = 1
    for c in range(1, chunks):
        b = c * L
        k = K
        while True:
            from_start = k >= b
            s = np.asarray([dfa.start]) if from_start else np.arange(dfa.num_states)
            for x in text[b - (b if from_start else k):b]:
                s = np.unique(T[s, col[x]])
            if s.size <= cap or from_start or k >= kmax:
                break
            k = min(4 * k, kmax)
        r = np.unique(T[:, col[text[b - 1]]]).size
        runs += s.size if s.size <= cap else r
    return runs


@pytest.mark.parametrize("K", [1, 7, 64, 700, 4096])
def test_lookback_sets(K):
    rng = np.random.default_rng(900 + K)
    dense = W.random_dense_dfa(rng, 700, bytes(rng.choice(256, size=4, replace=False).astype(np.uint8)),
                               num_accepting=50)
    sym = rng.choice(256, size=20, replace=False).astype(np.uint8)
    sparse = W.sparse_dfa(rng, 1500, bytes(sym), 4, 16, rng.choice(1500, size=24, replace=False))
    dna, _ = W.dna_motif(n=1024)
    cases = [("dense", dense), ("sparse", sparse), ("dna", dna)]
    for name, dfa in cases:
        text = W.uniform_text(rng, dfa.alphabet, (1 << 19) + 33)
        for L, G in ((1024, 8), (8192, 16), (64, 4)):
            got = run_case(f"lookback K={K} {name} L={L}", dfa, text, chunk_len=L, lookback=K, group=G,
                           check_spec=False)
            if L >= 1024 and K <= 64:
                assert got.spec_runs == lookback_runs(dfa, text, L, K), (name, L, K)
            assert got.spec_runs <= expected_spec_runs(dfa, text, L)
    # small texts: every chunk's set checked
    small = W.uniform_text(rng, dense.alphabet, 3000)
    got = run_case(f"lookback K={K} small", dense, small, chunk_len=128, lookback=K, check_spec=False)
    assert got.spec_runs == lookback_runs(dense, small, 128, K)


def test_lookback_invalid_bytes():
    rng = np.random.default_rng(31)
    dfa = W.random_dense_dfa(rng, 300, b"ACGT", num_accepting=20)
    base = W.uniform_text(rng, dfa.alphabet, 50_000)
    for pos in (0, 1, 1023, 1024, 1025, 2047, 30_000, 49_999):
        text = base.copy()
        text[pos] = ord("x")
        for K in (1, 16, 512):
            say(f"[case] lookback invalid pos={pos} K={K}")
            m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=1024, lookback=K)
            dev = torch.from_numpy(text).cuda()
            with pytest.raises(P.ParemError) as e:
                m.match(dev)
            assert e.value.status == P.PAREM_ESYMBOL
            m.close()


def test_sparse4096_full_size():
    """The large sparse byte DFA over its full 4 GiB Zipf text (the
    benchmark's sparse workload), sparse-row layout (the automatic choice),
    against the oracle."""
    dfa, text = W.sparse4096()
    say(f"[case] sparse4096 full: n={text.size}")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    assert m.describe()["layout"] == P.LAYOUT_SPARSE_LDS
    dev = torch.from_numpy(text).cuda()
    got = m.match(dev)
    m.close()
    want = oracle.walk_dfa(dfa, text)
    assert (got.final_state, got.accept, got.count) == (want.final_state, want.accept, want.count)


def perm_final_closed_form(text, start, q=7):
    """Final state of the permutation automaton delta(s, k-th symbol) =
    (s + k + 1) mod q: the start plus the sum of (k + 1) over the text, mod q."""
    total = 0
    for lo in range(0, text.size, 1 << 28):
        blk = text[lo:lo + (1 << 28)]
        total += int(np.count_nonzero(blk == ord("a"))) + 2 * int(np.count_nonzero(blk == ord("b"))) + \
            3 * int(np.count_nonzero(blk == ord("c")))
    return (start + total) % q


def test_count_beyond_32_bits():
    """2^32 + 17 bytes with every state final: the count equals the length
    (arithmetic; the oracle's u64 count is pinned the same way on the CPU)
    and the final state of the permutation automaton has a closed form. Its
    chunk maps never merge, so every composition level carries general maps
    with u64 segment counts above 2^32."""
    n = (1 << 32) + 17
    q = 7
    table = np.stack([(np.arange(q) + k + 1) % q for k in range(3)], axis=1).astype(np.uint8)
    dfa = W.Dfa(table, b"abc", 2, np.arange(q, dtype=np.uint32))
    rng = np.random.default_rng(2 ** 32 + 17)
    text = W.uniform_text(rng, b"abc", n)
    want_final = perm_final_closed_form(text, 2, q)
    say(f"[case] count beyond 32 bits: n={n}")
    d = torch.from_numpy(text).cuda()
    del text
    for opts in ({}, {"chunk_len": 32768}):
        m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, **opts)
        r = m.match(d)
        assert (r.final_state, r.accept, r.count) == (want_final, True, n), (opts, r)
        m.close()
    # one state, one symbol: k-gram entries carry the final-step counts
    one = W.Dfa(np.zeros((1, 1), dtype=np.uint8), b"a", 0, np.asarray([0], dtype=np.uint32))
    d.fill_(ord("a"))
    m = P.Matcher(one.table, one.alphabet, one.start, one.accepting)
    r = m.match(d)
    assert (r.final_state, r.accept, r.count) == (0, True, n), r
    m.close()
    del d
    torch.cuda.empty_cache()
