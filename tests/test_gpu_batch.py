"""GPU parity of the batched persistent launch against the CPU oracle.

Every pair of a batch must give the sequential run's (final state, accept
flag, count) bit-exactly, whatever the per-pair options (chunk length,
lockstep group, staged tile, merging), with the run captured in a HIP graph
or enqueued eagerly, and across graph replays with new texts.
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


def batch_chunk_len(n):
    """The batch's automatic chunk length (about 256 chunks, 64 B .. 8 KiB)."""
    L = 64
    while L < 8192 and L * 256 < n:
        L *= 2
    return L


def spec_runs(dfa, text, L):
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


def random_pairs(seed, count, max_states=600, max_len=300_000):
    rng = np.random.default_rng(seed)
    lens = [0, 1, 15, 16, 17, 63, 64, 65, 127, 129, 1000, 4097]
    pairs = []
    for i in range(count):
        q = int(np.floor(np.exp(rng.uniform(0, np.log(max_states)))))
        a = int(rng.choice([1, 2, 3, 4, 5, 8, 20, 256]))
        alphabet = bytes(rng.choice(256, size=a, replace=False).astype(np.uint8))
        if rng.random() < 0.5:
            dfa = W.random_dense_dfa(rng, q, alphabet, num_accepting=int(rng.integers(0, q + 1)))
        else:
            acc = rng.choice(q, size=int(rng.integers(0, q + 1)), replace=False)
            dfa = W.sparse_dfa(rng, q, alphabet, 1, 4, acc)
        dfa.start = int(rng.integers(0, q))
        n = lens[i] if i < len(lens) else int(np.exp(rng.uniform(0, np.log(max_len))))
        pairs.append((dfa, W.uniform_text(rng, alphabet, n)))
    return pairs


def to_device(texts):
    out = []
    for t in texts:
        d = torch.empty(t.size, dtype=torch.uint8, device="cuda")
        if t.size:
            d.copy_(torch.from_numpy(t))
        out.append(d)
    return out


def check(pairs, got, name, opts=None):
    for i, ((dfa, text), r) in enumerate(zip(pairs, got)):
        want = oracle.walk_dfa(dfa, text)
        assert (r.final_state, r.accept, r.count) == (want.final_state, want.accept, want.count), \
            f"{name}: pair {i} Q={dfa.num_states} A={dfa.alphabet_size} n={text.size}"
        L = (opts[i].get("chunk_len") if opts else 0) or batch_chunk_len(text.size)
        assert r.chunks == ((text.size + L - 1) // L if text.size else 0), f"{name}: pair {i}"
        if opts and opts[i].get("lookback"):
            assert r.spec_runs <= spec_runs(dfa, text, L), f"{name}: pair {i}"
            assert r.spec_runs >= r.chunks
        else:
            assert r.spec_runs == spec_runs(dfa, text, L), f"{name}: pair {i}"
        assert r.rerun_chunks == 0


def matchers(pairs):
    return [P.Matcher(d.table, d.alphabet, d.start, d.accepting) for d, _ in pairs]


def test_batch_mixed_graph_and_eager():
    pairs = random_pairs(101, 96)
    say(f"[case] batch mixed: {len(pairs)} pairs, {sum(t.size for _, t in pairs)} bytes")
    ms = matchers(pairs)
    b = P.Batch(ms, [t.size for _, t in pairs])
    info = b.describe()
    say(f"[info] {info}")
    assert info["pairs"] == len(pairs)
    dev = to_device([t for _, t in pairs])
    check(pairs, b.run(dev, use_graph=False), "eager")
    check(pairs, b.run(dev, use_graph=True), "graph")
    assert b.describe()["graph_nodes"] >= info["walk_launches"] + info["levels"]


def test_batch_graph_replays_new_texts():
    pairs = random_pairs(202, 40)
    ms = matchers(pairs)
    lens = [t.size for _, t in pairs]
    b = P.Batch(ms, lens)
    rng = np.random.default_rng(7)
    for rep in range(3):
        texts = [W.uniform_text(rng, d.alphabet, n) for (d, _), n in zip(pairs, lens)]
        cur = [(d, t) for (d, _), t in zip(pairs, texts)]
        say(f"[case] replay {rep}")
        dev = to_device(texts)
        # eager work of the program between replays
        scratch = torch.arange(1 << 20, device="cuda", dtype=torch.int32).sum()
        out = b.run_async(dev, use_graph=True)
        torch.cuda.synchronize()
        assert int(scratch) == (1 << 20) * ((1 << 20) - 1) // 2
        check(cur, P.Batch.results(out, len(cur)), f"replay {rep}")
        check(cur, b.run(dev, use_graph=False), f"eager {rep}")


def test_batch_sparse_row_handles():
    """Handles compiled with sparse rows (large sparse byte DFAs) in a batch:
    walked with their byte table through L2, beside other pairs."""
    rng = np.random.default_rng(77)
    pairs = []
    for q in (300, 1200, 4000):
        sym = rng.choice(256, size=32, replace=False).astype(np.uint8)
        dfa = W.sparse_dfa(rng, q, bytes(range(256)), 1, 4, rng.choice(np.arange(1, q), size=7, replace=False),
                           explicit_cols=sym)
        pairs.append((dfa, W.zipf_text(rng, sym, int(rng.integers(5_000, 400_000)))))
    pairs += random_pairs(404, 12, max_len=200_000)
    ms = matchers(pairs)
    assert [m.describe()["layout"] for m in ms[:3]] == [P.LAYOUT_SPARSE_LDS] * 3
    say("[case] batch with sparse-row handles")
    b = P.Batch(ms, [t.size for _, t in pairs])
    check(pairs, b.run(to_device([t for _, t in pairs])), "sparse rows")


def test_batch_per_pair_options():
    pairs = random_pairs(303, 32, max_len=100_000)
    ms = matchers(pairs)
    rng = np.random.default_rng(3)
    opts = []
    for _ in pairs:
        opts.append({"chunk_len": int(rng.choice([64, 128, 256, 1024, 4096])),
                     "group": int(rng.choice([4, 8, 16])), "tile": int(rng.choice([64, 128])),
                     "no_merge": int(rng.random() < 0.2),
                     "lookback": int(rng.choice([0, 0, 1, 16, 256, 4096]))})
    say(f"[case] per-pair options")
    b = P.Batch(ms, [t.size for _, t in pairs], opts)
    got = b.run(to_device([t for _, t in pairs]))
    check(pairs, got, "options", opts)
    kinds = set()
    for (d, t), m, o in zip(pairs, ms, opts):
        if t.size:
            kinds.add((m.describe()["layout"], m.describe()["kgram"], o["group"], o["tile"], o["lookback"] > 0))
    assert b.describe()["walk_launches"] >= len({(k[2], k[3], k[4]) for k in kinds})


def test_batch_invalid_byte_and_errors():
    pairs = random_pairs(404, 20, max_len=20_000)
    bad_i = next(i for i, (d, t) in enumerate(pairs) if t.size > 100 and d.alphabet_size < 256)
    d, t = pairs[bad_i]
    t = t.copy()
    invalid = next(x for x in range(256) if x not in d.alphabet)
    t[t.size // 2] = invalid
    pairs[bad_i] = (d, t)
    ms = matchers(pairs)
    lens = [x.size for _, x in pairs]
    say("[case] invalid byte in one pair")
    dev = to_device([x for _, x in pairs])
    got = P.Batch(ms, lens).run(dev)
    for i, ((dd, tt), r) in enumerate(zip(pairs, got)):
        if i == bad_i:
            assert r.final_state == P.INVALID_STATE and not r.accept and r.count == 0
        else:
            want = oracle.walk_dfa(dd, tt)
            assert (r.final_state, r.accept, r.count) == (want.final_state, want.accept, want.count)
    out = torch.empty(len(pairs) * P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.ParemError) as e:
        P.parem_match_batch([m.handle for m in ms], [x.data_ptr() for x in dev], lens,
                            torch.cuda.current_stream().cuda_stream, out.data_ptr())
    assert e.value.status == P.PAREM_ESYMBOL
    # misaligned text pointer
    b = P.Batch(ms, lens)
    buf = torch.empty(lens[bad_i] + 32, dtype=torch.uint8, device="cuda")
    dev2 = list(dev)
    dev2[bad_i] = buf[1:1 + lens[bad_i]]
    with pytest.raises(P.ParemError) as e:
        b.run(dev2)
    assert e.value.status == P.PAREM_EINVAL
    # a lockstep group of 2 is not offered by the batch kernels
    with pytest.raises(P.ParemError) as e:
        P.Batch(ms, lens, [{"group": 2}] * len(ms))
    assert e.value.status == P.PAREM_EUNSUPPORTED


def test_match_batch_one_shot():
    pairs = random_pairs(505, 24, max_len=50_000)
    ms = matchers(pairs)
    lens = [t.size for _, t in pairs]
    dev = to_device([t for _, t in pairs])
    out = torch.empty(len(pairs) * P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    say("[case] parem_match_batch")
    P.parem_match_batch([m.handle for m in ms], [x.data_ptr() for x in dev], lens,
                        torch.cuda.current_stream().cuda_stream, out.data_ptr())
    check(pairs, P.Batch.results(out, len(pairs)), "one-shot")


def test_tune_candidates_agree():
    rng = np.random.default_rng(9)
    dfa = W.sparse_dfa(rng, 300, bytes(rng.choice(256, size=20, replace=False).astype(np.uint8)), 4, 16,
                       rng.choice(300, size=5, replace=False))
    text = W.uniform_text(rng, dfa.alphabet, 1 << 20)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    dev = to_device([text])[0]
    cands = [{"chunk_len": L, "group": g, "tile": t, "lookback": k} for L in (1024, 4096) for g in (4, 8, 16)
             for t in (64, 128) for k in (0, 64)]
    cands.append({"chunk_len": 1 << 16})  # above the maximum: not runnable
    say("[case] parem_tune")
    ms_, best = P.parem_tune(m.handle, dev.data_ptr(), text.size, 16, cands, 2,
                             torch.cuda.current_stream().cuda_stream)
    assert ms_[-1] == -1.0 and all(x > 0 for x in ms_[:-1])
    assert best == int(np.argmin(np.where(np.asarray(ms_) > 0, ms_, np.inf)))
    want = oracle.walk_dfa(dfa, text)
    for o in cands[:-1]:
        r = P.Batch([m], [text.size], [o]).run([dev])[0]
        assert (r.final_state, r.accept, r.count) == (want.final_state, want.accept, want.count), o


def test_batch_uneven_4096_full_size():
    """The 4096-pair uneven workload at full size (25.98 GB), planned as the
    benchmark plans it (autotuner cache, no new measurements), in one graph
    replay: every pair's result equals the oracle's. The oracle runs in the
    generation thread pool (its C walk releases the interpreter lock), each
    worker keeping only the (final, accept, count) triple."""
    import concurrent.futures as cf
    import os

    from paper_1412_1741_amd.autotune import Autotuner

    specs = W.batch_specs()

    def make(spec):
        dfa, text = W.batch_pair(spec)
        want = oracle.walk_dfa(dfa, text)
        return dfa, text, (want.final_state, want.accept, want.count)

    dfas, devs, wants = [], [], []
    say(f"[case] uneven batch: generating {len(specs)} pairs with their oracle results")
    with cf.ThreadPoolExecutor(16) as ex:
        for i, (dfa, text, want) in enumerate(ex.map(make, specs)):
            dfas.append(dfa)
            devs.append(torch.from_numpy(text).cuda())
            wants.append(want)
            if (i + 1) % 512 == 0:
                say(f"[case] uneven batch: {i + 1} pairs")
    cache = os.path.join(os.path.dirname(P.__file__), "tuned", "batch_mi355x.json")
    tuner = Autotuner(cache_path=cache, measure=False)
    ms, opts = tuner.plan(dfas, devs)
    b = P.Batch(ms, [d.numel() for d in devs], opts)
    say(f"[info] {b.describe()}")
    got = b.run(devs, use_graph=True)
    total = sum(d.numel() for d in devs)
    bad = [i for i, r in enumerate(got) if (r.final_state, r.accept, r.count) != wants[i]]
    say(f"[case] uneven batch: {len(got) - len(bad)} of {len(got)} pairs ({total} bytes) equal the oracle")
    assert not bad, bad[:10]
    for i, r in enumerate(got):
        assert r.chunks == 0 or r.spec_runs >= r.chunks


def test_batch_learned_pairs():
    """Pairs with a proposal run learned speculation inside the batch (on a
    branch of their own); results stay exact with an untrained proposal (many
    re-walks) and a briefly trained one, in graph and eager runs and across
    replays with new texts (new pointers re-capture the graph)."""
    rng = np.random.default_rng(77)
    pairs = random_pairs(606, 12, max_states=300, max_len=200_000)
    dna, dtext = W.dna_motif(n=(1 << 20) + 13)
    dense = W.random_dense_dfa(rng, 1200, bytes(rng.choice(256, size=4, replace=False).astype(np.uint8)),
                               num_accepting=40)
    pairs += [(dna, dtext), (dense, W.uniform_text(rng, dense.alphabet, 300_000))]
    ms = matchers(pairs)
    lens = [t.size for _, t in pairs]
    dev = to_device([t for _, t in pairs])
    say("[case] batch learned: training the DNA proposal")
    trained, _ = P.train_proposal(ms[-2], dev[-2], W.mlp_init_params(dna.num_states), steps=60, batch=2048,
                                  lr=2e-3, seed=3)
    untrained = P.Proposal(ms[-1], W.mlp_init_params(dense.num_states, seed=5))
    props = [None] * len(pairs)
    props[-2], props[-1] = trained, untrained
    mvec = [0] * len(pairs)
    mvec[-2], mvec[-1] = 4, 2
    b = P.Batch(ms, lens, [{"chunk_len": 1024}] * len(pairs), props, mvec)
    assert b.describe()["learned_pairs"] == 2
    for use_graph in (False, True, True):
        say(f"[case] batch learned graph={use_graph}")
        got = b.run(dev, use_graph=use_graph)
        for i, ((dfa, text), r) in enumerate(zip(pairs, got)):
            want = oracle.walk_dfa(dfa, text)
            assert (r.final_state, r.accept, r.count) == (want.final_state, want.accept, want.count), i
        assert got[-1].rerun_chunks > 0  # the untrained proposal misses
    # new texts (and pointers) for every pair
    texts2 = [W.uniform_text(rng, d.alphabet, n) for (d, _), n in zip(pairs, lens)]
    dev2 = to_device(texts2)
    say("[case] batch learned: new texts")
    got = b.run(dev2, use_graph=True)
    for i, ((dfa, _), text, r) in enumerate(zip(pairs, texts2, got)):
        want = oracle.walk_dfa(dfa, text)
        assert (r.final_state, r.accept, r.count) == (want.final_state, want.accept, want.count), i
    # a proposal of another handle is rejected
    with pytest.raises(P.ParemError) as e:
        P.Batch(ms[:1], lens[:1], None, [trained], [4])
    assert e.value.status == P.PAREM_EINVAL
