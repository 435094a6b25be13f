"""CPU checks of the seeded input generators and of the autotuner's host logic
(size classes, defaults, cache round trip); no GPU."""
import json
import math

import numpy as np

import workloads as W


def test_uniform_text_is_uniform_and_seeded():
    for a in (1, 3, 4, 20, 100, 256):
        rng = np.random.default_rng(a)
        alpha = bytes(rng.choice(256, size=a, replace=False).astype(np.uint8))
        t = W.uniform_text(np.random.default_rng(7), alpha, 1 << 18)
        t2 = W.uniform_text(np.random.default_rng(7), alpha, 1 << 18)
        assert np.array_equal(t, t2)
        assert np.isin(t, np.frombuffer(alpha, dtype=np.uint8)).all()
        counts = np.bincount(t, minlength=256)[np.frombuffer(alpha, dtype=np.uint8)]
        expect = t.size / a
        # chi-square with a - 1 degrees of freedom, far tail
        chi2 = float(((counts - expect) ** 2 / expect).sum())
        assert chi2 < (a - 1) + 8 * math.sqrt(2 * max(a - 1, 1)) + 10, (a, chi2)


def test_zipf_text_blocks_do_not_depend_on_threads():
    sym = np.arange(64, dtype=np.uint8)
    n = (W._BLOCK * 2) + 12345
    a = W.zipf_text(np.random.default_rng(3), sym, n, threads=1)
    b = W.zipf_text(np.random.default_rng(3), sym, n, threads=8)
    assert np.array_equal(a, b)
    c = np.bincount(a, minlength=64).astype(np.float64)
    # rank order: frequencies fall with rank, roughly as k^-1.1
    assert (np.diff(c[:8]) < 0).all()
    assert abs(math.log(c[0] / c[7]) / math.log(8) - 1.1) < 0.05


def test_batch_specs_follow_their_distributions():
    specs = W.batch_specs()
    assert len(specs) == 4096
    q = np.array([s.num_states for s in specs])
    a = np.array([s.alphabet_size for s in specs])
    n = np.array([s.text_len for s in specs])
    assert q.min() >= 4 and q.max() < 4096 and set(a) == {4, 20, 256}
    assert n.min() >= 1024 and n.max() < 64 << 20
    # log-uniform: medians near the geometric means
    assert abs(math.log(np.median(q)) - math.log(128)) < 0.3
    assert abs(math.log(np.median(n)) - (math.log(1024) + math.log(64 << 20)) / 2) < 0.3
    assert 0.15 < float((q >= 1024).mean()) < 0.25
    dfa, text = W.batch_pair(specs[5])
    assert dfa.table.shape == (specs[5].num_states, specs[5].alphabet_size)
    assert text.size == specs[5].text_len and np.isin(text, np.frombuffer(dfa.alphabet, dtype=np.uint8)).all()
    # explicit transitions: 4..16 per state, capped at A; the rest go to state 0
    explicit = (dfa.table != 0).sum(axis=1)
    assert explicit.max() <= min(16, dfa.alphabet_size)


def test_autotune_size_classes_and_defaults(tmp_path):
    from paper_1412_1741_amd.autotune import Autotuner, batch_chunk_len, size_class
    assert size_class(35, 4, 1 << 20) == "A4/Q4^2/N4^10"
    assert size_class(4095, 256, (64 << 20) - 1) == "A256/Q4^5/N4^12"
    assert [batch_chunk_len(n) for n in (1, 16384, 16385, 1 << 20, 1 << 30)] == [64, 64, 128, 4096, 8192]
    rng = np.random.default_rng(1)
    wide = W.random_dense_dfa(rng, 500, b"ACGT")
    narrow, _ = W.dna_motif(n=64)
    assert Autotuner.default(wide)[1].get("lookback") == 256
    assert Autotuner.default(narrow)[1] == {}
    path = tmp_path / "cache.json"
    t = Autotuner(cache_path=str(path))
    t.cache["A4/Q4^2/N4^10"] = {"layout": 3, "chunk_len": 8192, "group": 4, "tile": 128, "lookback": 0,
                                "ms_per_copy": 0.001}
    t.save()
    t2 = Autotuner(cache_path=str(path), measure=False)
    assert t2.cache == json.loads(path.read_text())
