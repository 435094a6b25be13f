"""GPU tests of the learned speculation path and the boundary states.

* boundary states: bit-exact against the oracle's state after every prefix
  length c * chunk_len;
* the proposal network: forward logits and gradients against the float64
  oracle computed on the same bf16-rounded weights (tolerances below, from
  the bf16 rounding of the hidden activations), training lowers the loss;
* top-m selection: exactly the oracle's top-m of the GPU's own float32
  logits (same precision on both sides);
* learned matches: bit-exact (final, accept, count) against the oracle for
  trained, untrained and adversarial proposals, and re-run counts equal to
  the number of chunks whose true entry state was not selected.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
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


def class_mask(dfa, text, positions):
    """allowed states per boundary: the image of the column of the byte
    before it (the speculated set)"""
    col = {c: j for j, c in enumerate(dfa.alphabet)}
    q = dfa.num_states
    masks = np.zeros((len(positions), q), dtype=bool)
    for i, p in enumerate(positions):
        masks[i, np.unique(dfa.table[:, col[int(text[p - 1])]])] = True
    return masks


def windows_of(text, positions):
    out = np.full((len(positions), 32), 256, dtype=np.int64)
    for i, p in enumerate(positions):
        lo = max(0, p - 32)
        seg = text[lo:p]
        out[i, 32 - len(seg):] = seg
    return out


def oracle_params_bf16(flat, states):
    """the weights as the GPU multiplies them: matrices and embedding rounded
    to bf16, biases kept in fp32"""
    p = omlp.unpack(np.asarray(flat, dtype=np.float64).copy(), states)
    for k in ("emb", "W1", "W2", "W3"):
        p[k] = omlp.bf16_round(p[k].astype(np.float32)).astype(np.float64)
    return omlp.pack(p)


# ---------------------------------------------------------------------------
# boundary states
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("L", [64, 128, 1024])
def test_boundary_states_match_oracle(L):
    rng = np.random.default_rng(L)
    cases = [W.config2(n=1 << 20, copies=300)]
    for _ in range(4):
        cases.append(W.random_case(rng, max_states=60, max_alpha=6, max_len=300000))
    q = 7
    perm = np.stack([(np.arange(q) + k + 1) % q for k in range(3)], axis=1).astype(np.uint8)
    cases.append((W.Dfa(perm, b"abc", 2, np.asarray([0], dtype=np.uint32)),
                  W.uniform_text(rng, b"abc", 150000)))
    for i, (dfa, text) in enumerate(cases):
        if text.size == 0:
            continue
        say(f"[case] boundary L={L} case={i} Q={dfa.num_states} n={text.size}")
        m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
        got = P.boundary_states(m, dev(text), L).cpu().numpy().view(np.uint32)
        pos = np.arange(0, text.size, L, dtype=np.uint64)
        want, _ = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, pos)
        assert np.array_equal(got, want), (i, np.flatnonzero(got != want)[:5])
        m.close()


def test_boundary_states_after_invalid_byte():
    rng = np.random.default_rng(3)
    dfa = W.random_dense_dfa(rng, 9, b"ACGT", num_accepting=2)
    text = W.uniform_text(rng, b"ACGT", 20000)
    text[5000] = ord("N")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    got = P.boundary_states(m, dev(text), 64).cpu().numpy().view(np.uint32)
    pos = np.arange(0, 5001, 64, dtype=np.uint64)
    want, _ = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, pos)
    assert np.array_equal(got[:want.size], want)
    assert np.all(got[want.size:] == 0xFFFFFFFF)
    m.close()


# ---------------------------------------------------------------------------
# the proposal network
# ---------------------------------------------------------------------------

def random_params(states, seed):
    rng = np.random.default_rng(seed)
    flat = W.mlp_init_params(states, seed=seed).astype(np.float64)
    flat += 0.02 * rng.standard_normal(flat.size)
    return flat.astype(np.float32)


def test_forward_logits_match_oracle():
    dfa, text = W.config2(n=1 << 18, copies=100)
    states = dfa.num_states
    params = random_params(states, 5)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, params)
    rng = np.random.default_rng(2)
    pos = np.sort(rng.integers(1, text.size, size=300)).astype(np.uint64)
    pos[:3] = [1, 5, 31]  # windows that reach before the text start
    got = prop.logits(dev(text), pos).cpu().numpy().astype(np.float64)
    want, _ = omlp.forward(oracle_params_bf16(params, states), states, windows_of(text, pos.astype(np.int64)),
                           np.ones((len(pos), states), dtype=bool))
    # bf16 rounding of the two hidden activations (relative 2^-9 each) spread
    # through 256-term sums: |error| well under 0.02 + 0.02 |z|
    err = np.abs(got - want)
    assert np.all(err <= 0.02 + 0.02 * np.abs(want)), float(err.max())
    prop.close()
    m.close()


def test_gradient_matches_oracle():
    dfa, text = W.config2(n=1 << 18, copies=100)
    states = dfa.num_states
    params = random_params(states, 9)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, params)
    rng = np.random.default_rng(4)
    pos = np.sort(rng.integers(1, text.size, size=512)).astype(np.uint64)
    labels_np, _ = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, pos)
    td = dev(text)
    loss = prop.train_step(td, dev(pos.view(np.int64)), dev(labels_np.astype(np.int32)), lr=0.0,
                           weight_decay=0.0).item()
    g_gpu = prop.grad().astype(np.float64)
    flat = oracle_params_bf16(params, states)
    wins = windows_of(text, pos.astype(np.int64))
    mask = class_mask(dfa, text, pos.astype(np.int64))
    loss_o, g_o = omlp.loss_and_grad(flat, states, wins, mask, labels_np.astype(np.int64))
    assert abs(loss - loss_o) <= 1e-2 * max(1.0, abs(loss_o))
    go = omlp.unpack(g_o, states)
    gg = omlp.unpack(g_gpu, states)
    for k in ("emb", "W1", "b1", "W2", "b2", "W3", "b3"):
        a, b = gg[k].reshape(-1), go[k].reshape(-1)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        cos = float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))
        assert rel < 0.05 and cos > 0.998, (k, rel, cos)
    prop.close()
    m.close()


def test_training_lowers_loss_and_predicts():
    dfa, text = W.config4_train_text(n=16 << 20)
    states = dfa.num_states
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    td = dev(text)
    prop, hist = P.train_proposal(m, td, W.mlp_init_params(states), steps=300, batch=2048, lr=2e-3,
                                  log_every=50, seed=1)
    say(f"[train] {hist}")
    assert hist[-1][1] < 0.5 * hist[0][1]
    # held-out boundaries of the benchmark text distribution
    _, test_text = W.config2(n=1 << 20, copies=100)
    pos = np.arange(64, test_text.size, 64, dtype=np.uint64)
    want, _ = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, test_text, pos)
    z = prop.logits(dev(test_text), pos).cpu().numpy()
    mask = class_mask(dfa, test_text, pos.astype(np.int64))
    pred = np.argmax(np.where(mask, z, -np.inf), axis=1)
    acc = float(np.mean(pred == want))
    say(f"[train] top-1 accuracy {acc:.4f}")
    assert acc > 0.9
    prop.close()
    m.close()


@pytest.mark.parametrize("mm", [1, 3, 16])
def test_topm_selection_matches_oracle(mm):
    dfa, text = W.config2(n=1 << 18, copies=100)
    states = dfa.num_states
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, random_params(states, 21))
    L = 256
    td = dev(text)
    sel, nsel = prop.select(td, L, mm)
    sel, nsel = sel.cpu().numpy().astype(np.int64), nsel.cpu().numpy()
    pos = np.arange(L, text.size, L, dtype=np.uint64)
    z = prop.logits(td, pos).cpu().numpy()
    allowed = class_mask(dfa, text, pos.astype(np.int64))
    want = omlp.topm(z, allowed, mm)
    col = {c: j for j, c in enumerate(dfa.alphabet)}
    assert nsel[0] == 1 and sel[0, 0] == 0
    for c in range(1, len(nsel)):
        lst = np.unique(dfa.table[:, col[int(text[c * L - 1])]])
        got_states = sorted(lst[sel[c, :nsel[c]]].tolist())
        assert got_states == sorted(want[c - 1]), c
    prop.close()
    m.close()


# ---------------------------------------------------------------------------
# learned matches
# ---------------------------------------------------------------------------

def learned_case(name, dfa, text, params, mm, chunk_len=0, **opts):
    say(f"[case] learned {name}: Q={dfa.num_states} n={text.size} m={mm} L={chunk_len}")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=chunk_len, **opts)
    prop = P.Proposal(m, params)
    got = m.match_learned(prop, dev(text), mm)
    want = oracle.walk_dfa(dfa, text)
    assert (got.final_state, got.accept, got.count) == (want.final_state, want.accept, want.count), name
    prop.close()
    m.close()
    return got


@pytest.mark.parametrize("mm", [1, 4, 16])
def test_learned_exact_untrained(mm):
    dfa, text = W.config2(n=4 << 20)
    got = learned_case("config2 untrained", dfa, text, random_params(dfa.num_states, 3), mm, chunk_len=2048)
    assert got.chunks == 2048
    if mm >= 16:
        assert got.rerun_chunks <= got.chunks


def test_learned_reruns_equal_misses():
    """m = 1 on the motif automaton (runs merge: every map is uniform): a chunk
    is walked again exactly when its true entry state was not selected."""
    dfa, text = W.config2(n=2 << 20)
    L = 1024
    params = random_params(dfa.num_states, 7)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=L)
    prop = P.Proposal(m, params)
    td = dev(text)
    sel, nsel = prop.select(td, L, 1)
    sel = sel.cpu().numpy().astype(np.int64)
    pos = np.arange(0, text.size, L, dtype=np.uint64)
    entries, _ = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, pos)
    col = {c: j for j, c in enumerate(dfa.alphabet)}
    misses = 0
    for c in range(1, len(pos)):
        lst = np.unique(dfa.table[:, col[int(text[c * L - 1])]])
        if lst[sel[c, 0]] != entries[c]:
            misses += 1
    got = m.match_learned(prop, td, 1)
    want = oracle.walk_dfa(dfa, text)
    assert (got.final_state, got.count) == (want.final_state, want.count)
    assert misses > 0
    assert got.rerun_chunks == misses
    prop.close()
    m.close()


@pytest.mark.parametrize("n,L", [(3_000_001, 1024), (1 << 20, 64), (50_017, 64), (200_000, 8192)])
def test_learned_subchunk_rewalk(n, L):
    """Chunks walked again from their whole set: up to 2048 marked chunks a
    round are walked in sub-chunks (64, or single bytes in a tail under 64),
    more go to the whole-set walk; ragged tails, both ways exact."""
    dfa, text = W.config2(n=n, copies=100)
    got = learned_case(f"sub-chunk re-walk n={n} L={L}", dfa, text, random_params(dfa.num_states, 17), 1,
                       chunk_len=L)
    assert got.rerun_chunks > 0


def test_learned_sparse_rows():
    """Learned speculation over the sparse-row layout (selected walks,
    coverage, re-walks)."""
    rng = np.random.default_rng(31)
    sym = rng.choice(256, size=16, replace=False).astype(np.uint8)
    dfa = W.sparse_dfa(rng, 60, bytes(range(256)), 1, 4, rng.choice(np.arange(1, 60), size=5, replace=False),
                       explicit_cols=sym)
    text = W.zipf_text(rng, sym, 3_000_017)
    for mm in (1, 4):
        learned_case("sparse rows", dfa, text, random_params(dfa.num_states, 41), mm, chunk_len=2048,
                     layout=P.LAYOUT_SPARSE_LDS)


def test_learned_adversarial_proposal():
    """A proposal that always prefers the highest state id (biases only) on a
    non-synchronising automaton: coverage fails along the whole text and the
    escalation walks every chunk from its whole set; still exact."""
    q = 7
    perm = np.stack([(np.arange(q) + k + 1) % q for k in range(3)], axis=1).astype(np.uint8)
    dfa = W.Dfa(perm, b"abc", 2, np.asarray([0, 4], dtype=np.uint32))
    rng = np.random.default_rng(8)
    text = W.uniform_text(rng, b"abc", 300000)
    flat = np.zeros(P.proposal_param_count(q), dtype=np.float32)
    flat[-q:] = np.arange(q, dtype=np.float32)  # b3
    for mm in (1, 2):
        got = learned_case("permutation adversarial", dfa, text, flat, mm, chunk_len=1024, group=4)
        assert got.rerun_chunks > 0


def test_learned_fuzz_and_invalid():
    rng = np.random.default_rng(99)
    for i in range(12):
        dfa, text = W.random_case(rng, max_states=40, max_alpha=6, max_len=60000)
        if text.size == 0:
            continue
        params = random_params(dfa.num_states, i)
        for mm in (1, 5):
            learned_case(f"fuzz {i}", dfa, text, params, mm, chunk_len=int(rng.choice([64, 256, 1024])))
    dfa, text = W.config2(n=1 << 20, copies=200)
    text = text.copy()
    text[70000] = ord("N")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=1024)
    prop = P.Proposal(m, random_params(dfa.num_states, 1))
    with pytest.raises(P.ParemError) as ei:
        m.match_learned(prop, dev(text), 2)
    assert ei.value.status == P.PAREM_ESYMBOL
    prop.close()
    m.close()


def test_learned_gain_over_plain_speculation():
    """What the trained network buys: one walk per chunk instead of the whole
    speculated set, with almost no chunk walked again, and the same result."""
    dfa, train_text = W.config4_train_text(n=16 << 20)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=2048)
    prop, hist = P.train_proposal(m, dev(train_text), W.mlp_init_params(dfa.num_states), steps=300, batch=2048,
                                  lr=2e-3, log_every=100, seed=2)
    _, text = W.config2(n=8 << 20)
    td = dev(text)
    plain = m.match(td)
    learned = m.match_learned(prop, td, 1)
    want = oracle.walk_dfa(dfa, text)
    assert (learned.final_state, learned.count) == (want.final_state, want.count)
    assert (plain.final_state, plain.count) == (want.final_state, want.count)
    share = learned.rerun_chunks / learned.chunks
    say(f"[gain] plain walks {plain.spec_runs}, learned walks {learned.spec_runs}, re-run share {share:.5f}")
    assert share < 0.01
    assert plain.spec_runs >= 5 * learned.spec_runs
    prop.close()
    m.close()
