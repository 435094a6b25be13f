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
    cases = [W.dna_motif(n=1 << 20, copies=300)]
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
    dfa, text = W.dna_motif(n=1 << 18, copies=100)
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


# Elementwise bounds against the bf16-operand oracle (same operands rounded
# at the same points, sums in float64). What is left is fp32 accumulation,
# at most K 2^-24 of an entry's scale (K <= 4096 terms: 2^-12), and the rare
# operand whose fp32 and float64 values round to different bf16 neighbours
# (that term moves by one bf16 spacing, at most 2^-7 of itself; in a sum of
# few terms, e.g. a head row of a state that few rows allow, that is nearly
# the whole scale). Every entry must stay within 2^-6 of its scale (two such
# flips), and all but 1 in 1000 within 2^-10.
TIGHT, LOOSE, TIGHT_SHARE = 2.0 ** -10, 2.0 ** -6, 1e-3

GRAD_TENSORS = ("emb", "W1", "b1", "W2", "b2", "W3", "b3")


def check_scaled(name, got, want, scale):
    err = np.abs(np.asarray(got, dtype=np.float64) - want)
    ratio = err / np.maximum(scale, 1e-300)
    over = float(np.mean(err > TIGHT * scale)) if err.size else 0.0
    say(f"[tol] {name}: max err/scale {float(ratio.max()):.3e}, share over 2^-10 {over:.2e}")
    assert np.all(err <= LOOSE * scale), (name, float(ratio.max()))
    assert over <= TIGHT_SHARE, (name, over)


def head_case(kind):
    """(dfa, text) for the proposal tests: the motif automaton (35 states,
    fused inference), a dense random 1200-state DFA over ACGT and the
    4096-state sparse byte DFA (unfused inference: heads over 64 states)."""
    if kind == "motif35":
        return W.dna_motif(n=1 << 18, copies=100)
    if kind == "dense1200":
        rng = np.random.default_rng(1200)
        dfa = W.random_dense_dfa(rng, 1200, b"ACGT", num_accepting=19)
        return dfa, W.uniform_text(rng, b"ACGT", 1 << 18)
    return W.sparse4096(n=1 << 20)


@pytest.mark.parametrize("kind,batch", [("motif35", 512), ("dense1200", 512), ("sparse4096", 256)])
def test_gradient_matches_oracle_elementwise(kind, batch):
    dfa, text = head_case(kind)
    states = dfa.num_states
    params = random_params(states, 9)
    say(f"[case] gradient {kind} Q={states} batch={batch}")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, params)
    rng = np.random.default_rng(4)
    pos = np.sort(rng.choice(np.arange(1, text.size), size=batch, replace=False)).astype(np.uint64)
    labels_np, _ = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, pos)
    td = dev(text)
    loss = prop.train_step(td, dev(pos.view(np.int64)), dev(labels_np.astype(np.int32)), lr=0.0,
                           weight_decay=0.0).item()
    g_gpu = prop.grad().astype(np.float64)
    flat = oracle_params_bf16(params, states)
    wins = windows_of(text, pos.astype(np.int64))
    mask = class_mask(dfa, text, pos.astype(np.int64))
    lab = labels_np.astype(np.int64)
    loss_o, g_o = omlp.loss_and_grad(flat, states, wins, mask, lab, rnd=omlp.bf16_round)
    _, g_s = omlp.magnitudes(flat, states, wins, mask, lab, rnd=omlp.bf16_round)
    assert abs(loss - loss_o) <= 1e-4 * max(1.0, abs(loss_o)), (loss, loss_o)
    go, gg, gs = (omlp.unpack(x, states) for x in (g_o, g_gpu, g_s))
    for k in GRAD_TENSORS:
        check_scaled(f"{kind} grad {k}", gg[k].reshape(-1), go[k].reshape(-1), gs[k].reshape(-1))
    prop.close()
    m.close()


def test_gradient_skips_invalid_rows():
    """Rows whose label is not a state of their speculated set (0xffffffff,
    as after a byte outside the alphabet) or whose position lies beyond the
    text take no part: the gradient is the oracle's over the other rows,
    scaled by their share of the batch (the mean divides by the whole batch)."""
    dfa, text = head_case("motif35")
    states = dfa.num_states
    params = random_params(states, 10)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, params)
    rng = np.random.default_rng(5)
    B = 256
    pos = np.sort(rng.choice(np.arange(1, text.size), size=B, replace=False)).astype(np.uint64)
    labels_np, _ = oracle.states_at(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, text, pos)
    labels_np = labels_np.astype(np.uint32)
    bad_label = np.arange(0, B, 7)
    bad_pos = np.arange(3, B, 11)
    labels_np[bad_label] = 0xFFFFFFFF
    pos_dev = pos.copy()
    pos_dev[bad_pos] = text.size + 1 + np.arange(bad_pos.size, dtype=np.uint64) * 1000003
    td = dev(text)
    loss = prop.train_step(td, dev(pos_dev.view(np.int64)), dev(labels_np.view(np.int32)), lr=0.0,
                           weight_decay=0.0).item()
    g_gpu = omlp.unpack(prop.grad().astype(np.float64), states)
    keep = np.ones(B, dtype=bool)
    keep[bad_label] = False
    keep[bad_pos] = False
    pk = pos[keep].astype(np.int64)
    flat = oracle_params_bf16(params, states)
    wins, mask, lab = windows_of(text, pk), class_mask(dfa, text, pk), labels_np[keep].astype(np.int64)
    assert 0 < keep.sum() < B
    loss_o, g_o = omlp.loss_and_grad(flat, states, wins, mask, lab, rnd=omlp.bf16_round, denom=B)
    _, g_s = omlp.magnitudes(flat, states, wins, mask, lab, rnd=omlp.bf16_round, denom=B)
    assert abs(loss - loss_o) <= 1e-4 * max(1.0, abs(loss_o))
    go, gs = omlp.unpack(g_o, states), omlp.unpack(g_s, states)
    for k in GRAD_TENSORS:
        check_scaled(f"skipped rows grad {k}", g_gpu[k].reshape(-1), go[k].reshape(-1), gs[k].reshape(-1))
    prop.close()
    m.close()


def test_training_on_text_with_invalid_bytes():
    """A training text holding bytes outside the alphabet: the boundaries
    after them have no state and are left out of the labels; training runs,
    its loss and weights stay finite, and matching that text still reports
    the invalid byte."""
    dfa, text = W.motif_train_text(n=4 << 20)
    text = text.copy()
    rng = np.random.default_rng(8)
    text[rng.integers(1000, text.size - 1000, size=40)] = ord("N")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=2048)
    td = dev(text)
    prop, hist = P.train_proposal(m, td, W.mlp_init_params(dfa.num_states), steps=20, batch=1024, lr=2e-3,
                                  log_every=5, seed=3)
    say(f"[train invalid] {hist}")
    assert all(np.isfinite(l) for _, l in hist)
    assert np.all(np.isfinite(prop.params()))
    with pytest.raises(P.ParemError) as ei:
        m.match_learned(prop, td, 2)
    assert ei.value.status == P.PAREM_ESYMBOL
    prop.close()
    m.close()


def test_adamw_matches_oracle():
    """Three AdamW steps with seeded gradients (zeros, tiny and ordinary
    entries) against the oracle's update in float64 with the same fp32
    hyper-parameters. The GPU's update is fp32 arithmetic: a few roundings of
    the moments and the ratio (each 2^-24 relative), of the weight itself,
    and bias corrections rounded once to fp32, so per step the weight may
    differ by 2^-22 of itself plus 2^-19 of the step's size; the bound is
    summed over the steps taken."""
    dfa, text = head_case("motif35")
    states = dfa.num_states
    params = random_params(states, 12)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, params)
    n = prop.nparams
    rng = np.random.default_rng(77)
    lr, wd = np.float32(2e-3), np.float32(0.01)
    b1, b2, eps = np.float32(0.9), np.float32(0.999), np.float32(1e-8)
    w = prop.params().astype(np.float64)
    assert np.array_equal(w, params.astype(np.float64))
    mo = np.zeros(n)
    vo = np.zeros(n)
    bound = np.zeros(n)
    for step in range(1, 4):
        g = (rng.standard_normal(n) * np.exp(rng.uniform(-12, 2, n))).astype(np.float32)
        g[rng.random(n) < 0.05] = 0.0
        prop.apply_grad(dev(g), float(lr), float(wd))
        m_prev = mo
        w_prev = w
        w, mo, vo = omlp.adamw(w, g.astype(np.float64), mo, vo, step, float(lr), beta1=float(b1), beta2=float(b2),
                               eps=float(eps), wd=float(wd))
        mhat = (np.abs(b1 * m_prev) + (1 - float(b1)) * np.abs(g)) / (1 - float(b1) ** step)
        vhat = vo / (1 - float(b2) ** step)
        size = float(lr) * (mhat / (np.sqrt(vhat) + float(eps)) + float(wd) * np.abs(w_prev))
        bound += 2.0 ** -22 * np.abs(w) + 2.0 ** -19 * size
        got = prop.params().astype(np.float64)
        err = np.abs(got - w)
        say(f"[adamw] step {step}: max err/bound {float((err / np.maximum(bound, 1e-300)).max()):.3e}")
        assert np.all(err <= bound), (step, int(np.argmax(err - bound)))
    prop.close()
    m.close()


def test_training_lowers_loss_and_predicts():
    dfa, text = W.motif_train_text(n=16 << 20)
    states = dfa.num_states
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    td = dev(text)
    prop, hist = P.train_proposal(m, td, W.mlp_init_params(states), steps=300, batch=2048, lr=2e-3,
                                  log_every=50, seed=1)
    say(f"[train] {hist}")
    assert hist[-1][1] < 0.5 * hist[0][1]
    # held-out boundaries of the benchmark text distribution
    _, test_text = W.dna_motif(n=1 << 20, copies=100)
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


@pytest.mark.parametrize("kind", ["motif35", "dense1200", "sparse4096"])
def test_forward_logits_elementwise(kind):
    """Logits against the bf16-operand oracle (hidden activations rounded
    where the GPU rounds them), entry by entry within the scale bounds above;
    fused (35 states) and unfused (1200, 4096) inference alike."""
    dfa, text = head_case(kind)
    states = dfa.num_states
    params = random_params(states, 6)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, params)
    rng = np.random.default_rng(3)
    pos = np.sort(rng.choice(np.arange(1, text.size), size=256, replace=False)).astype(np.uint64)
    pos[:3] = [1, 5, 31]
    pos = np.sort(pos)
    got = prop.logits(dev(text), pos).cpu().numpy().astype(np.float64)
    flat = oracle_params_bf16(params, states)
    wins = windows_of(text, pos.astype(np.int64))
    full = np.ones((len(pos), states), dtype=bool)
    want, _ = omlp.forward(flat, states, wins, full, rnd=omlp.bf16_round)
    lab = np.zeros(len(pos), dtype=np.int64)
    zs, _ = omlp.magnitudes(flat, states, wins, full, lab, rnd=omlp.bf16_round)
    check_scaled(f"{kind} logits", got.reshape(-1), want.reshape(-1), zs.reshape(-1))
    prop.close()
    m.close()


def topm_check(dfa, text, prop, L, mm):
    """The selection is the oracle's top-m (ties: lower state id) of the
    GPU's own fp32 logits (the same precision decides on both sides); where
    the m-th and (m+1)-th best logits of the bf16-operand oracle are further
    apart than twice the tight logit bound (2^-10 of the scale, which the
    logit tests hold all but rare entries to), it is also the oracle's own
    top-m."""
    td = dev(text)
    sel, nsel = prop.select(td, L, mm)
    sel, nsel = sel.cpu().numpy().astype(np.int64), nsel.cpu().numpy()
    pos = np.arange(L, text.size, L, dtype=np.uint64)
    z = prop.logits(td, pos).cpu().numpy()
    allowed = class_mask(dfa, text, pos.astype(np.int64))
    want = omlp.topm(z, allowed, mm)
    flat = oracle_params_bf16(prop.params(), dfa.num_states)
    wins = windows_of(text, pos.astype(np.int64))
    zo, _ = omlp.forward(flat, dfa.num_states, wins, allowed, rnd=omlp.bf16_round)
    zs, _ = omlp.magnitudes(flat, dfa.num_states, wins, allowed, np.zeros(len(pos), dtype=np.int64),
                            rnd=omlp.bf16_round)
    want_o = omlp.topm(zo, allowed, mm)
    col = {c: j for j, c in enumerate(dfa.alphabet)}
    assert nsel[0] == 1 and sel[0, 0] == 0
    decided = 0
    for c in range(1, len(nsel)):
        lst = np.unique(dfa.table[:, col[int(text[c * L - 1])]])
        assert nsel[c] == min(mm, lst.size)
        got_states = sorted(lst[sel[c, :nsel[c]]].tolist())
        assert got_states == sorted(want[c - 1]), c
        if lst.size > mm:
            vals = np.sort(zo[c - 1, lst])[::-1]
            tol = 2 * TIGHT * float(zs[c - 1, lst].max())
            if vals[mm - 1] - vals[mm] > tol:
                decided += 1
                assert got_states == sorted(want_o[c - 1]), ("oracle logits", c)
    return decided


@pytest.mark.parametrize("mm", [1, 3, 16])
def test_topm_selection_matches_oracle(mm):
    dfa, text = head_case("motif35")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, random_params(dfa.num_states, 21))
    topm_check(dfa, text, prop, 256, mm)
    prop.close()
    m.close()


@pytest.mark.parametrize("kind,mm", [("dense1200", 1), ("dense1200", 4), ("dense1200", 16),
                                     ("sparse4096", 1), ("sparse4096", 4), ("sparse4096", 16)])
def test_topm_selection_wide_heads(kind, mm):
    """Heads over 64 states take the unfused path (layer GEMMs, then a top-m
    kernel over the class lists)."""
    dfa, text = head_case(kind)
    say(f"[case] top-m {kind} m={mm}")
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    prop = P.Proposal(m, random_params(dfa.num_states, 22))
    decided = topm_check(dfa, text, prop, 512, mm)
    say(f"[top-m] {kind} m={mm}: {decided} selections also decided by the oracle's logits")
    assert decided > 0
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
    dfa, text = W.dna_motif(n=4 << 20)
    got = learned_case("dna_motif untrained", dfa, text, random_params(dfa.num_states, 3), mm, chunk_len=2048)
    assert got.chunks == 2048
    if mm >= 16:
        assert got.rerun_chunks <= got.chunks


def test_learned_reruns_equal_misses():
    """m = 1 on the motif automaton (runs merge: every map is uniform): a chunk
    is walked again exactly when its true entry state was not selected."""
    dfa, text = W.dna_motif(n=2 << 20)
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
    dfa, text = W.dna_motif(n=n, copies=100)
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
    dfa, text = W.dna_motif(n=1 << 20, copies=200)
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
    dfa, train_text = W.motif_train_text(n=16 << 20)
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=2048)
    prop, hist = P.train_proposal(m, dev(train_text), W.mlp_init_params(dfa.num_states), steps=300, batch=2048,
                                  lr=2e-3, log_every=100, seed=2)
    _, text = W.dna_motif(n=8 << 20)
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


@pytest.mark.parametrize("kind,mm,L", [("sparse4096", 1, 1024), ("sparse4096", 4, 4096), ("dense1200", 4, 2048)])
def test_learned_exact_wide_heads(kind, mm, L):
    """Learned matches whose proposal head has more than 64 rows (unfused
    selection) are exact; untrained proposals miss often, so the re-walk
    path runs too."""
    dfa, text = head_case(kind)
    got = learned_case(f"wide head {kind}", dfa, text, random_params(dfa.num_states, 5), mm, chunk_len=L)
    say(f"[wide head] {kind} m={mm}: re-walked {got.rerun_chunks} of {got.chunks}")


def test_learned_rewalk_from_lookback_sets():
    """A handle compiled with lookback sets (as the tuner picks for dense
    4-symbol DFAs with thousands of states, whose speculated sets hold most
    states) walks chunks whose selection missed again from their lookback
    sets, not from the whole set: exact, and far fewer walks."""
    rng = np.random.default_rng(2048)
    dfa = W.random_dense_dfa(rng, 2000, b"ACGT", num_accepting=31)
    text = W.uniform_text(rng, b"ACGT", 2_000_003)
    params = random_params(dfa.num_states, 13)
    got = {}
    for look in (0, 64):
        m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=4096, lookback=look)
        prop = P.Proposal(m, params)
        r = m.match_learned(prop, dev(text), 2)
        want = oracle.walk_dfa(dfa, text)
        assert (r.final_state, r.accept, r.count) == (want.final_state, want.accept, want.count), look
        say(f"[relook] lookback={look}: walks {r.spec_runs}, re-walked {r.rerun_chunks} of {r.chunks}")
        got[look] = r
        prop.close()
        m.close()
    assert got[64].rerun_chunks > 0
    assert got[64].spec_runs * 5 < got[0].spec_runs
