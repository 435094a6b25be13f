"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module builds automata and texts only. It holds none of the matching
arithmetic (no DFA walk, no speculation, no composition): the automata are
made by explicit construction (random tables, or the subset construction of a
motif-search NFA) and the texts by seeded random draws. Both the CPU oracle
and the HIP path consume what it returns; neither is imported here.

Workload shapes (the five workloads the path is measured and tested on):

* ``random8``: random 8-state DFA over {A,C,G,T}, 1 MiB uniform text, 1024
  chunks.
* ``dna_motif``: Sigma*.P search automaton for a random length-16 DNA motif with
  4 wildcard positions (17-state NFA, subset construction), 1 GiB uniform
  ACGT text with 1e5 planted motif copies.
* ``sparse4096``: 4096-state sparse byte DFA (4 explicit transitions per state,
  the rest to state 0), 4 GiB Zipf(1.1) text over 64 byte values.
* ``motif_train``: training text for the learned proposal: the DNA motif distribution,
  another seed, 128 MiB.
* ``batch_pairs``: 4096 (DFA, text) pairs of log-uniform sizes.

The paper gives no input text (its five strings of 6.69e7..1.07e9 characters
are unspecified), so these stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ACGT = b"ACGT"


@dataclass
class Dfa:
    """A total DFA: ``table[q, j]`` is the successor of state ``q`` on the
    byte ``alphabet[j]``; ``accepting`` lists the final states."""

    table: np.ndarray            # [Q, A] unsigned integer
    alphabet: bytes              # A distinct bytes, column order
    start: int
    accepting: np.ndarray        # sorted unique uint32 state ids
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_states(self) -> int:
        return int(self.table.shape[0])

    @property
    def alphabet_size(self) -> int:
        return int(self.table.shape[1])

    def final_mask(self) -> np.ndarray:
        m = np.zeros(self.num_states, dtype=np.uint8)
        m[self.accepting] = 1
        return m


# ---------------------------------------------------------------------------
# texts
# ---------------------------------------------------------------------------

_BLOCK = 1 << 26  # generate large texts in 64 MiB blocks to bound host memory


def _random_bytes(rng: np.random.Generator, m: int) -> np.ndarray:
    """``m`` i.i.d. uniform bytes (64-bit draws: several times faster than
    Generator.bytes)."""
    k = (m + 7) // 8
    return rng.integers(0, 2 ** 64 - 1, size=k, dtype=np.uint64, endpoint=True).view(np.uint8)[:m]


def uniform_text(rng: np.random.Generator, alphabet: bytes, n: int) -> np.ndarray:
    """``n`` bytes drawn i.i.d. uniformly from ``alphabet``."""
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    a = len(alpha)
    out = np.empty(n, dtype=np.uint8)
    if n == 0:
        return out
    if a == 4:
        # each random byte carries four independent 2-bit draws
        lut = np.empty((256, 4), dtype=np.uint8)
        v = np.arange(256)
        for k in range(4):
            lut[:, k] = alpha[(v >> (2 * k)) & 3]
        lut32 = lut.reshape(-1).view(np.uint32)
        q = n // 4
        pos = 0
        while pos < q:
            m = min(_BLOCK, q - pos)
            rb = _random_bytes(rng, m)
            out[4 * pos:4 * (pos + m)].view(np.uint32)[:] = lut32[rb]
            pos += m
        tail = n - 4 * q
        if tail:
            out[4 * q:] = alpha[rng.integers(0, 4, size=tail)]
        return out
    if a == 256:
        # every byte value is in the alphabet: uniform bytes are uniform symbols
        pos = 0
        while pos < n:
            m = min(_BLOCK, n - pos)
            out[pos:pos + m] = _random_bytes(rng, m)
            pos += m
        return out
    # other sizes: a random byte b < (256 // a) * a gives symbol b % a
    # (rejection sampling keeps the draws exactly uniform and independent)
    lim = (256 // a) * a
    lut = alpha[np.arange(lim) % a]
    pos = 0
    while pos < n:
        m = min(_BLOCK, n - pos)
        rb = _random_bytes(rng, m + m // 8 + 64)
        rb = rb[rb < lim][: m]
        out[pos:pos + rb.size] = lut[rb]
        pos += rb.size
    return out

def zipf_lut(symbols: np.ndarray, s: float = 1.1) -> np.ndarray:
    """65536-entry inverse-CDF table: a uniform 16-bit draw ``u`` maps to
    ``lut[u]``; symbol of rank k (1-based) has weight k**-s. Probabilities are
    quantised to multiples of 2**-16 by rounding the CDF."""
    k = np.arange(1, len(symbols) + 1, dtype=np.float64)
    w = k ** (-s)
    cdf = np.cumsum(w) / w.sum()
    edges = np.rint(cdf * 65536.0).astype(np.int64)
    edges[-1] = 65536
    lut = np.empty(65536, dtype=np.uint8)
    lo = 0
    for i, hi in enumerate(edges):
        lut[lo:hi] = symbols[i]
        lo = max(lo, hi)
    return lut


def zipf_text(rng: np.random.Generator, symbols: np.ndarray, n: int, s: float = 1.1,
              threads: int = 16) -> np.ndarray:
    """``n`` bytes i.i.d. Zipf(s) over ``symbols`` (rank order). Each 64 MiB
    block draws from its own generator, seeded from ``rng``, so blocks are
    generated by several threads with the same result."""
    lut = zipf_lut(symbols, s)
    out = np.empty(n, dtype=np.uint8)
    nblk = (n + _BLOCK - 1) // _BLOCK
    seeds = rng.integers(0, 2 ** 63, size=nblk)

    def block(k):
        pos = k * _BLOCK
        m = min(_BLOCK, n - pos)
        u = _random_bytes(np.random.default_rng(int(seeds[k])), 2 * m).view(np.uint16)
        out[pos:pos + m] = lut[u]

    if nblk <= 1:
        for k in range(nblk):
            block(k)
    else:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(min(threads, nblk)) as ex:
            list(ex.map(block, range(nblk)))
    return out


# ---------------------------------------------------------------------------
# automata
# ---------------------------------------------------------------------------

def random_dense_dfa(rng: np.random.Generator, num_states: int, alphabet: bytes,
                     num_accepting: int = 1, name: str = "random") -> Dfa:
    """Every entry drawn uniformly from [0, num_states)."""
    a = len(alphabet)
    table = rng.integers(0, num_states, size=(num_states, a)).astype(np.uint32)
    acc = np.sort(rng.choice(num_states, size=min(num_accepting, num_states), replace=False)).astype(np.uint32)
    return Dfa(table, bytes(alphabet), 0, acc, name)


def sparse_dfa(rng: np.random.Generator, num_states: int, alphabet: bytes,
               explicit_lo: int, explicit_hi: int, accepting: np.ndarray,
               explicit_cols: np.ndarray | None = None, name: str = "sparse") -> Dfa:
    """Each state gets k in [explicit_lo, explicit_hi] (capped at the alphabet
    size) explicit transitions to uniform targets; every other entry goes to
    state 0. ``explicit_cols`` restricts which columns may be explicit."""
    a = len(alphabet)
    cols_pool = np.arange(a) if explicit_cols is None else np.asarray(explicit_cols)
    p = len(cols_pool)
    table = np.zeros((num_states, a), dtype=np.uint32)
    k = rng.integers(explicit_lo, explicit_hi + 1, size=num_states)
    k = np.minimum(k, p)
    # choose k columns without replacement per state: rank a random key matrix
    keys = rng.random((num_states, p))
    order = np.argsort(keys, axis=1)
    sel = np.arange(p)[None, :] < k[:, None]
    rows = np.repeat(np.arange(num_states), p).reshape(num_states, p)
    cols = cols_pool[order]
    targets = rng.integers(0, num_states, size=(num_states, p)).astype(np.uint32)
    table[rows[sel], cols[sel]] = targets[sel]
    acc = np.sort(np.asarray(accepting, dtype=np.uint32))
    return Dfa(table, bytes(alphabet), 0, acc, name)


def motif_dfa(motif: bytes, wild: np.ndarray, alphabet: bytes = ACGT) -> Dfa:
    """Search automaton for Sigma*.P by subset construction.

    NFA: states 0..m; state 0 loops on every symbol; state i moves to i+1 on
    motif[i] (on every symbol where ``wild[i]``); state m is final. DFA states
    are the reachable NFA state sets, discovered breadth-first from {0} with
    the columns taken in alphabet order; ids follow discovery order."""
    m = len(motif)
    syms = list(alphabet)

    def step(sset: frozenset, c: int) -> frozenset:
        nxt = {0}
        for i in sset:
            if i < m and (wild[i] or motif[i] == c):
                nxt.add(i + 1)
        return frozenset(nxt)

    start = frozenset({0})
    ids = {start: 0}
    order = [start]
    rows = []
    head = 0
    while head < len(order):
        cur = order[head]
        head += 1
        row = []
        for c in syms:
            nx = step(cur, c)
            if nx not in ids:
                ids[nx] = len(order)
                order.append(nx)
            row.append(ids[nx])
        rows.append(row)
    table = np.asarray(rows, dtype=np.uint32)
    acc = np.asarray([i for i, s in enumerate(order) if m in s], dtype=np.uint32)
    return Dfa(table, bytes(alphabet), 0, acc, "motif",
               meta={"motif": bytes(motif), "wild": np.asarray(wild, dtype=bool)})


def plant_motifs(rng: np.random.Generator, text: np.ndarray, motif: bytes, wild: np.ndarray,
                 copies: int, alphabet: bytes = ACGT) -> np.ndarray:
    """Write ``copies`` motif instances at uniform offsets in [0, N-len];
    wildcard positions get i.i.d. symbols; later copies overwrite earlier."""
    m = len(motif)
    n = len(text)
    if n < m or copies == 0:
        return np.zeros(0, dtype=np.int64)
    offs = rng.integers(0, n - m + 1, size=copies)
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    fill = alpha[rng.integers(0, len(alpha), size=(copies, m))]
    base = np.frombuffer(motif, dtype=np.uint8)
    w = np.asarray(wild, dtype=bool)
    pieces = np.where(w[None, :], fill, base[None, :])
    for j in range(copies):
        o = offs[j]
        text[o:o + m] = pieces[j]
    return offs


# ---------------------------------------------------------------------------
# the five configurations
# ---------------------------------------------------------------------------

SEED_RANDOM8 = 1
SEED_MOTIF = 2
SEED_SPARSE = 3
SEED_TRAIN = 4
SEED_BATCH = 5


def random8(seed: int = SEED_RANDOM8, n: int = 1 << 20):
    """Random 8x4 uint8 table over ACGT, start 0, F={7}; i.i.d. text."""
    rng = np.random.default_rng(seed)
    table = rng.integers(0, 8, size=(8, 4), dtype=np.uint8)
    dfa = Dfa(table, ACGT, 0, np.asarray([7], dtype=np.uint32), "random8")
    text = uniform_text(rng, ACGT, n)
    return dfa, text, 1024


# Table I of the paper (Section II-C): the 9-state automaton that finds the
# word "parallel" over the symbols p, a, r, e, l (columns in that order).
PAREL = b"parel"
TABLE1 = np.asarray([[1, 0, 0, 0, 0], [1, 2, 0, 0, 0], [1, 0, 3, 0, 0], [1, 4, 0, 0, 0], [1, 0, 0, 0, 5],
                     [1, 0, 0, 0, 6], [1, 0, 0, 7, 0], [1, 0, 0, 0, 8], [1, 0, 0, 0, 0]], dtype=np.uint8)
# input lengths of the paper's measurements (Section IV-A)
PAPER_LENGTHS = (66_900_000, 134_000_000, 268_000_000, 536_000_000, 1_070_000_000)


def paper_parallel(n: int, seed: int = 1412, copies_per_mib: int = 64):
    """Table I's automaton (F = {8}) and n i.i.d. uniform symbols over
    p,a,r,e,l with the word "parallel" planted at random offsets (the paper
    does not give its input strings)."""
    rng = np.random.default_rng([seed, n])
    dfa = Dfa(TABLE1.copy(), PAREL, 0, np.asarray([8], dtype=np.uint32), "table1")
    text = uniform_text(rng, PAREL, n)
    k = max(1, n * copies_per_mib >> 20)
    word = np.frombuffer(b"parallel", dtype=np.uint8)
    for o in rng.integers(0, max(1, n - 8), size=k):
        text[o:o + 8] = word[: max(0, min(8, n - int(o)))]
    return dfa, text


def motif_spec(seed: int):
    rng = np.random.default_rng([seed, 0xD7A])
    alpha = np.frombuffer(ACGT, dtype=np.uint8)
    motif = bytes(alpha[rng.integers(0, 4, size=16)])
    wild = np.zeros(16, dtype=bool)
    wild[rng.choice(16, size=4, replace=False)] = True
    return motif, wild


def dna_motif_dfa(seed: int = SEED_MOTIF) -> Dfa:
    motif, wild = motif_spec(seed)
    d = motif_dfa(motif, wild)
    d.name = "dna_motif"
    return d


def dna_motif(seed: int = SEED_MOTIF, n: int = 1 << 30, copies: int | None = None,
            text_seed: int | None = None):
    """Motif DFA plus i.i.d. ACGT text with planted copies (1e5 per GiB)."""
    dfa = dna_motif_dfa(seed)
    rng = np.random.default_rng([seed if text_seed is None else text_seed, 0x7E47])
    text = uniform_text(rng, ACGT, n)
    if copies is None:
        copies = int(round(1e5 * n / float(1 << 30)))
    plant_motifs(rng, text, dfa.meta["motif"], dfa.meta["wild"], copies)
    return dfa, text


def sparse4096_dfa(seed: int = SEED_SPARSE, num_states: int = 4096):
    rng = np.random.default_rng([seed, 0x5A])
    symbols = rng.choice(256, size=64, replace=False).astype(np.uint8)  # Zipf rank order
    alphabet = bytes(range(256))
    acc = np.sort(rng.choice(np.arange(1, num_states), size=16, replace=False))
    d = sparse_dfa(rng, num_states, alphabet, 4, 4, acc, explicit_cols=symbols, name="sparse4096")
    d.table = d.table.astype(np.uint16)
    d.meta["symbols"] = symbols
    return d


def sparse4096(seed: int = SEED_SPARSE, n: int = 1 << 32, num_states: int = 4096):
    dfa = sparse4096_dfa(seed, num_states)
    rng = np.random.default_rng([seed, 0x7E47])
    text = zipf_text(rng, dfa.meta["symbols"], n)
    return dfa, text


def sparse4096_train_text(seed: int = SEED_TRAIN, n: int = 64 << 20, dfa_seed: int = SEED_SPARSE):
    """The sparse byte DFA's text distribution (Zipf over its 64 symbols),
    drawn from another seed: training text for a 4096-row proposal."""
    dfa = sparse4096_dfa(dfa_seed)
    rng = np.random.default_rng([seed, 0x7E48])
    return dfa, zipf_text(rng, dfa.meta["symbols"], n)


def motif_train_text(seed: int = SEED_TRAIN, n: int = 128 << 20, dfa_seed: int = SEED_MOTIF):
    """The DNA motif text distribution for the same motif, drawn from another seed."""
    dfa, text = dna_motif(dfa_seed, n=n, text_seed=seed)
    return dfa, text


@dataclass
class PairSpec:
    index: int
    num_states: int
    alphabet_size: int
    text_len: int


def batch_specs(seed: int = SEED_BATCH, pairs: int = 4096,
                  q_range=(4, 4096), len_range=(1 << 10, 64 << 20)):
    rng = np.random.default_rng([seed, 0xBA7C])
    q = np.floor(np.exp(rng.uniform(math.log(q_range[0]), math.log(q_range[1]), size=pairs))).astype(np.int64)
    a = rng.choice(np.asarray([4, 20, 256]), size=pairs)
    ln = np.floor(np.exp(rng.uniform(math.log(len_range[0]), math.log(len_range[1]), size=pairs))).astype(np.int64)
    return [PairSpec(i, int(q[i]), int(a[i]), int(ln[i])) for i in range(pairs)]


def batch_pair(spec: PairSpec, seed: int = SEED_BATCH, with_text: bool = True):
    """Regenerates pair ``spec.index`` alone (its own seed stream)."""
    rng = np.random.default_rng([seed, 0x9A1, spec.index])
    alphabet = bytes(rng.choice(256, size=spec.alphabet_size, replace=False).astype(np.uint8))
    acc = rng.choice(spec.num_states, size=math.ceil(spec.num_states / 64), replace=False)
    dfa = sparse_dfa(rng, spec.num_states, alphabet, 4, 16, acc, name=f"batch[{spec.index}]")
    if spec.num_states <= 256:
        dfa.table = dfa.table.astype(np.uint8)
    elif spec.num_states <= 65536:
        dfa.table = dfa.table.astype(np.uint16)
    text = uniform_text(rng, alphabet, spec.text_len) if with_text else None
    return dfa, text


def random_case(rng: np.random.Generator, max_states: int = 64, max_alpha: int = 8,
                max_len: int = 4096):
    """A small random total DFA and text for fuzzing."""
    q = int(rng.integers(1, max_states + 1))
    a = int(rng.integers(1, max_alpha + 1))
    alphabet = bytes(rng.choice(256, size=a, replace=False).astype(np.uint8))
    dfa = random_dense_dfa(rng, q, alphabet, num_accepting=int(rng.integers(0, q + 1)))
    dfa.start = int(rng.integers(0, q))
    n = int(rng.integers(0, max_len + 1))
    text = uniform_text(rng, alphabet, n)
    return dfa, text


# ---------------------------------------------------------------------------
# initial weights of the learned proposal (an input like any other)
# ---------------------------------------------------------------------------

MLP_WINDOW, MLP_EMB, MLP_HID = 32, 16, 256


def mlp_param_shapes(states: int):
    """Flat parameter layout: emb [256,16], W1 [256,512], b1 [256],
    W2 [256,256], b2 [256], W3 [states,256], b3 [states]."""
    return [("emb", (256, MLP_EMB)), ("W1", (MLP_HID, MLP_WINDOW * MLP_EMB)), ("b1", (MLP_HID,)),
            ("W2", (MLP_HID, MLP_HID)), ("b2", (MLP_HID,)), ("W3", (states, MLP_HID)), ("b3", (states,))]


def mlp_init_params(states: int, seed: int = 11) -> np.ndarray:
    """Seeded initial weights (float32): N(0, 1/fan_in) matrices, N(0, 1)
    embedding, zero biases."""
    rng = np.random.default_rng([seed, 0x3117])
    parts = []
    for name, shape in mlp_param_shapes(states):
        if name.startswith("b"):
            parts.append(np.zeros(shape))
        elif name == "emb":
            parts.append(rng.standard_normal(shape))
        else:
            parts.append(rng.standard_normal(shape) / math.sqrt(shape[1]))
    return np.concatenate([x.reshape(-1) for x in parts]).astype(np.float32)
