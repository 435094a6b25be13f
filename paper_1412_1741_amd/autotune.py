"""Autotuner of the batched launch: table layout, chunk length, lockstep group
and staged tile per size class, chosen by measurement on the GPU.

A size class groups pairs whose best options should agree: the alphabet
size, the number of states and the text length, each bucketed by powers of
four. For a new class the tuner takes the first pair of the batch that falls
in it and times candidates with ``parem_tune`` (a batch of copies of that
pair, replayed from a HIP graph), in two rounds:

  1. every table layout the DFA can use x speculated sets (Algorithm 1's,
     or lookback sets over 32, 256 or 2048 bytes), at the batch's automatic chunk
     length, 8 walks in lockstep and 128-byte tiles;
  2. for the winning layout and sets: chunk lengths {1/4, 1, 4} x the
     automatic one (clipped to 64 .. 8192 and to the text) x lockstep
     groups {4, 8, 16} x tiles {64, 128}.

Texts shorter than ``min_tune_bytes`` keep the defaults (the layout the
compile step picks, the automatic chunk length, lookback sets when a column
image is wide): they carry a negligible share of the bytes. Choices persist in a JSON cache keyed by class, so a workload is
tuned once per machine; ``seconds`` reports the time spent measuring.

For DFAs with at least ``learned_min_states`` states (1024) the tuner also
tries learned speculation when it is given ``init_params`` (a function of the
state count returning initial proposal weights): it trains a proposal on the
pair's own text for ``learned_steps`` AdamW steps (labels: the boundary
states of the text), times one learned match for top-m in {1, 4, 16}, and
keeps learned speculation for the class only when it beats the plain
choice's time per text. Pairs of such classes get a proposal trained on their
own text when the batch is planned.

Every candidate computes the same result (the sequential run): only speed
differs, so a choice never affects correctness.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import (LAYOUT_AUTO, LAYOUT_BYTE_GLOBAL, LAYOUT_BYTE_LDS, LAYOUT_CLASS_LDS, LAYOUT_HOT_LDS, LAYOUT_KGRAM_LDS,
               Matcher, parem_tune)

# Inside a batch a work item (256 chunks, one lane each) takes about as long
# as one lane needs for one chunk; longer chunks would raise throughput in
# isolation but leave a few long items at the end of the run.
MAX_CHUNK = 8192


def batch_chunk_len(n: int) -> int:
    """The batch's automatic chunk length: about 256 chunks, 64 B .. 8 KiB."""
    L = 64
    while L < 8192 and L * 256 < n:
        L *= 2
    return L


def _bucket4(x: int) -> int:
    return 0 if x <= 1 else int(math.floor(math.log(x, 4)))


def size_class(num_states: int, alphabet_size: int, n: int) -> str:
    return f"A{alphabet_size}/Q4^{_bucket4(num_states)}/N4^{_bucket4(n)}"


class Autotuner:
    def __init__(self, cache_path: str | None = None, min_tune_bytes: int = 16 << 10, target_bytes: int = 1 << 30,
                 reps: int = 2, max_copies: int = 256, measure: bool = True, log=None, init_params=None,
                 learned_min_states: int = 1024, learned_steps: int = 60):
        self.cache_path = cache_path
        self.log = log
        self.init_params = init_params
        self.learned_min_states = learned_min_states
        self.learned_steps = learned_steps
        self.trained = 0          # proposals trained while planning
        self.train_seconds = 0.0
        self.measure = measure  # False: classes missing from the cache keep the defaults
        self.min_tune_bytes = min_tune_bytes
        self.target_bytes = target_bytes
        self.reps = reps
        self.max_copies = max_copies
        self.cache: dict[str, dict] = {}
        self.seconds = 0.0
        self.measured = 0
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def save(self):
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    # -- measurement -------------------------------------------------------

    def _time(self, matcher: Matcher, text, cands):
        import torch
        n = text.numel()
        copies = int(max(1, min(self.max_copies, math.ceil(self.target_bytes / max(n, 1)))))
        t0 = time.perf_counter()
        ms, best = parem_tune(matcher.handle, text.data_ptr(), n, copies, cands, self.reps,
                              torch.cuda.current_stream().cuda_stream)
        self.seconds += time.perf_counter() - t0
        self.measured += len(cands)
        return ms, best

    def tune_pair(self, dfa, text) -> dict:
        """Measure the candidates for one (DFA, device text) pair."""
        n = text.numel()
        matchers = {}
        for lay in (LAYOUT_BYTE_GLOBAL, LAYOUT_BYTE_LDS, LAYOUT_KGRAM_LDS, LAYOUT_CLASS_LDS, LAYOUT_HOT_LDS):
            m = Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, layout=lay)
            if m.describe()["layout"] == lay:
                matchers[lay] = m
            else:
                m.close()
        L0 = batch_chunk_len(n)
        best = None
        for lay, m in matchers.items():
            cands = [{"chunk_len": L0, "group": 8, "tile": 128, "lookback": k} for k in (0, 32, 256, 2048)]
            ms, b = self._time(m, text, cands)
            if ms[b] > 0 and (best is None or ms[b] < best[0]):
                best = (ms[b], lay, cands[b]["lookback"])
        _, lay, k = best
        Ls = sorted({min(MAX_CHUNK, max(64, int(L0 * f))) for f in (0.25, 1, 4)})
        Ls = [L for L in Ls if L == L0 or L <= max(64, n)]
        cands = [{"chunk_len": L, "group": g, "tile": t, "lookback": k} for L in Ls for g in (4, 8, 16)
                 for t in (64, 128)]
        ms, b = self._time(matchers[lay], text, cands)
        for m in matchers.values():
            m.close()
        choice = {"layout": lay, **cands[b], "ms_per_copy": ms[b],
                  "bytes": int(n), "GBps": round(n / (ms[b] * 1e-3) / 1e9, 2) if ms[b] > 0 else None}
        if self.init_params is not None and dfa.num_states >= self.learned_min_states:
            choice["learned"] = self._tune_learned(dfa, text, cands[b], ms[b])
        return choice

    def _train(self, matcher, dfa, text):
        from . import train_proposal
        t0 = time.perf_counter()
        prop, _ = train_proposal(matcher, text, self.init_params(dfa.num_states), steps=self.learned_steps,
                                 batch=2048, lr=2e-3, seed=1)
        self.train_seconds += time.perf_counter() - t0
        self.trained += 1
        return prop

    def _tune_learned(self, dfa, text, plain_opts, plain_ms):
        """Time learned speculation (one match per top-m) against the plain choice."""
        import torch
        from . import Batch
        m0 = Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
        t0 = time.perf_counter()
        prop = self._train(m0, dfa, text)
        opts = [{"chunk_len": int(plain_opts["chunk_len"]), "group": int(plain_opts["group"]),
                 "tile": int(plain_opts["tile"])}]
        res = {}
        for mm in (1, 4, 16):
            b = Batch([m0], [text.numel()], opts, [prop], [mm])
            out = b.run_async([text], use_graph=True)  # capture + warm-up
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(self.reps):
                b.run_async([text], out, use_graph=True)
            e1.record()
            torch.cuda.synchronize()
            r = Batch.results(out, 1)[0]
            res[mm] = (e0.elapsed_time(e1) / self.reps, r.rerun_chunks / max(r.chunks, 1))
            b.close()
        prop.close()
        m0.close()
        self.seconds += time.perf_counter() - t0
        best = min(res, key=lambda k: res[k][0])
        return {"m": best, "ms": res[best][0], "rerun_share": round(res[best][1], 5),
                "ms_by_m": {str(k): round(v[0], 4) for k, v in res.items()},
                "use": bool(res[best][0] < plain_ms)}

    # -- planning ------------------------------------------------------------

    @staticmethod
    def default(dfa) -> tuple[int, dict]:
        """Untuned pairs: the compile step's layout; lookback sets over 256
        bytes when a column image is large (speculation would be costly)."""
        t = np.asarray(dfa.table)
        widest = max(np.unique(t[:, j]).size for j in range(t.shape[1]))
        return LAYOUT_AUTO, ({"chunk_len": 0, "lookback": 256} if widest > 64 else {})

    def choose(self, dfa, text) -> tuple[int, dict]:
        """(layout, options) for one pair; tunes its class on first sight."""
        n = text.numel()
        if n < self.min_tune_bytes:
            return self.default(dfa)
        key = size_class(dfa.num_states, dfa.alphabet_size, n)
        if key not in self.cache:
            if not self.measure:
                return self.default(dfa)
            self.cache[key] = self.tune_pair(dfa, text)
            if self.log:
                self.log(f"{key}: {self.cache[key]} ({self.seconds:.1f} s so far)")
        c = self.cache[key]
        if (self.measure and self.init_params is not None and dfa.num_states >= self.learned_min_states
                and "learned" not in c):
            c["learned"] = self._tune_learned(dfa, text, c, c["ms_per_copy"])
            if self.log:
                self.log(f"{key} learned: {c['learned']} (plain {c['ms_per_copy']:.4f} ms)")
        return int(c["layout"]), {"chunk_len": int(c["chunk_len"]), "group": int(c["group"]),
                                  "tile": int(c["tile"]), "lookback": int(c.get("lookback", 0))}

    def learned_m(self, dfa, text) -> int:
        """top-m when learned speculation was chosen for the pair's class, else 0."""
        n = text.numel()
        if self.init_params is None or n < self.min_tune_bytes or dfa.num_states < self.learned_min_states:
            return 0
        c = self.cache.get(size_class(dfa.num_states, dfa.alphabet_size, n), {})
        lr = c.get("learned")
        return int(lr["m"]) if lr and lr.get("use") else 0

    def plan(self, dfas, texts, proposals: bool = False):
        """Matchers compiled with the chosen layouts and per-pair options; with
        ``proposals``, also (proposals, m) for the batch (None / 0 for plain
        pairs), training a proposal for every pair whose class chose learned
        speculation."""
        matchers, opts, props, ms = [], [], [], []
        for dfa, text in zip(dfas, texts):
            lay, o = self.choose(dfa, text)
            m = Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, layout=lay)
            matchers.append(m)
            opts.append(o if o else {"chunk_len": 0})
            mm = self.learned_m(dfa, text) if proposals else 0
            props.append(self._train(m, dfa, text) if mm else None)
            ms.append(mm)
        if proposals:
            return matchers, opts, props, ms
        return matchers, opts
