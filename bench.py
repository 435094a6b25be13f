"""Benchmark: matched input GB/s of the speculative chunked DFA walk on one GPU.

Workload: the DNA motif search automaton (Sigma*.P for a random length-16
motif with 4 wildcard positions, subset construction) over 1 GiB of i.i.d.
ACGT text with 1e5 planted motif copies; the text is resident in HBM before
timing starts. A step is one complete match (walk + composition + result).

Prints one JSON line. ``value`` is the mean over the K timed steps between
two synchronisations; the per-step HIP-event times give the median and the
minimum. ``roofline`` describes the walk kernel (the dominant kernel):
algorithmic bytes per launch (text bytes read + chunk-map bytes written)
over its average duration, measured with HIP events recorded on the launch
stream around that kernel alone, beside the measured read ceiling of the
same bytes (one coalesced 16-byte-load pass). ``cpu_baseline`` times the CPU
oracle (sequential walk, one thread) on the host over the same text.

Further modes (``--modes``): the paper's scheme without merging, learned
speculation (with top-1 accuracy), PaREM against the Enumeration policy (on
the DNA text and on the paper's 9-state automaton at its five input
lengths), the small random 8-state configuration timed for latency, the
large sparse byte DFA, and the batch of 4096 uneven pairs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WALK_KERNEL = {1: "k_walk_byte", 2: "k_walk_byte", 3: "k_walk_kgram"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_traffic.json")
WALK_SOURCES = [os.path.join(ROOT, "paper_1412_1741_amd", "csrc", f)
                for f in ("parem_device.h", "parem_walk_kernels.h", "parem_walk.hip")]
TUNED_CACHE = os.path.join(ROOT, "paper_1412_1741_amd", "tuned", "batch_mi355x.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in WALK_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(n: int):
    """HBM bytes per walk launch from the committed counter runs, or None when
    the kernel source changed since they were taken or the size differs."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash() or int(t.get("text_bytes", -1)) != n:
        return None
    return int(t["fetch_bytes"] * t["fetch_scale"] + t["write_bytes"] * t["write_scale"])


def cpu_baseline(dfa, text, budget_s: float = 10.0):
    import oracle
    reps = 0
    t0 = time.perf_counter()
    res = None
    while True:
        res = oracle.walk_dfa(dfa, text)
        reps += 1
        if time.perf_counter() - t0 >= budget_s or reps >= 3:
            break
    dt = time.perf_counter() - t0
    gbs = reps * text.size / dt / 1e9
    return res, {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                 "sample": f"sequential oracle walk over the full {text.size} B text x{reps} "
                           f"({dt:.1f} s, single thread)"}


def event_times(fn, steps, stream, warmup=1):
    """Per-call milliseconds from HIP events recorded around each call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def summary(ms_list, nbytes):
    med, mn = statistics.median(ms_list), min(ms_list)
    return {"GBps_median": round(nbytes / (med * 1e-3) / 1e9, 2), "GBps_best": round(nbytes / (mn * 1e-3) / 1e9, 2),
            "ms_median": round(med, 5), "ms_min": round(mn, 5), "repeats": len(ms_list)}


def read_ceiling(dev, stream, steps):
    """The measured HBM read rate of the same bytes: one coalesced 16-byte-load
    pass per call (median over `steps` calls)."""
    import torch
    import paper_1412_1741_amd as P
    n = dev.numel() // 16 * 16
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    ms = event_times(lambda: P.parem_read_sweep(dev.data_ptr(), n, stream.cuda_stream, sink.data_ptr()), steps,
                     stream, warmup=2)
    return {"GBps": round(n / (statistics.median(ms) * 1e-3) / 1e9, 1), "bytes": n, "ms_median": round(
        statistics.median(ms), 5), "kernel": "k_read_sweep"}


def bench_small(args):
    """The small random 8-state DFA over 1 MiB, 1024 chunks: a latency
    configuration (the HBM time of 1 MiB is about 0.13 us)."""
    import torch
    import oracle
    import paper_1412_1741_amd as P
    import workloads as W
    dfa, text, chunks = W.random8()
    L = text.size // chunks
    dev = torch.from_numpy(text).cuda()
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=L)
    out = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    ms = event_times(lambda: m.match_async(dev, out), max(20, args.steps), stream, warmup=3)
    r = P.MatchResult.from_bytes(out.cpu().numpy().tobytes())
    want = oracle.walk_dfa(dfa, text)
    res = summary(ms, text.size)
    res.update({"us_median": round(statistics.median(ms) * 1e3, 2), "us_min": round(min(ms) * 1e3, 2),
                "chunks": r.chunks, "spec_runs": r.spec_runs, "text_bytes": int(text.size),
                "bit_exact_vs_oracle": (r.final_state, r.accept, r.count) == (want.final_state, want.accept,
                                                                               want.count)})
    m.close()
    return res


def bench_enum(args, dfa2, dev2):
    """PaREM's speculated sets against the Enumeration policy (every state for
    every chunk after the first), with and without merging of runs that meet:
    on the DNA text and on the paper's 9-state automaton at its five input
    lengths (uniform p,a,r,e,l text with the word planted)."""
    import torch
    import paper_1412_1741_amd as P
    import workloads as W
    stream = torch.cuda.current_stream()
    out = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    steps = max(5, args.steps // 2)

    def one(dfa, dev, policy, no_merge, group):
        m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, policy=policy, no_merge=no_merge,
                      group=group)
        ms = event_times(lambda: m.match_async(dev, out), steps, stream)
        r = P.MatchResult.from_bytes(out.cpu().numpy().tobytes())
        m.close()
        s = summary(ms, dev.numel())
        s.update({"spec_runs": r.spec_runs, "group": group})
        return s, (r.final_state, r.count)

    def compare(dfa, dev):
        # the paper's scheme (every run walks its whole chunk) at the best of
        # three lockstep widths per policy (a lane steps G runs per pass, so
        # the width decides how closely the time follows the run count);
        # merged runs at the default width
        res, keys = {}, set()
        for pol, pname in ((P.POLICY_PAREM, "parem"), (P.POLICY_ENUMERATE, "enumeration")):
            best = None
            for g in (2, 4, 16):
                s, key = one(dfa, dev, pol, True, g)
                keys.add(key)
                if best is None or s["ms_median"] < best["ms_median"]:
                    best = s
            res[f"{pname}_paper_scheme"] = best
            s, key = one(dfa, dev, pol, False, 0)
            res[f"{pname}_merged"] = s
            keys.add(key)
        res["enumeration_over_parem_time_paper_scheme"] = round(
            res["enumeration_paper_scheme"]["ms_median"] / res["parem_paper_scheme"]["ms_median"], 3)
        res["agree"] = len(keys) == 1
        return res

    out_all = {"dna_motif_1GiB": compare(dfa2, dev2)}
    log("enum: the paper's automaton at its input lengths")
    dfa1, text1 = W.paper_parallel(max(W.PAPER_LENGTHS))
    d1 = torch.from_numpy(text1).cuda()
    del text1
    for n in W.PAPER_LENGTHS:
        out_all[f"table1_{n}"] = compare(dfa1, d1[:n])
    del d1
    return out_all


def bench_sparse(args):
    """The large sparse byte DFA (4096 states, 256 columns) over Zipf text:
    GB/s per table layout and speculated-set choice; every variant must give
    the same result."""
    import torch

    import paper_1412_1741_amd as P
    import workloads as W

    log(f"sparse: generating {args.sparse_size} bytes")
    dfa, text = W.sparse4096(n=args.sparse_size)
    dev = torch.from_numpy(text).cuda()
    del text
    stream = torch.cuda.current_stream()
    out = {}
    ref = None
    agree = True
    S = P.LAYOUT_SPARSE_LDS
    for name, kw in (("hot_rows", {"layout": P.LAYOUT_HOT_LDS}), ("byte_l2", {"layout": P.LAYOUT_BYTE_GLOBAL}),
                     ("hot_rows_lookback64", {"layout": P.LAYOUT_HOT_LDS, "lookback": 64}),
                     ("sparse_rows", {"layout": S}),
                     ("sparse_rows_g2", {"layout": S, "group": 2}),
                     ("sparse_rows_g4", {"layout": S, "group": 4}),
                     ("sparse_rows_lookback4", {"layout": S, "lookback": 4}),
                     ("sparse_rows_L32k", {"layout": S, "chunk_len": 32768})):
        m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, **kw)
        res_t = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ms = event_times(lambda: m.match_async(dev, res_t), max(3, args.steps // 4), stream)
        r = P.MatchResult.from_bytes(res_t.cpu().numpy().tobytes())
        key = (r.final_state, r.accept, r.count)
        ref = ref or key
        agree &= key == ref
        d = m.describe()
        s = summary(ms, dev.numel())
        s.update({"GBps": s["GBps_median"], "layout": d["layout"], "chunks": r.chunks, "spec_runs": r.spec_runs,
                  "max_spec": d["max_spec"]})
        out[name] = s
        m.close()
    out["text_bytes"] = int(dev.numel())
    out["variants_agree"] = agree
    return out


def bench_batch(args):
    """The batched workload: uneven (DFA, text) pairs in one graph-captured
    run, options from the autotuner; a sample of pairs is matched again one
    by one (single-text path, each handle's own options) and must agree.
    Parity with the oracle is the tests' job."""
    import concurrent.futures as cf

    import torch

    import paper_1412_1741_amd as P
    import workloads as W
    from paper_1412_1741_amd.autotune import Autotuner

    specs = W.batch_specs()[: args.batch_pairs]
    log(f"batch: generating {len(specs)} pairs")
    t0 = time.perf_counter()
    order = np.argsort([s.text_len for s in specs])
    sample = set(int(i) for i in order[: len(order) // 2: 16]) | set(int(i) for i in order[-4:])
    dfas, devs, host = [], [], {}
    with cf.ThreadPoolExecutor(16) as ex:
        for i, (dfa, text) in enumerate(ex.map(W.batch_pair, specs)):
            dfas.append(dfa)
            devs.append(torch.from_numpy(text).cuda())
            if i in sample:
                host[i] = text.size
            if (i + 1) % 512 == 0:
                log(f"batch: {i + 1} pairs generated ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    tuner = Autotuner(cache_path=TUNED_CACHE, init_params=W.mlp_init_params,
                      log=lambda msg: log(f"tune {msg}"))
    t0 = time.perf_counter()
    matchers, opts, props, ms_ = tuner.plan(dfas, devs, proposals=True)
    plan_s = time.perf_counter() - t0
    if args.tune_out:
        tuner.cache_path = args.tune_out
        tuner.save()
    lens = [d.numel() for d in devs]
    b = P.Batch(matchers, lens, opts, props, ms_)
    out = torch.empty(len(devs) * P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    log("batch: capture + warm-up")
    b.run_async(devs, out, use_graph=True)
    torch.cuda.synchronize()
    ms_list = event_times(lambda: b.run_async(devs, out, use_graph=True), max(3, args.batch_steps), stream, warmup=0)
    ms = statistics.median(ms_list)
    got = P.Batch.results(out, len(devs))
    total = int(sum(lens))
    log(f"batch: single-text check of {len(host)} pairs")
    agree = True
    for i in host:
        r1 = matchers[i].match(devs[i])
        r = got[i]
        agree &= (r.final_state, r.accept, r.count) == (r1.final_state, r1.accept, r1.count)
    info = b.describe()
    b.close()
    for pr in props:
        if pr is not None:
            pr.close()
    for mm in matchers:
        mm.close()
    spec_runs = int(sum(r.spec_runs for r in got))
    # algorithmic bytes of a replay: every text byte once, the chunk-map
    # entries written by the walks (4 B each) and one class + one leader end
    # per chunk (4 B)
    alg = total + 4 * spec_runs + 4 * int(info["chunks"])
    learned_classes = {k: v["learned"] for k, v in tuner.cache.items() if "learned" in v}
    s = summary(ms_list, total)
    s.update({"GBps": s["GBps_median"], "ms": round(ms, 4), "pairs": len(devs), "text_bytes": total,
              "graph_nodes": info["graph_nodes"], "walk_launches": info["walk_launches"],
              "walk_items": info["walk_items"], "compose_levels": info["levels"], "chunks": info["chunks"],
              "workspace_bytes": info["workspace_bytes"], "spec_runs": spec_runs,
              "roofline": {"bound": "hbm", "alg_bytes_per_replay": alg,
                           "achieved": round(alg / (ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
              "invalid_pairs": int(sum(r.final_state == P.INVALID_STATE for r in got)),
              "learned_pairs": info["learned_pairs"], "learned_classes_tried": len(learned_classes),
              "learned_classes_chosen": sum(1 for v in learned_classes.values() if v.get("use")),
              "learned_vs_plain": {k: {"learned_ms": round(v["ms"], 4), "m": v["m"],
                                       "plain_ms": round(tuner.cache[k]["ms_per_copy"], 4),
                                       "rerun_share": v["rerun_share"]} for k, v in learned_classes.items()},
              "proposals_trained": tuner.trained, "train_seconds": round(tuner.train_seconds, 2),
              "tuned_classes": len(tuner.cache), "tune_seconds": round(tuner.seconds, 2),
              "tune_candidates_measured": tuner.measured, "plan_seconds": round(plan_s, 2),
              "generate_seconds": round(gen_s, 2), "single_text_checked_pairs": len(host),
              "single_text_checked_bytes": int(sum(host.values())), "agrees_with_single_text": agree})
    return s


def bench_learned(args, m, dfa, dev, stream, steps):
    """Learned speculation on the DNA text: training on 128 MiB of the same
    distribution (another seed), then m in the given list; top-1 accuracy of
    the proposal at the chunk boundaries of the benchmarked text."""
    import torch
    import paper_1412_1741_amd as P
    import workloads as W
    log("training the proposal")
    _, train_text = W.motif_train_text()
    tdev = torch.from_numpy(train_text).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop, hist = P.train_proposal(m, tdev, W.mlp_init_params(dfa.num_states), steps=args.train_steps,
                                  batch=4096, lr=2e-3, log_every=max(1, args.train_steps // 4), seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del tdev
    res, results = {}, {}
    n = dev.numel()
    for mm in [int(x) for x in args.learned_m.split(",") if x]:
        log(f"learned m={mm}")
        outl = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ms = event_times(lambda: m.match_learned_async(prop, dev, mm, outl), steps, stream)
        rl = P.MatchResult.from_bytes(outl.cpu().numpy().tobytes())
        results[f"learned_m{mm}"] = rl
        s = summary(ms, n)
        s.update({"GBps": s["GBps_median"], "ms": s["ms_median"], "spec_runs": rl.spec_runs,
                  "rerun_share": round(rl.rerun_chunks / max(rl.chunks, 1), 6)})
        res[f"learned_m{mm}"] = s
    # top-1 accuracy at the chunk boundaries the learned match uses
    L = n // max(results[next(iter(results))].chunks, 1) if results else 8192
    L = max(64, L // 64 * 64)
    truth = P.boundary_states(m, dev, L).cpu().numpy().view(np.uint32)
    sel, nsel = prop.select(dev, L, 1)
    sel = sel[:, 0].cpu().numpy().astype(np.int64)
    # the selected position indexes the chunk's speculated list (sorted ids):
    # recover the state from the column image of the byte before the chunk
    col = {c: j for j, c in enumerate(dfa.alphabet)}
    images = [np.unique(dfa.table[:, j]) for j in range(dfa.alphabet_size)]
    prev = dev[L - 1::L].cpu().numpy()[: truth.size - 1]
    chosen = np.asarray([images[col[int(x)]][s] for x, s in zip(prev, sel[1:truth.size])])
    top1 = float(np.mean(chosen == truth[1:]))
    res["learned_training"] = {"text_bytes": 128 << 20, "steps": args.train_steps, "batch": 4096,
                               "seconds": round(train_s, 3), "loss": [[a, round(b, 5)] for a, b in hist],
                               "top1_accuracy": round(top1, 5), "chunk_len": L}
    prop.close()
    return res, results


def bench_learned_wide(args):
    """Learned speculation at the full head width: the 4096-state sparse
    byte DFA over 1 GiB of its Zipf text (sparse rows), a proposal with 4096
    logits trained on 64 MiB of the same distribution (another seed), top-m
    in the given list against the plain walk of the same handle; top-1
    accuracy at the chunk boundaries."""
    import torch
    import paper_1412_1741_amd as P
    import workloads as W
    log("learned (4096 states): generating")
    dfa, text = W.sparse4096(n=args.wide_size)
    dev = torch.from_numpy(text).cuda()
    del text
    _, train_text = W.sparse4096_train_text()
    tdev = torch.from_numpy(train_text).cuda()
    del train_text
    stream = torch.cuda.current_stream()
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting)
    n = dev.numel()
    out = {"text_bytes": int(n), "dfa_states": int(dfa.num_states), "layout": m.describe()["layout"]}
    res_t = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    ms = event_times(lambda: m.match_async(dev, res_t), max(5, args.steps // 2), stream)
    plain = P.MatchResult.from_bytes(res_t.cpu().numpy().tobytes())
    s = summary(ms, n)
    s.update({"GBps": s["GBps_median"], "spec_runs": plain.spec_runs})
    out["plain"] = s
    log("learned (4096 states): training")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop, hist = P.train_proposal(m, tdev, W.mlp_init_params(dfa.num_states), steps=args.wide_train_steps,
                                  batch=4096, lr=2e-3, log_every=max(1, args.wide_train_steps // 4), seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del tdev
    agree = True
    chunks = plain.chunks
    for mm in [int(x) for x in args.learned_m.split(",") if x]:
        log(f"learned (4096 states) m={mm}")
        outl = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ms = event_times(lambda: m.match_learned_async(prop, dev, mm, outl), max(5, args.steps // 2), stream)
        rl = P.MatchResult.from_bytes(outl.cpu().numpy().tobytes())
        agree &= (rl.final_state, rl.accept, rl.count) == (plain.final_state, plain.accept, plain.count)
        chunks = rl.chunks
        s = summary(ms, n)
        s.update({"GBps": s["GBps_median"], "spec_runs": rl.spec_runs,
                  "rerun_share": round(rl.rerun_chunks / max(rl.chunks, 1), 6)})
        out[f"learned_m{mm}"] = s
    L = max(64, (n // max(chunks, 1)) // 64 * 64)
    truth = P.boundary_states(m, dev, L).cpu().numpy().view(np.uint32)
    sel, _ = prop.select(dev, L, 1)
    sel = sel[:, 0].cpu().numpy().astype(np.int64)
    images = [np.unique(dfa.table[:, j]) for j in range(dfa.alphabet_size)]
    prev = dev[L - 1::L].cpu().numpy()[: truth.size - 1]
    chosen = np.asarray([images[int(x)][s_] for x, s_ in zip(prev, sel[1:truth.size])])
    out["training"] = {"text_bytes": 64 << 20, "steps": args.wide_train_steps, "batch": 4096,
                       "seconds": round(train_s, 3), "loss": [[a, round(b, 5)] for a, b in hist],
                       "top1_accuracy": round(float(np.mean(chosen == truth[1:])), 5), "chunk_len": L}
    out["learned_agrees_with_plain"] = agree
    prop.close()
    m.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=1 << 30, help="text bytes")
    ap.add_argument("--chunk-len", type=int, default=0)
    ap.add_argument("--group", type=int, default=0)
    ap.add_argument("--layout", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-merge", action="store_true", help="walk every speculated run through its whole chunk")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="plain,paper,learned,wide,enum,small,sparse,batch",
                    help="comma list: plain (merged runs), paper (every run walks its chunk), learned, "
                         "wide (learned speculation over the 4096-state sparse DFA), "
                         "enum (PaREM vs Enumeration), small (8-state DFA, 1 MiB, latency), "
                         "sparse (4096-state byte DFA), batch (4096 uneven pairs)")
    ap.add_argument("--learned-m", default="1,4,16")
    ap.add_argument("--wide-size", type=int, default=1 << 30, help="text bytes of the 4096-state learned run")
    ap.add_argument("--wide-train-steps", type=int, default=200)
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--batch-pairs", type=int, default=4096, help="pairs of the batched workload")
    ap.add_argument("--sparse-size", type=int, default=1 << 32, help="text bytes of the sparse byte DFA workload")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--tune-out", default="", help="write the autotuner cache here (default: not written)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of --size bytes instead (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the walk shards by contiguous text segments; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        src = torch.randint(0, 255, (args.size,), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        print(json.dumps({"copy_bytes": args.size, "read_bytes": args.size, "write_bytes": args.size,
                          "ms": round(ms, 5), "GBps_read_plus_write": round(2 * args.size / ms / 1e6, 1)}))
        return

    import paper_1412_1741_amd as P
    import workloads as W

    log(f"generating workload n={args.size}")
    dfa, text = W.dna_motif(n=args.size)
    dev = torch.from_numpy(text).cuda()
    torch.cuda.synchronize()
    m = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=args.chunk_len,
                  group=args.group, layout=args.layout, tile=args.tile, no_merge=args.no_merge)
    desc = m.describe()
    ws = m.workspace(text.size)
    out = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def launch(ev_b=None, ev_e=None):
        P.parem_match_async_timed(m.handle, dev.data_ptr(), text.size, ws.data_ptr(), ws.numel(),
                                  stream.cuda_stream, out.data_ptr(), ev_b, ev_e)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        launch()
    torch.cuda.synchronize()
    first = P.MatchResult.from_bytes(out.cpu().numpy().tobytes())

    K = args.steps
    # whole-step throughput: K plain launches between two synchronisations
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    log(f"timing {K} steps")
    t_start.record(stream)
    for k in range(K):
        launch()
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_per_step = t_start.elapsed_time(t_end) / K
    # per-step times (median, minimum)
    step_ms = event_times(launch, K, stream, warmup=0)

    # walk kernel alone: events recorded around it inside each launch
    evb = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    eve = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in evb + eve:
        e.record(stream)  # creates the underlying hipEvent_t
    torch.cuda.synchronize()
    for k in range(K):
        launch(evb[k].cuda_event, eve[k].cuda_event)
    torch.cuda.synchronize()
    walk_ms = [evb[k].elapsed_time(eve[k]) for k in range(K)]
    walk_avg_ms = statistics.mean(walk_ms)
    res = P.MatchResult.from_bytes(out.cpu().numpy().tobytes())
    assert (res.final_state, res.count) == (first.final_state, first.count)
    log("read ceiling")
    ceiling = read_ceiling(dev, stream, K)

    n = text.size
    # per launch: text read + chunk maps written (4-byte packed entries, one
    # 2-byte class and one 2-byte leader end per chunk)
    alg_bytes = n + res.spec_runs * 4 + res.chunks * 4
    achieved = alg_bytes / (walk_avg_ms * 1e-3) / 1e9
    value = n / (ms_per_step * 1e-3) / 1e9
    plain = summary(step_ms, n)
    plain.update({"GBps": round(value, 2), "ms": round(ms_per_step, 4), "spec_runs": res.spec_runs,
                  "rerun_share": 0.0})
    modes = {"plain_merged": plain}
    results = {"plain_merged": res}
    wanted = set(args.modes.split(","))

    if "paper" in wanted:
        log("paper scheme (no merging)")
        mp = P.Matcher(dfa.table, dfa.alphabet, dfa.start, dfa.accepting, chunk_len=args.chunk_len,
                       group=16, layout=args.layout, tile=args.tile, no_merge=True)
        outp = torch.empty(P.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        ms = event_times(lambda: mp.match_async(dev, outp), max(5, K // 2), stream)
        rp = P.MatchResult.from_bytes(outp.cpu().numpy().tobytes())
        results["plain_paper"] = rp
        s = summary(ms, n)
        s.update({"GBps": s["GBps_median"], "ms": s["ms_median"], "spec_runs": rp.spec_runs, "rerun_share": 0.0})
        modes["plain_paper"] = s
        mp.close()

    if "learned" in wanted:
        lres, lresults = bench_learned(args, m, dfa, dev, stream, K)
        modes.update(lres)
        results.update(lresults)
        best = max((v["GBps"] for k, v in lres.items() if k.startswith("learned_m")), default=0.0)
        modes["learned_vs_plain"] = {"best_learned_GBps": best, "plain_merged_GBps": plain["GBps_median"],
                                     "plain_paper_GBps": modes.get("plain_paper", {}).get("GBps_median"),
                                     "learned_over_merged": round(best / plain["GBps_median"], 3),
                                     "learned_over_paper": round(best / modes["plain_paper"]["GBps_median"], 3)
                                     if "plain_paper" in modes else None}
    agree = all((r.final_state, r.accept, r.count) == (res.final_state, res.accept, res.count)
                for r in results.values())

    if "wide" in wanted:
        modes["learned_wide_sparse4096_1GiB"] = bench_learned_wide(args)
    if "enum" in wanted:
        log("PaREM vs Enumeration")
        modes["parem_vs_enumeration"] = bench_enum(args, dfa, dev)
    if "small" in wanted:
        log("small configuration (latency)")
        modes["random8_1MiB_1024_chunks"] = bench_small(args)
    if "sparse" in wanted:
        modes["sparse_byte_4096"] = bench_sparse(args)
    if "batch" in wanted:
        modes["batch_uneven_4096"] = bench_batch(args)

    cpu = None
    exact = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        ref, cpu = cpu_baseline(dfa, text)
        exact = all((ref.final_state, ref.accept, ref.count) == (r.final_state, r.accept, r.count)
                    for r in results.values())

    line = {
        "metric": "matched input GB/s & %HBM peak, learned vs plain speculation, bit-exact",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "dna_motif_1GiB", "text_bytes": n, "dfa_states": dfa.num_states,
                   "alphabet": 4, "mode": "plain", "chunk_len": int(n // max(res.chunks, 1)) if res.chunks else 0,
                   "chunks": res.chunks, "layout": desc["layout"], "max_spec": desc["max_spec"],
                   "spec_runs": res.spec_runs, "rerun_share": 0.0, "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
                   "ms_median": plain["ms_median"], "ms_min": plain["ms_min"],
                   "GBps_median": plain["GBps_median"], "GBps_best": plain["GBps_best"],
                   "bit_exact_vs_oracle": exact, "modes_agree": agree, "modes": modes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(n),
                     "kernel": WALK_KERNEL.get(desc["layout"], "walk"), "kernel_ms": round(walk_avg_ms, 5),
                     "kernel_ms_median": round(statistics.median(walk_ms), 5),
                     "alg_bytes_per_launch": alg_bytes, "read_ceiling": ceiling,
                     "frac_of_read_ceiling": round(achieved / ceiling["GBps"], 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    m.close()


if __name__ == "__main__":
    main()
