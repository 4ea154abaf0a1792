#!/usr/bin/env python3
"""Throughput of the chunk-parallel SLPF parser on one MI355X.

One step = one full parse of the workload text already resident in HBM:
speculative reach, join, build & merge (the SLPF is written), and the tree
count.  Prints one JSON line (rank 0).  The CPU baseline is the serial oracle
on a bounded prefix of the same text, timed on this host.

Workload (the single-RE large-text configuration): a seeded random RE tree of
depth 7 with 40 operators over the 26 lowercase letters (seed 23, 304
segments, 336 forward-table states, W = 5 words per column), a 256 MiB text
sampled from its language, then 5 % of the bytes overwritten by seeded
random-byte blocks (64..4096 bytes).  The clean text (no corruption) is timed
as a companion.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "parsed GB/s per GPU + % HBM roofline, bit-exact SLPF; p50/p99 latency when served"
HBM_PEAK_GBS = 8000.0
RE_SEED, TEXT_SEED, CORRUPT_SEED = 23, 23, 24
TEXT_BYTES = 1 << 28
KERNEL_SOURCES = ["paper_2503_06763_amd/csrc/kernels.hpp", "paper_2503_06763_amd/csrc/slpf.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload, khash):
    """HBM bytes per k_build launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "k_build_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != khash:
        return None
    return t.get("bytes_per_launch")


def make_text(n, corrupt):
    from gen import regen, textgen
    tree = regen.random_re(RE_SEED)
    text = textgen.sample_text(tree, TEXT_SEED, n)
    if corrupt:
        text = textgen.corrupt(text, CORRUPT_SEED, frac=0.05, block=(64, 4096))
    return regen.to_re(tree), text


def run_gpu(parser, text_np, steps, warmup, chunk_bytes):
    import numpy as np
    import torch
    import paper_2503_06763_amd as S
    dev = torch.device("cuda:0")
    n = text_np.size
    text = torch.from_numpy(text_np).to(dev)
    W = parser.W
    cols = torch.empty((n + 1, W), dtype=torch.int64, device=dev)
    sc = torch.empty(3, dtype=torch.int64, device=dev)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(S.NUM_PHASE_EVENTS)] for _ in range(steps)]
    for _ in range(warmup):
        parser.parse_into(text, n, cols, sc, chunk_bytes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        parser.parse_into(text, n, cols, sc, chunk_bytes, events=evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    phase = {name: sum(e[i].elapsed_time(e[i + 1]) for e in evs) / steps
             for i, name in enumerate(S.PHASES)}
    s = sc.cpu().numpy().view(np.uint64)
    return ms, phase, (int(s[0]), int(s[1]), int(s[2])), cols


def cpu_baseline(pat, text_np, sample_bytes):
    from oracle.oracle import Oracle
    o = Oracle(pat)
    x = text_np[:sample_bytes].tobytes()
    t0 = time.perf_counter()
    o.parse(x)
    dt = time.perf_counter() - t0
    return {"value": round(len(x) / dt / 1e9, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "first %d bytes of the same text, serial NFA parser (Fig. serialparser) "
                      "with in-place intersection and tree count, single thread, %.1f s" % (len(x), dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--bytes", type=int, default=TEXT_BYTES)
    ap.add_argument("--chunk-bytes", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=32 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-companion", action="store_true")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="after timing, copy this many bytes device-to-device (scale reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2503_06763_amd as S
    S.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    t0 = time.perf_counter()
    pat, text = make_text(args.bytes, corrupt=True)
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    parser = S.Parser(pat)
    compile_ms = (time.perf_counter() - t0) * 1e3
    n, W = text.size, parser.W
    print("workload: n=%d W=%d segments=%d fwd=%d rev=%d placement=%d gen %.1fs" % (
        n, W, parser.nseg, parser.info.fwd_states, parser.info.rev_states, parser.info.placement, gen_s),
        file=sys.stderr, flush=True)
    ms, phase, scal, _ = run_gpu(parser, text, args.steps, args.warmup, args.chunk_bytes)
    print("timed: %.3f ms/step, phases %s, scalars %s" % (ms, phase, scal), file=sys.stderr, flush=True)
    algo = n + (n + 1) * 8 * W
    build_ms = phase["build"]
    khash = kernel_hash()
    roof = {"bound": "hbm", "achieved": round(algo / (build_ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(algo / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles("single_re_large", khash), "kernel": "k_build",
            "algorithmic_bytes": algo}
    out = {
        "metric": METRIC, "value": round(n / (ms * 1e-3) / 1e9, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "single-RE large text: seeded random RE (depth 7, 40 operators, 26 letters, "
                               "seed %d), %d-byte text sampled from its language with 5%% random-byte "
                               "corruption blocks" % (RE_SEED, n),
                   "text_bytes": n, "words_per_column": W, "segments": parser.nseg,
                   "fwd_states": parser.info.fwd_states, "rev_states": parser.info.rev_states,
                   "table_placement": "lds" if parser.info.placement == 0 else "l2",
                   "lane_chunks": parser.num_chunks(n, args.chunk_bytes), "chunk_bytes": args.chunk_bytes or "auto",
                   "accepted": scal[0], "trees_mod_2_64": scal[1], "count_status": scal[2],
                   "compile_ms": round(compile_ms, 2)},
        "phases_ms": {k: round(v, 4) for k, v in phase.items()},
        "slpf_gbs": round(algo / (ms * 1e-3) / 1e9, 2),
        "roofline": roof,
    }
    del _
    torch.cuda.empty_cache()
    if args.copy_calib:
        a = torch.empty(args.copy_calib, dtype=torch.uint8, device="cuda:0")
        bb = torch.empty_like(a)
        bb.copy_(a)
        torch.cuda.synchronize()
        del a, bb
        torch.cuda.empty_cache()
    if not args.no_companion:
        pat2, clean = make_text(args.bytes, corrupt=False)
        ms2, phase2, scal2, _c = run_gpu(parser, clean, args.steps, args.warmup, args.chunk_bytes)
        del _c
        n2 = clean.size
        algo2 = n2 + (n2 + 1) * 8 * W
        out["companion_clean_text"] = {
            "value": round(n2 / (ms2 * 1e-3) / 1e9, 3), "ms_per_step": round(ms2, 4),
            "accepted": scal2[0], "trees_mod_2_64": scal2[1], "count_status": scal2[2],
            "phases_ms": {k: round(v, 4) for k, v in phase2.items()},
            "build_frac_of_hbm_peak": round(algo2 / (phase2["build"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        print("companion: %.3f ms/step phases %s scalars %s" % (ms2, phase2, scal2), file=sys.stderr,
              flush=True)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pat, text, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
