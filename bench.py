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
BATCH_RE_SEED, BATCH_LEN_SEED, BATCH_TEXT_SEED = 4000, 4001, 4002
SERVE_RE_SEED, SERVE_LEN_SEED, SERVE_TEXT_SEED, SERVE_ARRIVAL_SEED = 5000, 5001, 5002, 5003
SERVE_RATES = [0.25, 0.5, 0.75, 0.9, 1.1]
SWEEP_CHUNK_BYTES = [256, 1024, 4096, 16384, 65536, 262144, 1048576]
RECORD_SEED, RECORD_BYTES = 31, 1 << 30
KERNEL_SOURCES = ["paper_2503_06763_amd/csrc/kernels.hpp", "paper_2503_06763_amd/csrc/count.hpp",
                  "paper_2503_06763_amd/csrc/slpf.hip"]


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


def run_gpu(parser, text_np, steps, warmup, chunk_bytes, compact=False, flags=0):
    """Timed parses; ``compact``: the compact SLPF (one word per column)."""
    import numpy as np
    import torch
    import paper_2503_06763_amd as S
    dev = torch.device("cuda:0")
    n = text_np.size
    text = torch.from_numpy(text_np).to(dev)
    W = parser.W
    cols = torch.empty((n + 1,) if compact else (n + 1, W), dtype=torch.int64, device=dev)
    sc = torch.empty(4, dtype=torch.int64, device=dev)
    flags |= S.PARSE_COMPACT if compact else 0
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(S.NUM_PHASE_EVENTS)] for _ in range(steps)]
    for _ in range(warmup):
        parser.parse_into(text, n, cols, sc, chunk_bytes, flags)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        parser.parse_into(text, n, cols, sc, chunk_bytes, flags, events=evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    phase = {name: sum(e[i].elapsed_time(e[i + 1]) for e in evs) / steps
             for i, name in enumerate(S.PHASES)}
    s = sc.cpu().numpy().view(np.uint64)
    return ms, phase, (int(s[0]), int(s[1]), int(s[2]), int(s[3])), cols


def run_recognize(parser, text_np, steps, warmup, chunk_bytes):
    """Recogniser mode (forward reach and forward join only) on the same text."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    text = torch.from_numpy(text_np).to(dev)
    for _ in range(warmup):
        sc = parser.recognize(text, chunk_bytes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sc = parser.recognize(text, chunk_bytes)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return ms, int(sc.cpu().numpy().view(np.uint64)[0])


def time_matches(parser, text_np, cols):
    """Match extraction on the parsed text: the group with the most matches on
    a 64 KiB prefix (a record field), then its matches over the whole text."""
    import torch
    import numpy as np
    n = text_np.size
    # a prefix of whole records (cut after its last newline), so that it is
    # accepted; the group with the most matches there is a field (the star's
    # group has one match spanning the text, walked in one wavefront)
    head = text_np[:1 << 16]
    cut = int(np.nonzero(head == 10)[0][-1]) + 1
    pre = torch.from_numpy(head[:cut].copy()).to("cuda:0")
    pcols, psc = parser.parse(pre)
    groups = sorted({int(t[:-1]) for i in range(parser.nseg) for t in parser.segment_text(i).split(" ")
                     if t.endswith("(")})
    counts = {g: len(parser.matches(pcols, g)) for g in groups}
    best = max(groups, key=lambda g: (counts[g], -g))
    del pcols
    if counts[best] <= 1:
        return {"skipped": "no field group with matches on the prefix"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = parser.matches(cols, best, capacity=n // 2)
    ms = (time.perf_counter() - t0) * 1e3
    lens = (m[:, 1] - m[:, 0]).astype(np.int64) if len(m) else np.zeros(0, np.int64)
    print("matches: group %d, %d matches in %.1f ms" % (best, len(m), ms), file=sys.stderr, flush=True)
    return {"group": best, "matches": int(len(m)), "ms": round(ms, 2),
            "mean_match_bytes": round(float(lens.mean()), 2) if len(m) else 0.0,
            "text_gbs": round(n / (ms * 1e-3) / 1e9, 3),
            "what": "slpf_get_matches over the whole parsed text (group spans; call time incl. its work buffers)"}


def cpu_baseline(pat, text_np, sample_bytes):
    from oracle.oracle import Oracle
    o = Oracle(pat)
    x = text_np[:sample_bytes].tobytes()
    t0 = time.perf_counter()
    o.parse(x)
    dt = time.perf_counter() - t0
    return {"value": round(len(x) / dt / 1e9, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "host": host_cpu(),
            "sample": "first %d bytes of the same text, serial NFA parser (Fig. serialparser) "
                      "with in-place intersection and tree count, single thread, %.1f s" % (len(x), dt)}


def host_cpu():
    """CPU model and logical core count of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def _aligned_offsets(sizes, align):
    offs, tot = [], 0
    for z in sizes:
        offs.append(tot)
        tot += (int(z) + align - 1) // align * align
    return offs, max(tot, align)


def oracle_pool_baseline(jobs, seconds_hint):
    """The oracle over host cores: one text per task on a process pool; jobs
    is a list of (pattern, bytes)."""
    import concurrent.futures as cf
    cores = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_oracle_task, jobs, chunksize=1))
    dt = time.perf_counter() - t0
    nb = sum(len(x) for _, x in jobs)
    return {"value": round(nb / dt / 1e9, 6), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "host": host_cpu(),
            "sample": "%d texts, %d bytes, serial oracle parser (Fig. serialparser) with tree count, one "
                      "text per process on %d processes, %.1f s" % (len(jobs), nb, cores, dt)}


_ORACLES = {}


def _oracle_task(job):
    from oracle.oracle import Oracle
    pat, x = job
    o = _ORACLES.get(pat)
    if o is None:
        o = _ORACLES[pat] = Oracle(pat)
    o.parse(x)
    return len(x)


def run_batched(args, leg=False):
    """Many REs and texts: 16 REs, 4096 texts of log-uniform length; per-text
    plain parses vs one batched job per RE (autotuned chunk size and table
    placement, jobs spread over streams).  Both results are compared.  With
    ``leg`` the result is returned (a leg of the default line) instead of
    printed, without a CPU baseline."""
    import numpy as np
    import torch
    import paper_2503_06763_amd as S
    from gen import regen, workloads as wl

    t0 = time.perf_counter()
    res = wl.batched_res(seed=BATCH_RE_SEED)
    lengths = wl.loguniform_lengths(BATCH_LEN_SEED, args.texts)
    texts = wl.texts_for(res, lengths, BATCH_TEXT_SEED)
    gen_s = time.perf_counter() - t0
    pats = [regen.to_re(t) for _, t in res]
    parsers = [S.Parser(pt) for pt in pats]
    dev = torch.device("cuda:0")
    ns = [int(x.size) for _, x in texts]
    Ws = [parsers[r].W for r, _ in texts]
    toffs, ttot = _aligned_offsets(ns, 256)
    tbuf = torch.empty(ttot, dtype=torch.uint8, device=dev)
    host = np.zeros(ttot, np.uint8)
    for (r, x), o in zip(texts, toffs):
        host[o:o + x.size] = x
    tbuf.copy_(torch.from_numpy(host))
    del host
    coffs, ctot = _aligned_offsets([(n + 1) * w for n, w in zip(ns, Ws)], 32)
    outs = []
    for _ in range(2):
        cbig = torch.zeros(ctot, dtype=torch.int64, device=dev)
        sc = torch.zeros((len(texts), 4), dtype=torch.int64, device=dev)
        items = [(tbuf[o:o + n], n, cbig[c:c + (n + 1) * w], sc[k])
                 for k, (o, n, c, w) in enumerate(zip(toffs, ns, coffs, Ws))]
        outs.append((cbig, sc, items))
    torch.cuda.synchronize()
    total = sum(ns)
    algo = sum(n + (n + 1) * 8 * w for n, w in zip(ns, Ws))
    print("batched workload: %d REs, %d texts, %d bytes (algorithmic %d), gen %.1fs" % (
        len(res), len(texts), total, algo, gen_s), file=sys.stderr, flush=True)

    # plain: one slpf_parse per text, in workload order, one stream
    _, _, items_p = outs[0]

    def plain_pass():
        for (r, _), it in zip(texts, items_p):
            parsers[r].parse_into(it[0], it[1], it[2], it[3])
    plain_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_pass()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / args.steps

    # batched: one job per RE, autotuned, over several streams
    _, _, items_b = outs[1]
    groups = [[k for k, (r, _) in enumerate(texts) if r == q] for q in range(len(res))]
    tuned, arrays = [], []
    for q, g in enumerate(groups):
        its = [items_b[k] for k in g]
        if not its:
            tuned.append(None)
            arrays.append(None)
            continue
        tuned.append(parsers[q].tune(its))
        arrays.append(parsers[q]._text_array(its))
    streams = [torch.cuda.Stream(device=dev) for _ in range(args.streams)]
    torch.cuda.synchronize()

    def batched_pass():
        for q, arr in enumerate(arrays):
            if arr is None:
                continue
            st = streams[q % len(streams)]
            parsers[q].parse_batch_prepared(arr, len(groups[q]), tuned[q][0], tuned[q][1], st)
    batched_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched_pass()
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    same = bool(torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]))
    sc = outs[1][1].cpu().numpy().view(np.uint64)
    print("plain %.3f ms, batched %.3f ms, identical %s" % (plain_ms, batch_ms, same), file=sys.stderr,
          flush=True)
    # the same texts in one slpf_parse_batch call (every item with its parser;
    # the tuned parsers use their tuned chunk size and placement)
    outs[0][0].zero_()
    outs[0][1].zero_()
    iarr = S.item_array([(parsers[r], it[0], it[1], it[2], it[3]) for (r, _), it in zip(texts, items_p)])
    S.parse_items_prepared(iarr, len(texts))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.parse_items_prepared(iarr, len(texts))
    torch.cuda.synchronize()
    one_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    same_one = bool(torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]))
    print("one call: %.3f ms, identical %s" % (one_ms, same_one), file=sys.stderr, flush=True)
    gbs = total / (batch_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(gbs, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": round(batch_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched: %d seeded random REs (depth 4-8; alphabets of 4, 26 and 128 "
                               "symbols) and the motif RE, %d texts of log-uniform length 1 KiB-4 MiB "
                               "sampled from their REs, one job per RE, jobs over %d streams" % (
                                   len(res) - 1, len(texts), len(streams)),
                   "texts": len(texts), "text_bytes": total, "algorithmic_bytes": algo,
                   "tuned": {res[q][0]: {"chunk_bytes": t[0], "placement": "l2" if t[1] & S.PARSE_FORCE_L2
                                         else "lds", "wide_count": bool(t[1] & S.PARSE_WIDE_COUNT),
                                         "ms": round(t[2], 3)}
                             for q, t in enumerate(tuned) if t},
                   "accepted": int(sc[:, 0].sum()), "count_ok": int((sc[:, 2] == 0).sum())},
        "plain_per_text": {"value": round(total / (plain_ms * 1e-3) / 1e9, 3), "ms_per_step": round(plain_ms, 4)},
        "speedup_vs_plain": round(plain_ms / batch_ms, 3),
        "identical_to_plain": same,
        "one_call": {"value": round(total / (one_ms * 1e-3) / 1e9, 3), "ms_per_step": round(one_ms, 4),
                     "identical_to_plain": same_one,
                     "what": "all texts in one slpf_parse_batch call, each item with its parser"},
        "roofline": {"bound": "hbm", "achieved": round(algo / (batch_ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(algo / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "whole job (all kernels of all jobs)",
                     "algorithmic_bytes": algo},
    }
    if leg:
        del outs, items_p, items_b, tbuf
        torch.cuda.empty_cache()
        return out
    if not args.no_cpu_baseline:
        jobs, acc = [], 0
        for r, x in texts:
            if acc + x.size > args.cpu_sample:
                continue
            jobs.append((pats[r], x.tobytes()))
            acc += x.size
        out["cpu_baseline"] = oracle_pool_baseline(jobs, 0)
    print(json.dumps(out), flush=True)


def run_served(args, leg=False):
    """Served: 64 resident REs, Poisson arrivals at 5 rates relative to the
    plain per-request capacity, lognormal text lengths; the request server
    (continuous batching, admission by projected SLPF bytes within the memory
    budget) against the plain per-request path (one request per job, one job
    in flight).  p50/p99 latency from arrival to finished, and aggregate GB/s.
    With ``leg`` the result is returned instead of printed, without a CPU
    baseline."""
    import numpy as np
    import torch
    import paper_2503_06763_amd as S
    from gen import regen, workloads as wl

    t0 = time.perf_counter()
    res = wl.served_res(seed=SERVE_RE_SEED)
    lengths = wl.lognormal_lengths(SERVE_LEN_SEED, args.pool)
    pool = wl.texts_for(res, lengths, SERVE_TEXT_SEED)
    gen_s = time.perf_counter() - t0
    pats = [regen.to_re(t) for _, t in res]
    parsers = [S.Parser(pt) for pt in pats]
    dev = torch.device("cuda:0")
    ns = [int(x.size) for _, x in pool]
    offs, tot = _aligned_offsets(ns, 256)
    host = np.zeros(tot, np.uint8)
    for (r, x), o in zip(pool, offs):
        host[o:o + x.size] = x
    tbuf = torch.from_numpy(host).to(dev)
    del host
    views = [tbuf[o:o + n] for o, n in zip(offs, ns)]
    torch.cuda.synchronize()
    print("served workload: %d REs, pool of %d texts (%d bytes), gen %.1fs" % (
        len(res), len(pool), sum(ns), gen_s), file=sys.stderr, flush=True)

    servers = {"plain": S.Server(slots=1, max_batch_texts=1, memory_budget=args.budget),
               "served": S.Server(slots=args.slots, max_batch_texts=args.max_batch, memory_budget=args.budget)}

    def run(mode, arrivals):
        """Drive one server through the arrival schedule; returns latencies (s), the span and bytes."""
        srv = servers[mode]
        nreq = len(arrivals)
        lat = np.zeros(nreq)
        nb = 0
        k = 0
        fin = 0
        start = time.perf_counter()
        while fin < nreq:
            now = time.perf_counter() - start
            while k < nreq and arrivals[k] <= now:
                j = k % len(pool)
                srv.submit(parsers[pool[j][0]], views[j], ns[j], k)
                nb += ns[j]
                k += 1
            for tag in srv.poll():
                lat[tag] = time.perf_counter() - start - arrivals[tag]
                srv.release(tag)
                fin += 1
        span = time.perf_counter() - start
        return lat, span, nb

    # warm both servers (work buffers of every parser on every slot stream),
    # then the capacities: the whole pool submitted at once
    run("served", np.zeros(len(pool)))
    run("plain", np.zeros(len(pool)))
    cap = {}
    for mode in ("plain", "served"):
        lat, span, nb = run(mode, np.zeros(len(pool)))
        cap[mode] = {"requests_per_s": round(len(pool) / span, 2), "gbs": round(nb / span / 1e9, 3),
                     "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                     "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3)}
    mu = cap["plain"]["requests_per_s"]
    print("capacity: plain %s | served %s" % (cap["plain"], cap["served"]), file=sys.stderr, flush=True)
    rows = []
    for f in SERVE_RATES:
        lam = f * mu
        arr = wl.poisson_arrivals(SERVE_ARRIVAL_SEED + int(f * 100), args.requests, lam)
        row = {"rate_vs_plain_capacity": f, "requests_per_s": round(lam, 2)}
        for mode in ("served", "plain"):
            lat, span, nb = run(mode, arr)
            row[mode] = {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                         "gbs": round(nb / span / 1e9, 3), "span_s": round(span, 3)}
        print("rate %.2f x mu: served p50 %.2f p99 %.2f ms %.2f GB/s | plain p50 %.2f p99 %.2f ms %.2f GB/s" % (
            f, row["served"]["p50_ms"], row["served"]["p99_ms"], row["served"]["gbs"], row["plain"]["p50_ms"],
            row["plain"]["p99_ms"], row["plain"]["gbs"]), file=sys.stderr, flush=True)
        rows.append(row)
    for srv in servers.values():
        srv.close()
    top = rows[-1]
    out = {
        "metric": METRIC, "value": cap["served"]["gbs"], "unit": "GB/s", "n_gpus": 1, "steps": len(rows),
        "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "served: %d resident REs (random REs of depth 4-8 over 4, 26 and 128 symbols, "
                               "and the motif RE), Poisson arrivals at %s x the plain per-request capacity, "
                               "%d requests per rate over a pool of %d texts with lognormal lengths (median "
                               "64 KiB, sigma 1.5, cap 64 MiB), admission by projected SLPF bytes within %d "
                               "bytes, %d slots, up to %d requests per job" % (
                                   len(res), SERVE_RATES, args.requests, len(pool), args.budget, args.slots,
                                   args.max_batch),
                   "plain_capacity_requests_per_s": round(mu, 2)},
        "capacity": cap,
        "speedup_vs_plain": round(cap["served"]["gbs"] / cap["plain"]["gbs"], 3),
        "latency_at_1.1x_plain_capacity": {"served": {"p50_ms": top["served"]["p50_ms"],
                                                      "p99_ms": top["served"]["p99_ms"]},
                                           "plain": {"p50_ms": top["plain"]["p50_ms"],
                                                     "p99_ms": top["plain"]["p99_ms"]}},
        "rates": rows,
    }
    if leg:
        del views, tbuf
        torch.cuda.empty_cache()
        return out
    if not args.no_cpu_baseline:
        jobs, acc = [], 0
        for r, x in pool:
            if acc + x.size > args.cpu_sample:
                continue
            jobs.append((pats[r], x.tobytes()))
            acc += x.size
        out["cpu_baseline"] = oracle_pool_baseline(jobs, 0)
    print(json.dumps(out), flush=True)


def record_leg(args):
    """The record workload at its full size (1 GiB of multi-schema log
    records, L2-resident tables): parse time, phases, the whole step's and
    k_build's fraction of the HBM roofline, and the accept flag and counts
    against the oracle's values in tests/golden/full_size_counts.yaml."""
    import yaml
    import torch
    import paper_2503_06763_amd as S
    from gen import regen, textgen
    t0 = time.perf_counter()
    pat, text = regen.to_re(regen.record_re()), textgen.record_text(RECORD_SEED, RECORD_BYTES)
    gen_s = time.perf_counter() - t0
    parser = S.Parser(pat)
    n, W = text.size, parser.W
    ms, phase, scal, cols = run_gpu(parser, text, args.leg_steps, 2, 0)
    del cols
    torch.cuda.empty_cache()
    algo = n + (n + 1) * 8 * W
    with open(os.path.join(ROOT, "tests", "golden", "full_size_counts.yaml")) as f:
        g = yaml.safe_load(f)["record_re"]
    same = (g["re_sha256"] == hashlib.sha256(pat).hexdigest() and g["text_bytes"] == n and
            (bool(scal[0]), scal[1], scal[3]) == (g["accepted"], g["trees_mod_2_64"], g["trees_mod_2_61_1"])
            and scal[2] == 0)
    print("record leg: %.3f ms/step phases %s scalars %s golden %s (gen %.1fs)" % (ms, phase, scal, same, gen_s),
          file=sys.stderr, flush=True)
    return {
        "workload": "record RE with L2-resident tables: multi-schema log records (14 schemas of 8 fields over "
                    "overlapping byte sets), %d states forward / %d reverse, W = %d; %d-byte text (seed %d)" % (
                        parser.info.fwd_states, parser.info.rev_states, W, n, RECORD_SEED),
        "value": round(n / (ms * 1e-3) / 1e9, 3), "unit": "GB/s", "ms_per_step": round(ms, 4),
        "steps": args.leg_steps, "warmup": 2,
        "phases_ms": {k: round(v, 4) for k, v in phase.items()},
        "roofline": {"bound": "hbm", "algorithmic_bytes": algo,
                     "step_frac": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "k_build_frac": round(algo / (phase["build"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "table_placement": "lds" if parser.info.placement == 0 else "l2",
        "accepted": scal[0], "trees_mod_2_64": scal[1], "trees_mod_2_61_1": scal[3], "count_status": scal[2],
        "equals_oracle_golden": same,
    }


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
    ap.add_argument("--workload", choices=["single", "record", "batched", "served"], default="single")
    ap.add_argument("--requests", type=int, default=4000, help="served: requests per arrival rate")
    ap.add_argument("--pool", type=int, default=1024, help="served: distinct texts the requests cycle over")
    ap.add_argument("--budget", type=int, default=64 << 30, help="served: SLPF bytes admitted at once")
    ap.add_argument("--slots", type=int, default=4, help="served: jobs in flight")
    ap.add_argument("--max-batch", type=int, default=256, help="served: requests per job at most")
    ap.add_argument("--texts", type=int, default=4096, help="batched: number of texts")
    ap.add_argument("--streams", type=int, default=4, help="batched: streams the per-RE jobs are spread over")
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload: skip the chunk-size sweep and the record, batched and served legs")
    ap.add_argument("--leg-steps", type=int, default=3, help="timed steps of the record and batched legs")
    ap.add_argument("--leg-requests", type=int, default=1000, help="served leg: requests per arrival rate")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="after timing, copy this many bytes device-to-device (scale reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the parser runs on a single MI355X and has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2503_06763_amd as S
    S.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batched":
        if args.steps == 10:
            args.steps = 3
        return run_batched(args)
    if args.workload == "served":
        return run_served(args)

    t0 = time.perf_counter()
    if args.workload == "record":
        from gen import regen, textgen
        if args.bytes == TEXT_BYTES:
            args.bytes = RECORD_BYTES
        pat, text = regen.to_re(regen.record_re()), textgen.record_text(RECORD_SEED, args.bytes)
        args.no_companion = True
        if args.cpu_sample == 32 << 20:
            args.cpu_sample = 8 << 20
    else:
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
            "traffic": traffic_from_profiles("single_re_large" if args.workload == "single" else "record_re",
                                             khash), "kernel": "k_build",
            "algorithmic_bytes": algo}
    out = {
        "metric": METRIC, "value": round(n / (ms * 1e-3) / 1e9, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": ("single-RE large text: seeded random RE (depth 7, 40 operators, 26 letters, "
                                "seed %d), %d-byte text sampled from its language with 5%% random-byte "
                                "corruption blocks" % (RE_SEED, n)) if args.workload == "single" else
                               ("record RE with L2-resident tables: multi-schema log records (timestamp, ':', "
                                "one of 14 schemas of 8 comma-separated fields over overlapping byte sets, "
                                "optional quoted field, newline) under one star, %d byte classes; %d-byte text "
                                "of records (seed %d), field lengths 1-12" % (parser.info.num_classes, n,
                                                                              RECORD_SEED)),
                   "text_bytes": n, "words_per_column": W, "segments": parser.nseg,
                   "fwd_states": parser.info.fwd_states, "rev_states": parser.info.rev_states,
                   "table_placement": "lds" if parser.info.placement == 0 else "l2",
                   "lane_chunks": parser.num_chunks(n, args.chunk_bytes), "chunk_bytes": args.chunk_bytes or "auto",
                   "accepted": scal[0], "trees_mod_2_64": scal[1], "trees_mod_2_61_1": scal[3],
                   "count_status": scal[2],
                   "compile_ms": round(compile_ms, 2)},
        "phases_ms": {k: round(v, 4) for k, v in phase.items()},
        "slpf_gbs": round(algo / (ms * 1e-3) / 1e9, 2),
        "roofline": roof,
    }
    if args.workload == "record":
        out["matches"] = time_matches(parser, text, _)
    # compact SLPF of the same text: one word per column over its candidate
    # list; checked against the plain layout through slpf_decode_compact
    if parser.info.max_entries <= 64:
        cms, cphase, cscal, ccols = run_gpu(parser, text, args.steps, args.warmup, args.chunk_bytes, compact=True)
        dec = parser.decode_compact(torch.from_numpy(text).to("cuda:0"), ccols)
        same = bool(torch.equal(dec, _)) and cscal == scal
        del dec, ccols
        calgo = n + (n + 1) * 8
        out["compact"] = {"value": round(n / (cms * 1e-3) / 1e9, 3), "unit": "GB/s",
                          "ms_per_step": round(cms, 4),
                          "phases_ms": {k: round(v, 4) for k, v in cphase.items()},
                          "algorithmic_bytes": calgo,
                          "build_achieved_gbs": round(calgo / (cphase["build"] * 1e-3) / 1e9, 2),
                          "build_frac_of_hbm_peak": round(calgo / (cphase["build"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "decodes_to_plain": same,
                          "what": "SLPF_PARSE_COMPACT: each column as one word over its candidate list"}
        print("compact: %.3f ms/step phases %s decodes_to_plain %s" % (cms, cphase, same), file=sys.stderr,
              flush=True)
    else:
        out["compact"] = {"skipped": "candidate lists of up to %d segments; the compact form holds 64"
                          % parser.info.max_entries}
    # lane-chunk size sweep over the same text (the configuration's 4 KiB -
    # 1 MiB, and the automatic size's neighbourhood): time per parse, and the
    # columns and scalars against those of the automatic size
    if args.workload == "single" and not args.no_legs:
        sweep = []
        for cb in SWEEP_CHUNK_BYTES:
            sms, sphase, sscal, scols = run_gpu(parser, text, 2, 1, cb)
            same = bool(torch.equal(scols, _)) and sscal == scal
            del scols
            torch.cuda.empty_cache()
            sweep.append({"chunk_bytes": cb, "lane_chunks": parser.num_chunks(n, cb),
                          "value": round(n / (sms * 1e-3) / 1e9, 3), "ms_per_step": round(sms, 4),
                          "phases_ms": {k: round(v, 4) for k, v in sphase.items()}, "identical": same})
            print("chunk %d: %.3f ms/step identical %s" % (cb, sms, same), file=sys.stderr, flush=True)
        out["chunk_sweep"] = {"unit": "GB/s", "auto_chunk_bytes": (-(-n // parser.num_chunks(n)) + 63) // 64 * 64, "sizes": sweep,
                              "what": "lane-chunk bytes per lane (one chunk per lane, 64 per wavefront), "
                                      "2 timed parses each; identical: columns and scalars equal the "
                                      "automatic size's"}
    del _
    torch.cuda.empty_cache()
    # speculation ablation: runs started from every segment whose end-letter
    # is the chunk's first byte, without the previous-byte filter
    nms, nphase, nscal, _n = run_gpu(parser, text, args.steps, args.warmup, args.chunk_bytes,
                                     flags=S.PARSE_NEXT_BYTE_ENTRIES)
    del _n
    out["speculation_ablation"] = {
        "reduced_entries": {"max_entries": parser.info.max_entries, "reach_ms": round(phase["reach"], 4),
                            "ms_per_step": round(ms, 4)},
        "next_byte_entries": {"max_entries": parser.info.max_entries_next_byte,
                              "reach_ms": round(nphase["reach"], 4), "ms_per_step": round(nms, 4),
                              "same_scalars": nscal == scal},
        "what": "lane-chunk runs from the reduced entry list X(previous byte, next byte) vs from every "
                "segment whose end-letter is the next byte"}
    print("next-byte entries: %.3f ms/step reach %.3f ms (reduced: reach %.3f ms)" % (
        nms, nphase["reach"], phase["reach"]), file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    # the standard speculation the paper compares ME-DFA entries with (Sect. 5):
    # runs from every DFA state at the inner lane-chunk edges
    dfa_states = max(parser.info.dfa_states, parser.info.rdfa_states)
    if dfa_states <= 2048:
        ams, aphase, ascal, _a = run_gpu(parser, text, args.steps, args.warmup, args.chunk_bytes,
                                         flags=S.PARSE_ALL_DFA_STATES)
        del _a
        out["speculation_ablation"]["all_dfa_states"] = {
            "max_entries": dfa_states, "reach_ms": round(aphase["reach"], 4), "join_ms": round(aphase["join"], 4),
            "ms_per_step": round(ams, 4), "same_scalars": ascal == scal,
            "reach_saved_by_me_dfa_entries": round(1 - phase["reach"] / aphase["reach"], 4),
            "step_saved_by_me_dfa_entries": round(1 - ms / ams, 4),
            "what": "lane-chunk runs from every forward (reverse) DFA state at inner edges: the standard "
                    "speculation, against the reduced ME-DFA entry lists"}
        print("all DFA states: %.3f ms/step reach %.3f join %.3f ms" % (ams, aphase["reach"], aphase["join"]),
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    rms, racc = run_recognize(parser, text, args.steps, args.warmup, args.chunk_bytes)
    out["recognizer"] = {"value": round(n / (rms * 1e-3) / 1e9, 3), "unit": "GB/s", "ms_per_step": round(rms, 4),
                         "accepted": racc, "what": "forward reach and forward join only (accept flag, no SLPF)"}
    print("recognizer: %.3f ms/step accepted %d" % (rms, racc), file=sys.stderr, flush=True)
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
            "accepted": scal2[0], "trees_mod_2_64": scal2[1], "trees_mod_2_61_1": scal2[3],
            "count_status": scal2[2],
            "phases_ms": {k: round(v, 4) for k, v in phase2.items()},
            "build_frac_of_hbm_peak": round(algo2 / (phase2["build"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        print("companion: %.3f ms/step phases %s scalars %s" % (ms2, phase2, scal2), file=sys.stderr,
              flush=True)
        torch.cuda.empty_cache()
        cms2, cphase2, cscal2, _c = run_gpu(parser, clean, args.steps, args.warmup, args.chunk_bytes, compact=True)
        del _c
        out["companion_clean_text"]["compact"] = {
            "value": round(n2 / (cms2 * 1e-3) / 1e9, 3), "ms_per_step": round(cms2, 4),
            "phases_ms": {k: round(v, 4) for k, v in cphase2.items()},
            "same_scalars": cscal2 == scal2}
        print("companion compact: %.3f ms/step phases %s" % (cms2, cphase2), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pat, text, args.cpu_sample)
    if args.workload == "single" and not args.no_legs:
        # the other configurations, bounded, measured in the same run
        del text
        torch.cuda.empty_cache()
        legs = {"record": record_leg(args)}
        bargs = argparse.Namespace(**vars(args))
        bargs.steps = args.leg_steps
        legs["batched"] = run_batched(bargs, leg=True)
        sargs = argparse.Namespace(**vars(args))
        sargs.requests = args.leg_requests
        legs["served"] = run_served(sargs, leg=True)
        out["legs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
