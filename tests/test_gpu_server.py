"""The request server (slpf_server_*): continuous batching with admission by
projected SLPF bytes.  Every result must be identical alone and in the mix:
each request's columns, accept flag, count and status equal those of
slpf_parse on that text alone (and of the oracle), whatever the arrival
order, the batch it landed in and the requests it overlapped with.
"""
import sys

import numpy as np
import pytest

from gen import regen, workloads as wl
from gpu_util import device, gpu_parse, to_device
from oracle.oracle import Oracle

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _workload(n_res, n_req, seed, median=2048, cap=1 << 16):
    res = wl.served_res()[:n_res]
    lengths = wl.lognormal_lengths(seed, n_req, median=median, sigma=1.5, cap=cap)
    texts = wl.texts_for(res, lengths, seed + 1)
    return res, texts


def test_server_alone_vs_mix():
    import torch
    device()
    res, texts = _workload(8, 160, 31)
    pats = [regen.to_re(t) for _, t in res]
    parsers = [S.Parser(p) for p in pats]
    # empty and one-byte requests in the mix
    texts[5] = (texts[5][0], texts[5][1][:0])
    texts[9] = (texts[9][0], texts[9][1][:1])
    dts = [to_device(x.tobytes()) for _, x in texts]
    torch.cuda.synchronize()
    # a small arena: requests wait for space; 3 slots overlap
    srv = S.Server(slots=3, max_batch_texts=12, memory_budget=6 << 20)
    rng = np.random.default_rng(5)
    order = rng.permutation(len(texts))
    pending, done = list(order), {}
    max_admitted = 0
    while len(done) < len(texts):
        # arrivals in small random bursts while earlier requests run
        for _ in range(int(rng.integers(0, 6))):
            if pending:
                k = int(pending.pop(0))
                r, x = texts[k]
                srv.submit(parsers[r], dts[k], x.size, k)
        for tag in srv.poll():
            r, x = texts[tag]
            done[tag] = srv.result_tensors(tag, x.size, parsers[r].W)
            srv.release(tag)
        st = srv.stats()
        max_admitted = max(max_admitted, st["admitted_bytes"])
        assert st["admitted_bytes"] <= st["arena_bytes"]
    say("server: %d requests, peak admitted %d of %d bytes" % (len(done), max_admitted, 6 << 20))
    assert srv.stats()["admitted_bytes"] == 0
    srv.close()
    oracles = {}
    for k, (r, x) in enumerate(texts):
        cols, sc = done[k]
        alone = gpu_parse(parsers[r], dts[k])
        assert np.array_equal(cols, alone[0]), k
        assert (bool(sc[0]), int(sc[1]), int(sc[2]), int(sc[3])) == alone[1:] + (alone.countp,), k
        if x.size <= 4096:
            o = oracles.setdefault(r, Oracle(pats[r]))
            c2, acc, cnt, cntp = o.parse_full(x.tobytes())
            assert np.array_equal(cols, c2) and bool(sc[0]) == acc, k
            assert int(sc[2]) == 0 and int(sc[1]) == cnt and int(sc[3]) == cntp, k


def test_server_capacity_and_arguments():
    import torch
    device()
    p = S.Parser("(ab|a)*")
    srv = S.Server(slots=1, max_batch_texts=4, memory_budget=1 << 16)
    big = to_device(b"ab" * 4096)                   # its SLPF needs more than the budget
    with pytest.raises(S.SlpfError) as e:
        srv.submit(p, big, 8192, 1)
    assert e.value.status == S.E_CAPACITY
    small = to_device(b"abaaba")
    torch.cuda.synchronize()
    srv.submit(p, small, 6, 7)
    got = []
    while not got:
        got = srv.poll()
    assert got == [7]
    cols, sc = srv.result_tensors(7, 6, p.W)
    assert bool(sc[0]) and int(sc[1]) == 1
    with pytest.raises(S.SlpfError):
        srv.result(8)                               # unknown tag
    srv.release(7)
    with pytest.raises(S.SlpfError):
        srv.release(7)                              # already released
    srv.close()


def test_server_compact_alone_vs_mix():
    # the server with SLPF_PARSE_COMPACT: admission by compact bytes, every
    # result equal to the compact parse of its text alone
    import torch
    device()
    res, texts = _workload(4, 40, 41, median=4096)
    parsers = [S.Parser(regen.to_re(t)) for _, t in res]
    dts = [to_device(x.tobytes()) for _, x in texts]
    torch.cuda.synchronize()
    srv = S.Server(slots=2, max_batch_texts=8, memory_budget=1 << 20, compact=True)
    for k, (r, x) in enumerate(texts):
        srv.submit(parsers[r], dts[k], x.size, k)
    done = {}
    while len(done) < len(texts):
        for tag in srv.poll():
            r, x = texts[tag]
            if parsers[r].info.max_entries > 64:
                # no compact form for entry lists over 64 segments: the request
                # is reported with the error, the rest of its slot is not affected
                with pytest.raises(S.SlpfError) as e:
                    srv.result(tag)
                assert e.value.status == S.E_TOO_LARGE
                done[tag] = None
            else:
                done[tag] = srv.result_tensors(tag, x.size, parsers[r].W)
            srv.release(tag)
    srv.close()
    for k, (r, x) in enumerate(texts):
        if done[k] is None:
            continue
        cmp, sc = parsers[r].parse_compact(dts[k])
        torch.cuda.synchronize()
        cols, s2 = done[k]
        assert np.array_equal(cols, cmp.cpu().numpy().view(np.uint64)), k
        assert np.array_equal(s2, sc.cpu().numpy().view(np.uint64)), k


def test_server_failed_parser_fails_only_its_requests():
    # a parser compiled for the host only cannot run a job: its requests are
    # reported finished with the error, the other parser's requests in the
    # same slot finish normally, and every arena range comes back on release
    import torch
    device()
    good = S.Parser("(ab|a)*")
    bad = S.Parser("(ab|a)*", host_only=True)
    srv = S.Server(slots=1, max_batch_texts=8, memory_budget=1 << 20)
    texts = [b"abab", b"aab", b"ab" * 100, b"abaaba"]
    dts = [to_device(t) for t in texts]
    for k, (t, d) in enumerate(zip(texts, dts)):
        srv.submit(bad if k % 2 else good, d, len(t), k)
    done = set()
    for _ in range(10000):
        done.update(srv.poll())
        if len(done) == len(texts):
            break
    assert done == set(range(len(texts)))
    for k, t in enumerate(texts):
        if k % 2:
            with pytest.raises(S.SlpfError) as e:
                srv.result(k)
            assert e.value.status == S.E_ARG
        else:
            cols, sc = srv.result_tensors(k, len(t), good.W)
            alone = gpu_parse(good, t)
            assert np.array_equal(cols, alone[0]) and bool(sc[0]) == alone[1] and int(sc[1]) == alone[2]
        srv.release(k)
    assert srv.stats()["admitted_bytes"] == 0
    srv.close()
    torch.cuda.synchronize()
