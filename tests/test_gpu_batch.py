"""Batched parsing: one job over many texts of one parser (slpf_parse_texts)
and one call over the texts of many parsers (slpf_parse_batch) give, for
every text, exactly the columns, accept flag, count and status of parsing
that text alone, and of the oracle.

Covers empty and one-byte texts between long ones, texts that are rejected
next to accepted ones, a text counted through general chunks with no anchor
next to texts counted through rank-1 chunks, enough lane chunks for a three-level join scan with text
boundaries inside every scan group, and the argument checks.
"""
import sys

import numpy as np
import pytest

from gen import regen, textgen
from gpu_util import device, gpu_parse, to_device
from oracle.oracle import P61, Oracle

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_batch(p, texts, chunk_bytes=0, count=True, force_l2=False):
    import torch
    dts = [to_device(t) for t in texts]
    res = p.parse_batch(dts, chunk_bytes=chunk_bytes, count=count, force_l2=force_l2)
    torch.cuda.synchronize()
    out = []
    for cols, sc in res:
        s = sc.cpu().numpy().view(np.uint64)
        out.append((cols.cpu().numpy().view(np.uint64), bool(s[0]), int(s[1]), int(s[2]), int(s[3])))
    return out


def mixed_texts(tree, seed, k, max_len):
    """Accepted samples and corrupted (mostly rejected) copies, log-uniform
    lengths, with empty and one-byte texts mixed in."""
    rng = np.random.default_rng(seed)
    texts = []
    for j in range(k):
        r = rng.random()
        if r < 0.08:
            texts.append(b"")
            continue
        n = int(np.exp(rng.uniform(0, np.log(max_len))))
        t = textgen.sample_text(tree, seed * 1000 + j, n).tobytes()
        if r > 0.7:
            t = textgen.corrupt(np.frombuffer(t, np.uint8), seed * 1000 + j, frac=0.05,
                                block=(1, 64)).tobytes()
        if r < 0.12:
            t = t[:1]
        texts.append(t)
    return texts


def check_batch(pat, texts, chunk_bytes=0, force_l2=False, oracle=True):
    say("batch", pat[:50], "texts=%d" % len(texts), "bytes=%d" % sum(map(len, texts)),
        "k=%d" % chunk_bytes, "l2=%d" % force_l2)
    p = S.Parser(pat)
    o = Oracle(pat) if oracle else None
    got = run_batch(p, texts, chunk_bytes=chunk_bytes, force_l2=force_l2)
    for j, t in enumerate(texts):
        alone = gpu_parse(p, t, chunk_bytes=chunk_bytes, force_l2=force_l2)
        b = got[j]
        assert b[0].shape == alone[0].shape, j
        bad = np.nonzero((b[0] != alone[0]).any(axis=1))[0]
        assert bad.size == 0, "text %d (n=%d): column %d differs from the single parse" % (j, len(t), bad[0])
        assert b[1:] == alone[1:] + (alone.countp,), (j, b[1:], alone[1:], alone.countp)
        if o is not None:
            cols, acc, cnt, cntp = o.parse_full(t)
            assert np.array_equal(b[0], cols), j
            assert b[1] == acc, j
            assert b[3] == 0 and b[2] == cnt and b[4] == cntp, (j, b[2:], cnt, cntp)
    return got


def test_batch_plain_small_mixed():
    device()
    tree = regen.plain_small_re()
    pat = regen.to_re(tree).decode()
    texts = mixed_texts(tree, 3, 40, 20000)
    for k in (0, 64, 256):
        got = check_batch(pat, texts, chunk_bytes=k)
    assert any(g[1] for g in got) and not all(g[1] for g in got)


def test_batch_force_l2_and_random_res():
    device()
    for seed in (5, 11):
        tree = regen.random_re(300 + seed, n_ops=12, max_depth=5, alphabet=b"abc")
        pat = regen.to_re(tree).decode()
        texts = mixed_texts(tree, seed, 24, 5000)
        check_batch(pat, texts, chunk_bytes=128)
        check_batch(pat, texts, chunk_bytes=128, force_l2=True)


def test_batch_char_set_res():
    # REs with character-set and wildcard leaves, mixed accepted and
    # rejected texts in one job
    device()
    for seed in (3, 8):
        tree = regen.random_re(7700 + seed, n_ops=14, max_depth=5, alphabet=b"abcdefghij", set_p=0.5)
        pat = regen.to_re(tree)
        check_batch(pat, mixed_texts(tree, 40 + seed, 24, 8000), chunk_bytes=128)


def test_batch_empty_and_tiny_only():
    device()
    pat = "(ab|a)*"
    texts = [b"", b"a", b"", b"ab", b"b", b"aba", b"", b"z", b"abaaba"]
    check_batch(pat, texts)
    check_batch(pat, [b""])
    check_batch(pat, [b"", b""])


def test_batch_count_without_anchor():
    # every column of a^n holds 20 segments: none of its 2100 lane chunks has
    # a singleton or a small column, so its count is one walk over the text;
    # the texts of b's (singleton columns) count through rank-1 chunks.
    # Every count is computed (20^n is 0 modulo 2^64 once n >= 32)
    device()
    pat = "((" + "|".join(["a"] * 20) + ")|b)*"
    texts = [b"b" * 300, b"a" * (64 * 2100), b"", b"b" * 5, b"a" * 21]
    got = check_batch(pat, texts, chunk_bytes=64)
    assert [g[3] for g in got] == [0, 0, 0, 0, 0]
    assert got[0][2] == 1 and got[3][2] == 1
    assert got[1][2] == 0 and got[4][2] == pow(20, 21, 1 << 64)
    assert got[1][4] == pow(20, 64 * 2100, P61) and got[4][4] == pow(20, 21, P61)


def test_batch_deep_join_scan():
    # about 6000 lane chunks of 64 bytes: a three-level join scan whose
    # groups of 64 items hold several text boundaries each
    device()
    tree = regen.plain_small_re()
    pat = regen.to_re(tree).decode()
    rng = np.random.default_rng(9)
    texts = []
    for j in range(700):
        n = int(rng.integers(0, 1100))
        t = textgen.sample_text(tree, 5000 + j, n).tobytes()[:n]
        if j % 7 == 3 and len(t) > 10:
            t = t[:len(t) // 2] + b"\x00" + t[len(t) // 2 + 1:]
        texts.append(t)
    p = S.Parser(pat)
    assert sum(p.num_chunks(len(t), 64) for t in texts) > 4096
    check_batch(pat, texts, chunk_bytes=64)


def test_batch_argument_errors():
    import torch
    dev = device()
    p = S.Parser("(ab|a)*")
    t = to_device(b"abab" * 8)
    cols = torch.empty((33, p.W), dtype=torch.int64, device=dev)
    sc = torch.empty(4, dtype=torch.int64, device=dev)
    small = torch.empty((3, p.W), dtype=torch.int64, device=dev)
    with pytest.raises(S.SlpfError) as e:
        p.parse_batch_into([(t, 32, cols, sc), (t, 32, small, sc)])
    assert e.value.status == S.E_CAPACITY
    with pytest.raises(S.SlpfError) as e:
        p.parse_batch_into([(t, 32, cols, sc), (t[1:], 31, cols, sc)])
    assert e.value.status == S.E_ARG
    with pytest.raises(S.SlpfError) as e:
        p.parse_batch_into([(t, 32, cols, sc)], chunk_bytes=100)
    assert e.value.status == S.E_ARG
    p.parse_batch_into([])
    torch.cuda.synchronize()


def test_batched_re_family_vs_oracle():
    # the batched workload's 16 REs (4, 26 and 128-symbol alphabets and the
    # motif RE), 64 texts of log-uniform length 256 B - 64 KiB, one job per RE
    import torch
    from gen import workloads as wl
    device()
    res = wl.batched_res()
    assert len(res) == 16
    texts = wl.texts_for(res, wl.loguniform_lengths(7, 64, lo=256, hi=64 << 10), 8)
    for q, (name, tree) in enumerate(res):
        mine = [x.tobytes() for r, x in texts if r == q]
        if not mine:
            continue
        pat = regen.to_re(tree)
        say("family", name, len(mine), "texts")
        p, o = S.Parser(pat), Oracle(pat)
        got = run_batch(p, mine)
        for t, g in zip(mine, got):
            cols, acc, cnt, cntp = o.parse_full(t)
            assert acc and g[1], name                    # sampled from the language
            assert np.array_equal(g[0], cols), name
            assert g[3] == 0 and g[2] == cnt and g[4] == cntp, (name, g[2:], cnt, cntp)
    torch.cuda.synchronize()


def test_tune_picks_a_candidate_and_keeps_results_exact():
    import torch
    dev = device()
    tree = regen.plain_small_re()
    pat = regen.to_re(tree).decode()
    texts = mixed_texts(tree, 21, 12, 30000)
    p, o = S.Parser(pat), Oracle(pat)
    dts = [to_device(t) for t in texts]
    cols = [torch.zeros((len(t) + 1, p.W), dtype=torch.int64, device=dev) for t in texts]
    sc = torch.zeros((len(texts), 4), dtype=torch.int64, device=dev)
    items = [(d, len(t), c, sc[k]) for k, (d, t, c) in enumerate(zip(dts, texts, cols))]
    chunk, flags, ms = p.tune(items)
    say("tuned", chunk, flags, ms)
    assert chunk in (256, 512, 1024, 2048, 4096) and ms > 0
    assert flags & ~S.PARSE_FORCE_L2 == 0
    torch.cuda.synchronize()
    s = sc.cpu().numpy().view(np.uint64)
    for k, t in enumerate(texts):
        c, acc, cnt, cntp = o.parse_full(t)
        assert np.array_equal(cols[k].cpu().numpy().view(np.uint64), c), k
        assert bool(s[k, 0]) == acc
        assert int(s[k, 2]) == 0 and int(s[k, 1]) == cnt and int(s[k, 3]) == cntp, k


def test_one_call_over_many_res():
    # slpf_parse_batch: the batched workload's 16 REs (4, 26 and 128-symbol
    # alphabets, the motif RE), 96 texts interleaved across the REs, one call;
    # then again after tuning some parsers (their tuned chunk sizes apply)
    import torch
    from gen import workloads as wl
    dev = device()
    res = wl.batched_res()
    texts = wl.texts_for(res, wl.loguniform_lengths(17, 96, lo=64, hi=32 << 10), 18)
    pats = [regen.to_re(t) for _, t in res]
    parsers = [S.Parser(pt) for pt in pats]
    oracles = {}
    dts = [to_device(x.tobytes()) for _, x in texts]

    def one_call():
        cols = [torch.zeros((x.size + 1, parsers[r].W), dtype=torch.int64, device=dev) for r, x in texts]
        sc = torch.full((len(texts), 4), 7, dtype=torch.int64, device=dev)
        S.parse_items([(parsers[r], d, x.size, c, sc[k])
                       for k, ((r, x), d, c) in enumerate(zip(texts, dts, cols))])
        torch.cuda.synchronize()
        return [c.cpu().numpy().view(np.uint64) for c in cols], sc.cpu().numpy().view(np.uint64)

    cols, sc = one_call()
    for k, (r, x) in enumerate(texts):
        t = x.tobytes()
        if r not in oracles:
            oracles[r] = Oracle(pats[r])
        oc, acc, cnt, cntp = oracles[r].parse_full(t)
        assert np.array_equal(cols[k], oc), (k, res[r][0])
        assert (bool(sc[k, 0]), int(sc[k, 1]), int(sc[k, 2]), int(sc[k, 3])) == (acc, cnt, 0, cntp), k
    say("one call over", len(res), "REs ok")
    for q in (0, 3, 15):   # tune three parsers on their own texts
        mine = [(dts[k], x.size, torch.zeros((x.size + 1, parsers[q].W), dtype=torch.int64, device=dev),
                 torch.zeros(4, dtype=torch.int64, device=dev)) for k, (r, x) in enumerate(texts) if r == q]
        if mine:
            parsers[q].tune(mine)
    cols2, sc2 = one_call()
    assert all(np.array_equal(a, b) for a, b in zip(cols, cols2)) and np.array_equal(sc, sc2)


def test_one_call_argument_errors():
    import torch
    dev = device()
    p, q = S.Parser("(ab|a)*"), S.Parser("(a|b)*c")
    h = S.Parser("(ab|a)*", host_only=True)
    t = to_device(b"abab" * 8)
    cols = torch.empty((33, 1), dtype=torch.int64, device=dev)
    small = torch.empty((3, 1), dtype=torch.int64, device=dev)
    sc = torch.full((2, 4), 7, dtype=torch.int64, device=dev)
    with pytest.raises(S.SlpfError) as e:
        S.parse_items([(p, t, 32, cols, sc[0]), (q, t, 32, small, sc[1])])
    assert e.value.status == S.E_CAPACITY
    with pytest.raises(S.SlpfError) as e:
        S.parse_items([(p, t, 32, cols, sc[0]), (h, t, 32, cols, sc[1])])
    assert e.value.status == S.E_ARG
    torch.cuda.synchronize()
    assert (sc.cpu() == 7).all()                       # nothing was launched
    S.parse_items([])
