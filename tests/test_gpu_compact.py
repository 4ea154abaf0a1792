"""Compact SLPF (SLPF_PARSE_COMPACT, slpf_decode_compact): every column is
one word over its candidate list.  The words must equal the oracle's compact
encoding bit for bit, decoding them must give the oracle's columns, and the
accept flag, tree count and status must be those of the plain parse; also in
batches and with general lane chunks (the count then reads the compact
columns).  The full-size test checks the compact words at 256 MiB.
"""
import sys

import numpy as np
import pytest

from gen import regen, textgen
from gpu_util import device, gpu_parse, to_device
from oracle.oracle import Oracle

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_compact(p, text, chunk_bytes=0, count=True, force_l2=False):
    import torch
    t = to_device(text) if not hasattr(text, "device") else text
    cmp, sc = p.parse_compact(t, chunk_bytes=chunk_bytes, count=count, force_l2=force_l2)
    dec = p.decode_compact(t, cmp)
    torch.cuda.synchronize()
    s = sc.cpu().numpy().view(np.uint64)
    return (cmp.cpu().numpy().view(np.uint64), dec.cpu().numpy().view(np.uint64),
            bool(s[0]), int(s[1]), int(s[2]), int(s[3]))


def check(pat, texts, chunks=(0, 64, 256), force_l2=False):
    p, o = S.Parser(pat), Oracle(pat)
    for t in texts:
        cols, acc, cnt, cntp = o.parse_full(t)
        want = o.compact(t, cols)
        for k in chunks:
            cmp, dec, a2, c2, st, c2p = gpu_compact(p, t, chunk_bytes=k, force_l2=force_l2)
            bad = np.nonzero(cmp != want)[0]
            assert bad.size == 0, "n=%d k=%d: word %d is %x, oracle %x" % (len(t), k, bad[0], cmp[bad[0]],
                                                                          want[bad[0]])
            assert np.array_equal(dec, cols), (len(t), k)
            assert a2 == acc and st == 0 and c2 == cnt and c2p == cntp, (len(t), k, a2, c2, st, cnt, c2p, cntp)
    return p


def _texts(tree, seed, k, max_len):
    rng = np.random.default_rng(seed)
    out = [b"", b"", b""]
    out[1] = textgen.sample_text(tree, seed, 1).tobytes()[:1]
    for j in range(k):
        n = int(np.exp(rng.uniform(0, np.log(max_len))))
        t = textgen.sample_text(tree, seed * 100 + j, n).tobytes()
        if j % 3 == 2:
            t = textgen.corrupt(np.frombuffer(t, np.uint8), seed * 100 + j, frac=0.05, block=(1, 32)).tobytes()
        out.append(t)
    return out


def test_compact_worked_examples_and_small():
    device()
    check("(ab|a)*", [b"", b"a", b"ab", b"abaaba", b"abab", b"ba", b"aab" * 50])
    check("(a|b|ab)+", [b"abab", b"a", b"bbab" * 40, b"abc"])
    tree = regen.plain_small_re()
    check(regen.to_re(tree).decode(), _texts(tree, 3, 6, 20000))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_compact_random_res(seed):
    device()
    alpha = [b"abc", b"ACGT", b"abcdefghijklmnopqrstuvwxyz", b"ab"][seed]
    tree = regen.random_re(700 + seed, n_ops=14, max_depth=6, alphabet=alpha)
    pat = regen.to_re(tree)
    say("compact random", seed, pat[:60])
    check(pat, _texts(tree, 40 + seed, 5, 12000), chunks=(0, 128))
    check(pat, _texts(tree, 50 + seed, 2, 6000), chunks=(64,), force_l2=True)


def test_compact_motif_and_general_chunks():
    # the motif RE and an RE whose lane chunks are general (no singleton
    # column, or none of at most 8 segments): the count reads compact columns
    device()
    tree = regen.motif_re()
    check(regen.to_re(tree), _texts(tree, 7, 4, 8000), chunks=(0, 64))
    mixed = "((a|a|a|a|a|a|a|a|a|a)|b|(c|cc)|(d|dd|ddd))*"
    rng = np.random.default_rng(5)
    texts = []
    for _ in range(5):
        parts = [bytes([int(rng.choice([97, 98, 99, 100]))]) * int(rng.integers(1, 400)) for _ in range(20)]
        texts.append(b"".join(parts))
    texts.append(b"a" * 3000)
    check(mixed, texts, chunks=(64, 0))


def test_compact_batch_equals_alone():
    import torch
    dev = device()
    tree = regen.plain_small_re()
    pat = regen.to_re(tree).decode()
    p, o = S.Parser(pat), Oracle(pat)
    texts = _texts(tree, 11, 30, 30000)
    dts = [to_device(t) for t in texts]
    cols = [torch.empty(len(t) + 1, dtype=torch.int64, device=dev) for t in texts]
    sc = torch.empty((len(texts), 4), dtype=torch.int64, device=dev)
    items = [(d, len(t), c, sc[k]) for k, (d, t, c) in enumerate(zip(dts, texts, cols))]
    for k in (0, 64):
        p.parse_batch_into(items, chunk_bytes=k, flags=S.PARSE_COMPACT)
        torch.cuda.synchronize()
        s = sc.cpu().numpy().view(np.uint64)
        for j, t in enumerate(texts):
            cmp, dec, a2, c2, st, c2p = gpu_compact(p, t, chunk_bytes=k)
            assert np.array_equal(cols[j].cpu().numpy().view(np.uint64), cmp), (k, j)
            assert (bool(s[j, 0]), int(s[j, 1]), int(s[j, 2]), int(s[j, 3])) == (a2, c2, st, c2p)
            want = o.compact(t)
            assert np.array_equal(cmp, want), (k, j)


def test_compact_capacity_and_arguments():
    import torch
    dev = device()
    p = S.Parser("(ab|a)*")
    t = to_device(b"abab" * 8)
    sc = torch.empty(4, dtype=torch.int64, device=dev)
    ok = torch.empty(33, dtype=torch.int64, device=dev)
    small = torch.empty(32, dtype=torch.int64, device=dev)
    with pytest.raises(S.SlpfError) as e:
        p.parse_into(t, 32, small, sc, 0, S.PARSE_COMPACT)
    assert e.value.status == S.E_CAPACITY
    p.parse_into(t, 32, ok, sc, 0, S.PARSE_COMPACT)
    torch.cuda.synchronize()
    assert p._L.slpf_compact_bytes(32) == 33 * 8
    assert p._L.slpf_decode_compact(p.handle, None, 0, None, None, None) == S.E_ARG


@pytest.mark.parametrize("seed", range(4))
def test_compact_char_set_res(seed):
    # character-set and wildcard leaves (App. A, character features): a
    # segment whose end-letter set spans several byte classes lies in several
    # candidate lists, so its bit index depends on both bytes around the column
    device()
    alpha = [b"abcd", b"abcdefghij"][seed % 2]
    while True:
        tree = regen.random_re(7300 + seed, n_ops=10, max_depth=4, alphabet=alpha, set_p=0.5)
        pat = regen.to_re(tree)
        if S.Parser(pat, host_only=True).info.max_entries <= 64:
            break
        seed += 100
    say("compact sets", pat[:70])
    check(pat, _texts(tree, 50 + seed, 6, 3000), chunks=(0, 64))
