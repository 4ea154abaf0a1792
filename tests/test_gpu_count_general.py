"""Tree count through general lane chunks (no singleton column, or a column
above the fast kernels' limit): chunks anchored at a small column (rank
above 1), chunks with no small column (walked through), and runs of them
between rank-1 chunks.  The count must equal the oracle's and a closed form
where there is one, and must not depend on the chunk size or on batching.
"""
import sys

import numpy as np
import pytest

from automata_props import column_unambiguous
from gpu_util import device, gpu_parse, to_device
from oracle.oracle import P61, Oracle

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fib_mod(n, m=1 << 64):
    """F(n) modulo m with F(1) = F(2) = 1."""
    a, b = 0, 1
    for _ in range(n):
        a, b = b, (a + b) % m
    return a


def test_rank2_columns_closed_form():
    # (a|aa)* over a^n: every inner column holds two or three segments, so
    # every chunk is general with an anchor of rank 2 or 3; the number of
    # trees is the number of compositions of n into 1s and 2s, F(n+1)
    device()
    p = S.Parser("(a|aa)*")
    for n in (1, 2, 63, 64, 65, 1000, 4097, 20000):
        text = b"a" * n
        for k in (64, 256, 0):
            g = gpu_parse(p, text, chunk_bytes=k)
            cols, acc, cnt, st = g
            assert acc and st == 0, (n, k, st)
            assert cnt == fib_mod(n + 1), (n, k, cnt)
            assert g.countp == fib_mod(n + 1, P61), (n, k, g.countp)
    say("rank-2 chains ok")


def _blocks(rng, alphabet_blocks, total):
    out = []
    size = 0
    while size < total:
        letter, lo, hi = alphabet_blocks[int(rng.integers(len(alphabet_blocks)))]
        k = int(rng.integers(lo, hi + 1))
        out.append(letter * k)
        size += k
    return b"".join(out)[:total]


MIXED_RE = "((a|a|a|a|a|a|a|a|a|a)|b|(c|cc)|(d|dd|ddd))*"


def test_mixed_runs_vs_oracle_and_chunking():
    # b-blocks give singleton columns (rank-1 chunks), c- and d-blocks small
    # ambiguous columns (anchored general chunks), a-blocks ten segments per
    # column (chunks with no anchor); block lengths around the chunk sizes
    device()
    p, o = S.Parser(MIXED_RE), Oracle(MIXED_RE)
    rng = np.random.default_rng(17)
    blocks = [(b"a", 1, 300), (b"b", 1, 200), (b"c", 1, 400), (b"d", 1, 150), (b"a", 200, 900)]
    texts = [_blocks(rng, blocks, int(rng.integers(1, 12000))) for _ in range(10)]
    texts += [b"a" * 5000, b"b" * 3 + b"a" * 3000 + b"b", b"c" * 3000 + b"a" * 700 + b"d" * 900]
    for t in texts:
        _, acc, want, wantp = o.parse_full(t)
        assert acc
        got = set()
        for k in (64, 128, 512, 0):
            g = gpu_parse(p, t, chunk_bytes=k)
            cols, a2, cnt, st = g
            assert a2 and st == 0, (len(t), k, st)
            assert cnt == want and g.countp == wantp, (len(t), k, cnt, want, g.countp, wantp)
            got.add((cnt, g.countp))
        assert len(got) == 1
    say("mixed runs ok:", len(texts), "texts")


def test_general_chunks_batched_equal_alone():
    import torch
    device()
    p, o = S.Parser(MIXED_RE), Oracle(MIXED_RE)
    rng = np.random.default_rng(23)
    blocks = [(b"a", 1, 400), (b"b", 1, 100), (b"c", 1, 300), (b"d", 50, 600)]
    texts = [_blocks(rng, blocks, int(rng.integers(0, 6000))) for _ in range(40)]
    dts = [to_device(t) for t in texts]
    for k in (64, 0):
        res = p.parse_batch(dts, chunk_bytes=k)
        torch.cuda.synchronize()
        for t, (cols, sc) in zip(texts, res):
            s = sc.cpu().numpy().view(np.uint64)
            alone = gpu_parse(p, t, chunk_bytes=k)
            assert np.array_equal(cols.cpu().numpy().view(np.uint64), alone[0])
            assert (bool(s[0]), int(s[1]), int(s[2]), int(s[3])) == alone[1:] + (alone.countp,)
            assert int(s[2]) == 0 and (int(s[1]), int(s[3])) == tuple(o.parse_full(t)[2:])
    say("batched general chunks ok")


def test_no_anchor_anywhere():
    # every column of a^n holds ten segments: no chunk has an anchor, and the
    # count is one walk over the whole text; 10^n mod 2^64 (zero once 2^n
    # divides it)
    device()
    p = S.Parser("(a|a|a|a|a|a|a|a|a|a)*")
    for n in (1, 5, 19, 64, 700, 3000):
        for k in (64, 0):
            g = gpu_parse(p, b"a" * n, chunk_bytes=k)
            _, acc, cnt, st = g
            assert acc and st == 0
            assert cnt == pow(10, n, 1 << 64) and g.countp == pow(10, n, P61), (n, k)
    say("no-anchor walks ok")


def test_column_unambiguous_res_one_tree():
    # REs whose clean columns are always singletons: one tree per accepted
    # text, counted without re-running the automata; empty texts, rejected
    # texts, chunk sizes and batching
    import torch
    device()
    rng = np.random.default_rng(31)
    for pat, alpha in (("(ab|cd)*e", b"abcde"), ("(a|b)*c(d|e)+", b"abcde"), ("x(yz)*", b"xyz"), ("(ab|a)*", b"ab")):
        p, o = S.Parser(pat), Oracle(pat)
        assert column_unambiguous(o), pat
        assert p.info.column_unambiguous == 1, pat   # the library skips the count walk for it
        texts = [b"", b"e", b"ab" * 700 + b"e", b"cd" * 3000 + b"ab" + b"e", b"abab" + b"x" + b"e", b"x", b"xyz" * 900,
                 b"ab" * 40 + b"c" + b"d" * 2000, b"c" + b"e" * 5000]
        texts += [bytes(rng.choice(list(alpha), int(rng.integers(1, 3000)))) for _ in range(4)]
        texts += [b"a" * 5000, b"ab" * 1500 + b"a" * 64]
        for t in texts:
            _, acc, want = o.parse(t)
            assert want == (1 if acc else 0)
            for k in (64, 256, 0):
                g = gpu_parse(p, t, chunk_bytes=k)
                _, a2, cnt, st = g
                assert (a2, cnt, st, g.countp) == (acc, want, 0, want), (pat, len(t), k, a2, cnt, st)
        dts = [to_device(t) for t in texts]
        for k in (64, 0):
            res = p.parse_batch(dts, chunk_bytes=k)
            torch.cuda.synchronize()
            for t, (cols, sc) in zip(texts, res):
                s = sc.cpu().numpy().view(np.uint64)
                alone = gpu_parse(p, t, chunk_bytes=k)
                assert np.array_equal(cols.cpu().numpy().view(np.uint64), alone[0])
                assert (bool(s[0]), int(s[1]), int(s[2]), int(s[3])) == alone[1:] + (alone.countp,)
    say("column-unambiguous REs ok")


def test_runs_reaching_the_text_end():
    # ambiguous runs that end on the text-end column n (its mark lies outside
    # the 64-column windows), for every text length modulo 64 and run lengths
    # across window and lane-chunk edges; both count moduli against the oracle
    device()
    rng = np.random.default_rng(41)
    for pat in ("(a|ab|b)*b?", "((c+)+(d|dd)?)*"):
        p, o = S.Parser(pat), Oracle(pat)
        alpha = b"ab" if pat.startswith("(a") else b"cd"
        texts = []
        for n in list(range(1, 70)) + [127, 128, 129, 255, 256, 257, 1000, 1024, 1087]:
            t = bytes(rng.choice(list(alpha), n))
            texts.append(t)
            texts.append(t[:max(n - 40, 0)] + alpha[:1] * min(n, 40))   # a long run at the end
        for t in texts:
            _, acc, cnt, cntp = o.parse_full(t)
            for k in (64, 128, 0):
                g = gpu_parse(p, t, chunk_bytes=k)
                assert (g[1], g[2], g[3], g.countp) == (acc, cnt if acc else 0, 0, cntp if acc else 0), \
                    (pat, len(t), k, g[1:], g.countp, acc, cnt, cntp)
    say("runs at the text end ok")


def test_wide_count_equals_oracle():
    # SLPF_PARSE_WIDE_COUNT counts the short runs with 16-segment vectors at
    # once: the same counts as the two-pass default and the oracle, on runs
    # of columns of 1-12 segments (the mixed blocks, and a 4-letter RE whose
    # ambiguous columns mostly hold more than 8 segments)
    device()
    from gen import regen, workloads as wl
    rng = np.random.default_rng(23)
    tree = dict(wl.batched_res(seed=4000))["rand3_a4_d4"]
    for pat in (MIXED_RE, regen.to_re(tree)):
        p, o = S.Parser(pat), Oracle(pat)
        if pat == MIXED_RE:
            blocks = [(b"a", 1, 300), (b"b", 1, 200), (b"c", 1, 400), (b"d", 1, 150), (b"a", 200, 900)]
            texts = [_blocks(rng, blocks, int(rng.integers(1, 12000))) for _ in range(4)]
        else:
            sampler = wl.StarSampler(tree, 7)
            texts = [sampler.text(int(rng.integers(1, 20000)), rng).tobytes() for _ in range(4)]
        for t in texts:
            _, acc, want, wantp = o.parse_full(t)
            for k in (256, 0):
                g = gpu_parse(p, t, chunk_bytes=k, flags=S.PARSE_WIDE_COUNT)
                d = gpu_parse(p, t, chunk_bytes=k)
                assert g[1] == d[1] == acc and g[3] == d[3] == 0, (len(t), k)
                assert (g[2], g.countp) == (d[2], d.countp) == (want, wantp), (pat[:20], len(t), k)
                assert np.array_equal(g[0], d[0])
    say("wide count ok")
