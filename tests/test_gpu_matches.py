"""Match extraction (slpf_get_matches): for every group of the RE, the
(start, end) pairs found on the GPU over the parsed SLPF equal the oracle's
match walk, which is pinned against brute-force tree enumeration.  Covers
groups that reopen in every star iteration, empty matches, a group spanning
the whole text, rejected texts, the record RE's fields, the capacity error
and bad group numbers.
"""
import sys

import numpy as np
import pytest

from gen import regen, textgen
from gpu_util import device, to_device
from oracle.oracle import Oracle

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def groups_of(p):
    gs = set()
    for i in range(p.nseg):
        for t in p.segment_text(i).split(" "):
            if t.endswith("("):
                gs.add(int(t[:-1]))
    return sorted(gs)


def check(pat, texts, groups=None):
    import torch
    p, o = S.Parser(pat), Oracle(pat)
    gs = groups if groups is not None else groups_of(p)
    for t in texts:
        cols, sc = p.parse(to_device(t))
        torch.cuda.synchronize()
        ocols = o.parse(t)[0]
        assert np.array_equal(cols.cpu().numpy().view(np.uint64), ocols)
        for g in gs:
            got = [tuple(map(int, x)) for x in p.matches(cols, g, capacity=4)]
            want = o.matches(t, g, ocols)
            assert got == want, (pat[:40], len(t), g, got[:5], want[:5])
    return p


def test_matches_small_res():
    device()
    check("(ab|a)*", [b"", b"a", b"abaaba", b"abb", b"aab" * 30])
    check("(a|b|ab)+", [b"abab", b"bab" * 20])
    check("(a|())b", [b"b", b"ab"])
    check("((a|b)*c)+", [b"abcbc", b"c" * 50, b"ab" * 40 + b"c"])
    check("x(y|yz)*(z|zy)*", [b"xyzzy", b"x" + b"yz" * 60])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_random_res(seed):
    device()
    tree = regen.random_re(800 + seed, n_ops=12, max_depth=5, alphabet=b"abc")
    pat = regen.to_re(tree)
    rng = np.random.default_rng(seed)
    texts = [textgen.sample_text(tree, seed * 10 + j, int(rng.integers(1, 3000))).tobytes() for j in range(3)]
    say("matches random", seed, pat[:60])
    check(pat, texts)


def test_matches_record_fields():
    # the CSV record RE's groups over 8 KB of records (fields, records, the star)
    device()
    pat = regen.to_re(regen.csv_record_re())
    x = textgen.csv_record_text(3, 8000).tobytes()
    p = S.Parser(pat)
    gs = groups_of(p)
    check(pat, [x], groups=gs[:12] + gs[-6:])


def test_matches_capacity_and_arguments():
    import torch
    device()
    p = S.Parser("(ab|a)*")
    cols, _ = p.parse(to_device(b"abaaba"))
    torch.cuda.synchronize()
    out = torch.empty((1, 2), dtype=torch.int64, device="cuda:0")
    import ctypes
    cnt = ctypes.c_uint64(0)
    st = p._L.slpf_get_matches(p.handle, cols.data_ptr(), 6, 2, out.data_ptr(), 1, ctypes.byref(cnt), None)
    assert st == S.E_CAPACITY and cnt.value == 4
    assert [int(v) for v in out.cpu().numpy().view(np.uint64)[0]] == [0, 2]
    for g in (0, 10_000):
        st = p._L.slpf_get_matches(p.handle, cols.data_ptr(), 6, g, out.data_ptr(), 1, ctypes.byref(cnt), None)
        assert st == S.E_ARG
    st = p._L.slpf_get_matches(p.handle, None, 6, 2, out.data_ptr(), 1, ctypes.byref(cnt), None)
    assert st == S.E_ARG
