"""The record-shaped RE: CSV-like traffic records under one star over a
128-symbol byte alphabet.  Its forward and reverse tables (618 and 869
states, 123 byte classes) are too large for LDS, so every kernel reads them
in place through the caches (the L2 placement).  Bit-exact against the
oracle on whole 2 MiB texts (clean and with corruption blocks, at several
lane-chunk sizes), and on sampled windows of a 64 MiB text with the
automatic chunking.
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


@pytest.fixture(scope="module")
def record():
    pat = regen.to_re(regen.record_re())
    return pat, S.Parser(pat), Oracle(pat)


def test_record_tables_are_l2_resident(record):
    device()
    pat, p, o = record
    assert p.info.placement == 1
    assert p.info.fwd_states > 500 and p.info.num_classes > 100
    assert p.segments == o.segments


@pytest.fixture(scope="module")
def record_texts(record):
    pat, p, o = record
    text = textgen.record_text(41, 2 << 20)
    out = []
    for name, t in (("clean", text), ("corrupted", textgen.corrupt(text, 42, frac=0.02, block=(8, 512)))):
        out.append((name, t, o.parse(t.tobytes())))
    return out


@pytest.mark.parametrize("chunk", [0, 256, 4096])
def test_record_text_whole(record, record_texts, chunk):
    device()
    pat, p, o = record
    for name, t, (cols, acc, cnt) in record_texts:
        say("record", name, t.size, "chunk", chunk)
        g = gpu_parse(p, to_device(t.tobytes()), chunk_bytes=chunk)
        bad = np.nonzero((g[0] != cols).any(axis=1))[0]
        assert bad.size == 0, "first differing column %d" % bad[0]
        assert g[1] == acc == (name == "clean")
        assert g[3] == 0 and g[2] == cnt


def test_record_large_sampled_windows(record):
    import torch
    device()
    pat, p, o = record
    text = textgen.record_text(43, 1 << 26)
    n = text.size
    t = torch.from_numpy(text).to("cuda:0")
    cols, sc = p.parse(t)
    torch.cuda.synchronize()
    win = 64
    s = p.num_chunks(n) and (n + p.num_chunks(n) - 1) // p.num_chunks(n)
    rng = np.random.default_rng(9)
    starts = sorted({0, n + 1 - win, s - win // 2, 5 * s - 1, *[int(x) for x in rng.integers(0, n + 1 - win, size=6)]})
    w, acc, cnt = o.parse_dfa(text, starts, win)
    scn = sc.cpu().numpy().view(np.uint64)
    assert bool(scn[0]) == acc and acc
    assert int(scn[2]) == 0 and int(scn[1]) == cnt
    for k, st in enumerate(starts):
        g = cols[st:st + win].cpu().numpy().view(np.uint64)
        assert np.array_equal(g, w[k]), "window at column %d" % st
    del cols
    torch.cuda.empty_cache()
