"""The record workload: a multi-schema log record RE under one star (a
timestamp, then one of 14 comma-separated schemas of 8 fields whose byte
sets overlap, an optional quoted field).  Its forward and reverse tables
hold 2k-5k states each, with 6 words per column; together they are too
large for LDS, so every kernel reads them in place through the caches (the
L2 placement).  A line may follow several schemas, so the text has many
trees.  Bit-exact against the oracle on whole 2 MiB texts (clean and with
corruption blocks, at several lane-chunk sizes), on sampled windows of a
64 MiB text with the automatic chunking, and at 1 GiB against the oracle's
accept flag and counts over the whole text.
"""
import hashlib
import os
import sys

import numpy as np
import pytest
import yaml

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
    assert 2000 <= p.info.fwd_states <= 5000 and 2000 <= p.info.rev_states <= 5000
    assert p.W <= 8
    assert p.segments == o.segments


@pytest.fixture(scope="module")
def record_texts(record):
    pat, p, o = record
    text = textgen.record_text(41, 2 << 20)
    out = []
    for name, t in (("clean", text), ("corrupted", textgen.corrupt(text, 42, frac=0.02, block=(8, 512)))):
        out.append((name, t, o.parse_full(t.tobytes())))
    return out


@pytest.mark.parametrize("chunk", [0, 256, 4096])
def test_record_text_whole(record, record_texts, chunk):
    device()
    pat, p, o = record
    for name, t, (cols, acc, cnt, cntp) in record_texts:
        say("record", name, t.size, "chunk", chunk)
        g = gpu_parse(p, to_device(t.tobytes()), chunk_bytes=chunk)
        bad = np.nonzero((g[0] != cols).any(axis=1))[0]
        assert bad.size == 0, "first differing column %d" % bad[0]
        assert g[1] == acc == (name == "clean")
        assert g[3] == 0 and g[2] == cnt and g.countp == cntp


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
    # windows and the accept flag (the counts are checked on the whole 2 MiB
    # texts above and on the 1 GiB text below)
    w, acc, _, _ = o.parse_dfa_full(text, starts, win, count=False)
    scn = sc.cpu().numpy().view(np.uint64)
    assert bool(scn[0]) == acc and acc
    assert int(scn[2]) == 0
    for k, st in enumerate(starts):
        g = cols[st:st + win].cpu().numpy().view(np.uint64)
        assert np.array_equal(g, w[k]), "window at column %d" % st
    del cols
    torch.cuda.empty_cache()


def test_record_full_size_sampled_records(record):
    # the record workload at its full size (1 GiB, the benchmark's automatic
    # chunking).  The RE is a star of records that end at the only newline of
    # each, so a run of whole records is a text of the language and its trees
    # are the full text's trees cut at the record boundaries: the oracle's
    # columns of the run, except its first and last column (the star's
    # opening and closing there), must equal the GPU's columns at the same
    # positions
    import torch
    device()
    pat, p, o = record
    text = textgen.record_text(31, 1 << 30)
    n = text.size
    t = torch.from_numpy(text).to("cuda:0")
    cols, sc = p.parse(t)
    torch.cuda.synchronize()
    scn = sc.cpu().numpy().view(np.uint64)
    # accept flag and counts from the oracle's serial parser over the whole
    # text (tests/golden/full_size_counts.yaml, make_full_size_goldens.py)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_counts.yaml")) as f:
        g = yaml.safe_load(f)["record_re"]
    assert g["re_sha256"] == hashlib.sha256(pat).hexdigest()
    assert g["text_bytes"] == n and g["text_sha256"] == hashlib.sha256(text.tobytes()).hexdigest()
    assert int(scn[2]) == 0
    assert (bool(scn[0]), int(scn[1]), int(scn[3])) == (g["accepted"], g["trees_mod_2_64"], g["trees_mod_2_61_1"])
    rng = np.random.default_rng(11)
    cuts = [0] + [int(x) for x in rng.integers(0, n - (1 << 12), size=8)] + [n - (1 << 12)]
    for a0 in cuts:
        # three whole records from the first record start at or after a0
        if a0 == 0:
            a = 0
        else:
            a = a0 + int(np.nonzero(text[a0:a0 + 4096] == 10)[0][0]) + 1
        ends = np.nonzero(text[a:a + 4096] == 10)[0]
        b = a + int(ends[min(2, ends.size - 1)]) + 1
        sub = text[a:b].tobytes()
        oc, acc, cnt = o.parse(sub)
        assert acc and cnt >= 1
        g = cols[a:b + 1].cpu().numpy().view(np.uint64)
        lo = 0 if a == 0 else 1                          # column 0 is the same at the text start
        hi = b - a + 1 if b == n else b - a              # and column n at the text end
        assert np.array_equal(g[lo:hi], oc[lo:hi]), "records %d..%d" % (a, b)
    del cols, t
    torch.cuda.empty_cache()
