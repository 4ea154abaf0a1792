"""Parity at the benchmark's full size and launch configuration.

The single-RE large-text workload (random RE seed 23, 256 MiB text, with and
without the 5 % corruption blocks) is parsed by the HIP path with the
benchmark's automatic chunking.  The accept flag and the tree count modulo
2^64 and modulo 2^61 - 1 must equal the values the oracle's DFA-lookup
serial parser computed over the whole text (tests/golden/full_size_counts.yaml,
written by make_full_size_goldens.py; the text's hash is checked first).  On
the clean text the count is 0 modulo 2^64 but not modulo 2^61 - 1.  The
oracle also runs here without the count and returns sampled column windows
(text start and end, lane-chunk edges, random interior positions), which must
equal the GPU's bit for bit; the same windows of the compact SLPF
(SLPF_PARSE_COMPACT) must equal the oracle's index words.
"""
import hashlib
import os

import numpy as np
import pytest
import yaml

from gen import regen, textgen
from oracle.oracle import Oracle

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu

N = 1 << 28
WIN = 96
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_counts.yaml")


def golden(name, pat, text):
    with open(GOLDEN) as f:
        g = yaml.safe_load(f)[name]
    assert g["re_sha256"] == hashlib.sha256(pat).hexdigest(), "the RE differs from the golden's"
    assert g["text_bytes"] == text.size and g["text_sha256"] == hashlib.sha256(text.tobytes()).hexdigest(), \
        "the generated text differs from the golden's"
    return g


@pytest.fixture(scope="module")
def workload():
    tree = regen.random_re(23)
    pat = regen.to_re(tree)
    clean = textgen.sample_text(tree, 23, N)
    bad = textgen.corrupt(clean, 24, frac=0.05, block=(64, 4096))
    return pat, clean, bad


@pytest.mark.parametrize("which", ["corrupted", "clean"])
def test_full_size_sampled_windows(workload, which):
    import torch
    pat, clean, bad = workload
    text = bad if which == "corrupted" else clean
    n = text.size
    p = S.Parser(pat)
    t = torch.from_numpy(text).to("cuda:0")
    cols, sc = p.parse(t)
    torch.cuda.synchronize()
    s = 1024
    rng = np.random.default_rng(5)
    starts = sorted({0, n + 1 - WIN, s - WIN // 2, 7 * s - 3, (n // s // 2) * s - 1,
                     *[int(x) for x in rng.integers(0, n + 1 - WIN, size=6)]})
    o = Oracle(pat)
    win, acc, _, _ = o.parse_dfa_full(text, starts, WIN, count=False)
    g = golden("single_re_" + which, pat, text)
    sc = sc.cpu().numpy().view(np.uint64)
    assert bool(sc[0]) == acc == g["accepted"] == (which == "clean")
    assert int(sc[2]) == 0
    assert (int(sc[1]), int(sc[3])) == (g["trees_mod_2_64"], g["trees_mod_2_61_1"])
    if which == "clean":
        assert g["trees_mod_2_61_1"] != 0                # a check that can fail
    for k, st in enumerate(starts):
        g = cols[st:st + WIN].cpu().numpy().view(np.uint64)
        assert np.array_equal(g, win[k]), "window at column %d" % st
    del cols
    torch.cuda.empty_cache()
    # the compact SLPF of the same parse: each sampled column as the index
    # word over its candidate list (the oracle's candidates)
    cmp, sc2 = p.parse_compact(t)
    torch.cuda.synchronize()
    assert np.array_equal(sc2.cpu().numpy().view(np.uint64), sc)
    cand = {}
    for k, st in enumerate(starts):
        g = cmp[st:st + WIN].cpu().numpy().view(np.uint64)
        for u in range(WIN):
            r = st + u
            key = (int(text[r - 1]) if r > 0 else None, int(text[r]) if r < n else None)
            if key not in cand:
                cand[key] = {s_: j for j, s_ in enumerate(o.candidates(*key))}
            want = 0
            for s_ in o.to_set(win[k][u]):
                want |= 1 << cand[key][s_]
            assert int(g[u]) == want, "compact column %d" % r
    del cmp
    torch.cuda.empty_cache()
