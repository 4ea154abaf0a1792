"""slpf_parse_noalloc (the work buffers in the library's file-scope device
array, nothing allocated) against slpf_parse on the same inputs, through the
C ABI: two calls in a row, the second with a smaller text, plain and compact
SLPF, and the capacity error for a text whose work buffers exceed the array.
"""
import sys

import numpy as np
import pytest

from gen import regen, textgen
from gpu_util import device, to_device

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(p, text, chunk_bytes=0, flags=0):
    import torch
    dev = device()
    t = to_device(text)
    n = len(text)
    shape = (n + 1,) if flags & S.PARSE_COMPACT else (n + 1, p.W)
    c1 = torch.full(shape, -1, dtype=torch.int64, device=dev)
    c2 = torch.full(shape, -2, dtype=torch.int64, device=dev)
    s1 = torch.full((4,), -1, dtype=torch.int64, device=dev)
    s2 = torch.full((4,), -2, dtype=torch.int64, device=dev)
    p.parse_into(t, n, c1, s1, chunk_bytes, flags)
    p.parse_noalloc_into(t, n, c2, s2, chunk_bytes, flags)
    torch.cuda.synchronize()
    return (c1.cpu().numpy().view(np.uint64), s1.cpu().numpy().view(np.uint64),
            c2.cpu().numpy().view(np.uint64), s2.cpu().numpy().view(np.uint64))


def test_noalloc_equals_parse_two_calls():
    device()
    cases = []
    tree = regen.plain_small_re()
    cases.append((regen.to_re(tree), textgen.sample_text(tree, 3, 600000).tobytes(),
                  textgen.sample_text(tree, 4, 70000).tobytes()))
    rt = regen.random_re(23)                                      # the single-RE workload's RE
    big = textgen.sample_text(rt, 23, 1 << 22)
    cases.append((regen.to_re(rt), big.tobytes(), textgen.corrupt(big[:300000], 5, 0.05, (64, 4096)).tobytes()))
    mid = textgen.sample_text(rt, 24, 24 << 20)                   # 24 MiB fits the array
    cases.append((regen.to_re(rt), mid.tobytes(), big[:1000000].tobytes()))
    amb = b"(a|ab|b)*b?"
    cases.append((amb, b"ab" * 300000, b"abb" * 1000 + b"a"))      # long ambiguous runs: the piece kernels
    for pat, first, second in cases:
        p = S.Parser(pat)
        for flags in (0, S.PARSE_COMPACT):
            for text, k in ((first, 0), (second, 128)):             # the second call is smaller
                say("noalloc", pat[:40], len(text), "flags", flags, "k", k)
                c1, s1, c2, s2 = _both(p, text, chunk_bytes=k, flags=flags)
                assert np.array_equal(c1, c2), (pat[:40], len(text), flags)
                assert np.array_equal(s1, s2), (pat[:40], len(text), flags, s1, s2)
                assert int(s1[2]) == 0


def test_noalloc_capacity_error():
    import torch
    dev = device()
    p = S.Parser(regen.to_re(regen.random_re(23)))
    n = 256 << 20                                                  # work buffers beyond 128 MiB
    t = torch.zeros(n, dtype=torch.uint8, device=dev)
    cols = torch.empty((n + 1, p.W), dtype=torch.int64, device=dev)
    sc = torch.empty(4, dtype=torch.int64, device=dev)
    with pytest.raises(S.SlpfError) as e:
        p.parse_noalloc_into(t, n, cols, sc)
    assert e.value.status == S.E_CAPACITY
    del cols, t
    torch.cuda.empty_cache()
    # and a normal call afterwards still works
    c1, s1, c2, s2 = _both(p, b"abc" * 10)
    assert np.array_equal(c1, c2) and np.array_equal(s1, s2)
