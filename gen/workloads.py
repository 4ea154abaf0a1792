"""Seeded synthetic workloads of many REs and texts (batched and served runs).

Only RE trees, texts and arrival schedules: nothing here parses.  An RE is
redrawn with the next seed only when the generator finds no tree of the drawn
shape; nothing is filtered by what a parser accepts.
"""
from __future__ import annotations

import numpy as np

from . import regen, textgen

ALPHA_DNA = b"ACGT"
ALPHA_26 = b"abcdefghijklmnopqrstuvwxyz"
ALPHA_128 = bytes(range(128))


def _depth_ops(rng):
    depth = int(rng.integers(4, 9))            # U[4, 8]
    n_ops = int(rng.integers(max(4, 2 * depth), min(40, 4 * depth - 1) + 1))
    return depth, n_ops


def re_family(seed: int, count: int, alphabets=None):
    """``count`` seeded random REs (cfg2 generator, depth U[4,8]) cycling over
    ``alphabets`` (default: 4 letters, 26 letters, 128 byte values in the
    proportions 5:6:4)."""
    if alphabets is None:
        alphabets = [ALPHA_DNA] * 5 + [ALPHA_26] * 6 + [ALPHA_128] * 4
    out = []
    s = seed
    for i in range(count):
        alpha = alphabets[i % len(alphabets)]
        while True:
            rng = np.random.default_rng(s)
            depth, n_ops = _depth_ops(rng)
            try:
                tree = regen.random_re(s, n_ops=n_ops, max_depth=depth, alphabet=alpha, max_tries=200)
            except RuntimeError:
                tree = None
            s += 1
            if tree is not None:
                break
        out.append(("rand%d_a%d_d%d" % (i, len(alpha), depth), tree))
    return out


def batched_res(seed: int = 4000):
    """16 REs: 15 random ones (5 over ACGT, 6 over 26 letters, 4 over 128
    byte values) and the union-heavy 4-letter motif RE."""
    return re_family(seed, 15) + [("motif", regen.motif_re())]


def served_res(seed: int = 5000):
    """64 REs from the same generator with other seeds (every 16th the motif RE)."""
    res = re_family(seed, 60)
    for k in range(4):
        res.insert(16 * k + 15, ("motif%d" % k, regen.motif_re()))
    return res


def loguniform_lengths(seed: int, count: int, lo: int = 1 << 10, hi: int = 4 << 20):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=count)).astype(np.int64)


def lognormal_lengths(seed: int, count: int, median: int = 1 << 16, sigma: float = 1.5, cap: int = 64 << 20):
    rng = np.random.default_rng(seed)
    x = np.exp(rng.normal(np.log(median), sigma, size=count))
    return np.clip(x, 1, cap).astype(np.int64)


class StarSampler:
    """Texts of a star-rooted RE as runs of i.i.d. body derivations drawn from
    a seeded pool of ``pool`` derivations (any run of body derivations is a
    string of the language).  A text of target length n is the shortest run
    reaching n bytes."""

    def __init__(self, tree, seed: int, pool: int = 4096):
        assert tree[0] == 'star'
        rng = np.random.default_rng(seed)
        items = [bytes(textgen.sample_natural(tree[1], rng)) for _ in range(pool)]
        items = [x for x in items if x] or [bytes(textgen.sample_natural(tree[1], rng))]
        self.lens = np.array([len(x) for x in items], dtype=np.int64)
        self.starts = np.concatenate([[0], np.cumsum(self.lens)[:-1]])
        self.flat = np.frombuffer(b"".join(items), dtype=np.uint8)
        self.mean = float(self.lens.mean())

    def text(self, n: int, rng) -> np.ndarray:
        if n <= 0:
            return np.zeros(0, np.uint8)
        m = int(n / self.mean * 1.1) + 16
        while True:
            idx = rng.integers(0, len(self.lens), size=m)
            cl = np.cumsum(self.lens[idx])
            if cl[-1] >= n:
                break
            m *= 2
        cut = int(np.searchsorted(cl, n)) + 1
        idx = idx[:cut]
        ln = self.lens[idx]
        total = int(ln.sum())
        # gather: byte t of the text comes from flat[starts[idx_j] + (t - offset_j)]
        off = np.concatenate([[0], np.cumsum(ln)[:-1]])
        src = np.repeat(self.starts[idx] - off, ln) + np.arange(total, dtype=np.int64)
        return self.flat[src]


def texts_for(res, lengths, seed: int):
    """One text per length, RE chosen uniformly; each text is in its RE's
    language with length close to (not below) the target."""
    rng = np.random.default_rng(seed)
    which = rng.integers(len(res), size=len(lengths))
    samplers = {}
    out = []
    for j, (r, n) in enumerate(zip(which, lengths)):
        r = int(r)
        if r not in samplers:
            samplers[r] = StarSampler(res[r][1], seed * 7919 + r)
        out.append((r, samplers[r].text(int(n), rng)))
    return out


def poisson_arrivals(seed: int, count: int, rate: float):
    """Arrival times (seconds from 0) of a Poisson process with ``rate`` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
