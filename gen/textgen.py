"""Seeded texts drawn from the language of an RE tree (no parsing method here).

A text is produced by a random walk over the RE syntax tree: at a union every
branch is equally likely, an iterator takes another iteration with
probability ``p_continue`` (0.7), an optional part is taken with probability
one half.  To reach a length budget the walk gives the budget to the
iterators that can absorb it (a uniformly random split between the absorbing
children of a concatenation, a uniformly chosen absorbing branch of a union);
an iterator holding a budget keeps drawing independent iterations of its body
until the budget is met.  For long budgets the iterations are drawn i.i.d.
from a pool of independently walked body samples.  Every text is therefore a
string of the RE's language.
"""
from __future__ import annotations

import numpy as np

from .regen import unbounded

P_CONTINUE = 0.7
P_OPTIONAL = 0.5
POOL = 4096
POOL_THRESHOLD = 1 << 16


def sample_natural(node, rng, p_continue=P_CONTINUE, out=None) -> bytearray:
    """One unbudgeted random derivation of ``node``."""
    if out is None:
        out = bytearray()
    k = node[0]
    if k == 'lit':
        out.append(node[1])
    elif k == 'set':
        out.append(node[1][int(rng.integers(len(node[1])))])
    elif k == 'eps':
        pass
    elif k == 'cat':
        for c in node[1]:
            sample_natural(c, rng, p_continue, out)
    elif k == 'alt':
        sample_natural(node[1][int(rng.integers(len(node[1])))], rng, p_continue, out)
    elif k == 'star':
        while rng.random() < p_continue:
            sample_natural(node[1], rng, p_continue, out)
    elif k == 'plus':
        sample_natural(node[1], rng, p_continue, out)
        while rng.random() < p_continue:
            sample_natural(node[1], rng, p_continue, out)
    elif k == 'opt':
        if rng.random() < P_OPTIONAL:
            sample_natural(node[1], rng, p_continue, out)
    else:
        raise ValueError(k)
    return out


def _iterations(body, rng, budget, p_continue, out: list):
    """Append i.i.d. body derivations to ``out`` until ``budget`` bytes."""
    if budget <= POOL_THRESHOLD:
        got = 0
        while got < budget:
            s = bytes(sample_natural(body, rng, p_continue))
            out.append(s)
            got += len(s)
        return
    pool = [bytes(sample_natural(body, rng, p_continue)) for _ in range(POOL)]
    lens = np.array([len(s) for s in pool], dtype=np.int64)
    mean = max(float(lens.mean()), 1.0)
    got = 0
    while got < budget:
        m = int((budget - got) / mean * 1.02) + 64
        idx = rng.integers(0, POOL, size=m)
        cl = np.cumsum(lens[idx])
        cut = int(np.searchsorted(cl, budget - got)) + 1
        cut = min(cut, m)
        out.extend(pool[i] for i in idx[:cut].tolist())
        got += int(cl[cut - 1])


def _budgeted(node, rng, budget, p_continue, out: list):
    k = node[0]
    if budget <= 0 or not unbounded(node):
        out.append(bytes(sample_natural(node, rng, p_continue)))
        return
    if k == 'cat':
        absorbing = [i for i, c in enumerate(node[1]) if unbounded(c)]
        shares = rng.dirichlet(np.ones(len(absorbing))) * budget
        share = dict(zip(absorbing, shares))
        for i, c in enumerate(node[1]):
            if i in share:
                _budgeted(c, rng, int(round(share[i])), p_continue, out)
            else:
                out.append(bytes(sample_natural(c, rng, p_continue)))
    elif k == 'alt':
        absorbing = [c for c in node[1] if unbounded(c)]
        _budgeted(absorbing[int(rng.integers(len(absorbing)))], rng, budget, p_continue, out)
    elif k == 'opt':
        _budgeted(node[1], rng, budget, p_continue, out)
    elif k in ('star', 'plus'):
        body = node[1]
        if unbounded(body) and budget > POOL_THRESHOLD:
            _iterations(body, rng, budget, p_continue, out)
        elif unbounded(body):
            got = 0
            while got < budget:
                part = []
                _budgeted(body, rng, min(budget - got, 4096), p_continue, part)
                s = b"".join(part)
                out.append(s)
                got += len(s)
                if not s:
                    break
        else:
            _iterations(body, rng, budget, p_continue, out)
    else:
        raise ValueError(k)


def sample_text(node, seed: int, target: int, p_continue=P_CONTINUE) -> np.ndarray:
    """A string of L(node) of length close to (and normally not below) ``target``."""
    rng = np.random.default_rng(seed)
    out: list = []
    _budgeted(node, rng, target, p_continue, out)
    return np.frombuffer(b"".join(out), dtype=np.uint8).copy()


def star_stream(node, seed: int, target: int, p_continue=P_CONTINUE):
    """For a tree whose root is a star: a stream of i.i.d. body derivations.

    Returns (text, bounds) where ``bounds`` are the iteration boundaries
    (0 = b_0 < b_1 < ... = len(text)); any run of consecutive iterations is a
    string of the language.
    """
    assert node[0] in ('star', 'plus')
    rng = np.random.default_rng(seed)
    out: list = []
    _iterations(node[1], rng, target, p_continue, out)
    lens = np.fromiter((len(s) for s in out), dtype=np.int64, count=len(out))
    bounds = np.concatenate([[0], np.cumsum(lens)])
    return np.frombuffer(b"".join(out), dtype=np.uint8).copy(), bounds


def corrupt(text: np.ndarray, seed: int, frac=0.05, block=(64, 4096)) -> np.ndarray:
    """Overwrite about ``frac`` of the bytes with seeded random-byte blocks.

    Block lengths are uniform in ``block`` (inclusive), offsets uniform, bytes
    uniform over 0..255.  Returns a new array.
    """
    rng = np.random.default_rng(seed)
    t = text.copy()
    n = t.size
    if n == 0:
        return t
    want = int(frac * n)
    done = 0
    while done < want:
        ln = int(rng.integers(block[0], block[1] + 1))
        ln = min(ln, n)
        off = int(rng.integers(0, n - ln + 1))
        t[off:off + ln] = rng.integers(0, 256, size=ln, dtype=np.uint8)
        done += ln
    return t


_DIGITS = np.frombuffer(b"0123456789", dtype=np.uint8)


def _pooled(recs, rng, target):
    """A text of i.i.d. records from the pool ``recs``, at least ``target`` bytes."""
    pool = len(recs)
    lens = np.array([len(r) for r in recs], dtype=np.int64)
    m = int(target / lens.mean() * 1.02) + 16
    idx = rng.integers(0, pool, size=m)
    cl = np.cumsum(lens[idx])
    cut = min(int(np.searchsorted(cl, target)) + 1, m)
    return np.frombuffer(b"".join(recs[i] for i in idx[:cut].tolist()), dtype=np.uint8).copy()


def record_text(seed: int, target: int, schemas=None, field_len=(1, 12), quoted=None,
                p_quoted=0.5, pool=65536) -> np.ndarray:
    """Records of the multi-schema record RE (see ``regen.record_re``).

    Timestamp digits uniform; the schema uniform over ``schemas``; every field
    of length uniform in ``field_len`` with bytes uniform over its type's
    set; the quoted field present with ``p_quoted``, length uniform in
    ``field_len``.  Records are drawn i.i.d. from a pool.
    """
    from .regen import _QUOTED, RECORD_FIELD_SETS, record_schemas
    schemas = record_schemas() if schemas is None else schemas
    q = np.frombuffer(quoted if quoted is not None else _QUOTED, dtype=np.uint8)
    sets = {k: np.frombuffer(v, dtype=np.uint8) for k, v in RECORD_FIELD_SETS.items()}
    rng = np.random.default_rng(seed)
    recs = []
    for _ in range(pool):
        d = _DIGITS[rng.integers(0, 10, size=14)].tobytes()
        r = bytearray(d[:4] + b"-" + d[4:6] + b"-" + d[6:8] + b" " + d[8:10] + b":" + d[10:12] + b":" + d[12:14] + b":")
        sch = schemas[int(rng.integers(len(schemas)))]
        for j, t in enumerate(sch):
            if j:
                r.append(0x2c)
            ln = int(rng.integers(field_len[0], field_len[1] + 1))
            r += sets[t][rng.integers(0, sets[t].size, size=ln)].tobytes()
        if rng.random() < p_quoted:
            ln = int(rng.integers(field_len[0], field_len[1] + 1))
            r += b',"' + q[rng.integers(0, q.size, size=ln)].tobytes() + b'"'
        r.append(0x0a)
        recs.append(bytes(r))
    return _pooled(recs, rng, target)


def csv_record_text(seed: int, target: int, ts_digits=(4, 2, 2, 2, 2, 2),
                    min_fields=3, max_fields=8, field_len=(1, 12),
                    quoted=None, p_quoted=0.5, pool=65536) -> np.ndarray:
    """Records of the CSV-like record RE (see ``regen.csv_record_re``).

    Field count uniform in [min_fields, max_fields], digit-field lengths
    uniform in ``field_len``, the quoted field present with ``p_quoted`` and
    its length uniform in ``field_len``.  Records are drawn i.i.d. from a pool.
    """
    from .regen import _QUOTED
    q = np.frombuffer(quoted if quoted is not None else _QUOTED, dtype=np.uint8)
    rng = np.random.default_rng(seed)
    seps = b"-- ::"
    recs = []
    for _ in range(pool):
        r = bytearray()
        for gi, w in enumerate(ts_digits):
            r += bytes(_DIGITS[rng.integers(0, 10, size=w)])
            if gi < len(ts_digits) - 1:
                r.append(seps[gi])
        r.append(0x3a)
        nf = int(rng.integers(min_fields, max_fields + 1))
        for f in range(nf):
            if f:
                r.append(0x2c)
            ln = int(rng.integers(field_len[0], field_len[1] + 1))
            r += bytes(_DIGITS[rng.integers(0, 10, size=ln)])
        if rng.random() < p_quoted:
            ln = int(rng.integers(field_len[0], field_len[1] + 1))
            r += b',"' + bytes(q[rng.integers(0, q.size, size=ln)]) + b'"'
        r.append(0x0a)
        recs.append(bytes(r))
    return _pooled(recs, rng, target)
