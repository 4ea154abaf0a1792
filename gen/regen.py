"""Seeded regular-expression trees and their concrete syntax.

This module holds no part of the parsing method: it only builds RE syntax
trees, prints them in the RE syntax accepted by the library and the oracle,
and answers plain language questions about a tree (can it derive the empty
string, can it derive arbitrarily long strings).  Both the GPU path and the
oracle read the RE strings printed here; neither imports anything else from
this package.

Tree nodes are tuples:
    ('lit', byte)            a terminal
    ('set', bytes)           a character-set terminal: any one of the (sorted,
                             distinct) bytes; printed as [...] or, for every
                             byte but the newline, as the wildcard '.'
    ('eps',)                 the empty string
    ('cat', [child, ...])    concatenation, arity >= 2
    ('alt', [child, ...])    union, arity >= 2
    ('star', child) ('plus', child) ('opt', child)

The RE syntax (shared by both parsers): bytes are literals; the metacharacters
are ( ) | * + ? . [ ]; a backslash escapes the next byte, with \\n, \\t and \\xHH as
shorthands; "()" denotes the empty string; [...] is a set of bytes and ranges
(a leading ^ complements it) and '.' any byte but the newline; precedence is iterator, then
concatenation, then union.  A parenthesised operator subexpression stays its
own node (it is never merged into an enclosing operator of the same kind).
"""
from __future__ import annotations

import numpy as np

META = set(b"()|*+?\\.[]")


def lit(ch):
    return ('lit', ch if isinstance(ch, int) else ord(ch))


def cat(*xs):
    return ('cat', list(xs))


def alt(*xs):
    return ('alt', list(xs))


def star(x):
    return ('star', x)


def plus(x):
    return ('plus', x)


def opt(x):
    return ('opt', x)


EPS = ('eps',)

WILDCARD = bytes(b for b in range(256) if b != 0x0A)


def cset(members):
    """Character-set terminal over ``members`` (bytes, str or ints)."""
    if isinstance(members, str):
        members = members.encode('latin-1')
    m = bytes(sorted(set(members)))
    assert m, "empty character set"
    return ('set', m)


def crange(lo, hi):
    return cset(range(ord(lo), ord(hi) + 1))


def lit_union(chars):
    """Union of single-byte terminals, one terminal per byte."""
    chars = [c if isinstance(c, int) else ord(c) for c in chars]
    if len(chars) == 1:
        return ('lit', chars[0])
    return ('alt', [('lit', c) for c in chars])


def _lit_bytes(b: int) -> bytes:
    if b in META:
        return b"\\" + bytes([b])
    if b == 0x0A:
        return b"\\n"
    if b == 0x09:
        return b"\\t"
    if 32 <= b < 127:
        return bytes([b])
    return b"\\x%02x" % b


def _set_byte(b: int) -> bytes:
    if (0x30 <= b <= 0x39) or (0x41 <= b <= 0x5A) or (0x61 <= b <= 0x7A):
        return bytes([b])
    return b"\\x%02x" % b


def _set_bytes(m: bytes) -> bytes:
    """[...] text of a byte set: maximal runs of consecutive bytes as ranges."""
    if m == WILDCARD:
        return b"."
    out, i = b"[", 0
    while i < len(m):
        j = i
        while j + 1 < len(m) and m[j + 1] == m[j] + 1:
            j += 1
        out += _set_byte(m[i])
        if j > i:
            out += (b"-" if j > i + 1 else b"") + _set_byte(m[j])
        i = j + 1
    return out + b"]"


def to_re(node) -> bytes:
    """Print a tree in the RE syntax; parsing the result gives back the tree."""
    k = node[0]
    if k == 'lit':
        return _lit_bytes(node[1])
    if k == 'set':
        return _set_bytes(node[1])
    if k == 'eps':
        return b"()"
    if k == 'cat':
        parts = []
        for ch in node[1]:
            s = to_re(ch)
            if ch[0] in ('cat', 'alt'):
                s = b"(" + s + b")"
            parts.append(s)
        return b"".join(parts)
    if k == 'alt':
        parts = []
        for ch in node[1]:
            s = to_re(ch)
            if ch[0] == 'alt':
                s = b"(" + s + b")"
            parts.append(s)
        return b"|".join(parts)
    if k in ('star', 'plus', 'opt'):
        op = {'star': b"*", 'plus': b"+", 'opt': b"?"}[k]
        ch = node[1]
        s = to_re(ch)
        if ch[0] not in ('lit', 'set'):
            s = b"(" + s + b")"
        return s + op
    raise ValueError(k)


def count_ops(node) -> int:
    k = node[0]
    if k in ('lit', 'set', 'eps'):
        return 0
    if k in ('cat', 'alt'):
        return 1 + sum(count_ops(c) for c in node[1])
    return 1 + count_ops(node[1])


def depth(node) -> int:
    k = node[0]
    if k in ('lit', 'set', 'eps'):
        return 0
    if k in ('cat', 'alt'):
        return 1 + max(depth(c) for c in node[1])
    return 1 + depth(node[1])


def nullable(node) -> bool:
    """Can the tree derive the empty string."""
    k = node[0]
    if k in ('lit', 'set'):
        return False
    if k in ('eps', 'star', 'opt'):
        return True
    if k == 'cat':
        return all(nullable(c) for c in node[1])
    if k == 'alt':
        return any(nullable(c) for c in node[1])
    return nullable(node[1])  # plus


def infinitely_ambiguous(node) -> bool:
    """An iterator over a nullable body gives some string infinitely many trees."""
    k = node[0]
    if k in ('lit', 'set', 'eps'):
        return False
    if k in ('cat', 'alt'):
        return any(infinitely_ambiguous(c) for c in node[1])
    if k in ('star', 'plus') and nullable(node[1]):
        return True
    return infinitely_ambiguous(node[1])


def unbounded(node) -> bool:
    """Does the tree contain an iterator, i.e. derive arbitrarily long strings."""
    k = node[0]
    if k in ('lit', 'set', 'eps'):
        return False
    if k in ('star', 'plus'):
        return True
    if k in ('cat', 'alt'):
        return any(unbounded(c) for c in node[1])
    return unbounded(node[1])


def alphabet_of(node) -> set:
    k = node[0]
    if k == 'lit':
        return {node[1]}
    if k == 'set':
        return set(node[1])
    if k == 'eps':
        return set()
    if k in ('cat', 'alt'):
        out = set()
        for c in node[1]:
            out |= alphabet_of(c)
        return out
    return alphabet_of(node[1])


# ---------------------------------------------------------------- random REs

_OP_KINDS = ('cat', 'alt', 'star', 'plus', 'opt')
_OP_WEIGHTS = np.array([0.30, 0.30, 0.15, 0.15, 0.10])


def random_re(seed: int, n_ops: int = 40, max_depth: int = 7,
              alphabet=b"abcdefghijklmnopqrstuvwxyz", root='star',
              arity=(2, 4), max_tries: int = 1000, set_p: float = 0.0):
    """Seeded random RE tree with exactly ``n_ops`` operators and depth <= ``max_depth``.

    The tree is grown from a root operator by turning a uniformly chosen leaf
    (above the depth limit) into an operator with fresh leaf children; operator
    kinds are drawn with weights concat .3, union .3, star .15, plus .15,
    optional .1 and concat/union arity uniform in ``arity``.  Leaves are
    uniform over ``alphabet``; with ``set_p`` > 0 a leaf is instead, with that
    probability, a character set: a uniformly sized random subset (2 or more
    bytes) of ``alphabet``, or one time in eight the wildcard.  Trees that are infinitely ambiguous are
    redrawn (the next attempt uses the same generator stream).  ``root`` fixes
    the root operator kind ('star' makes the language absorb any text length).
    """
    rng = np.random.default_rng(seed)
    alphabet = list(alphabet)
    for _ in range(max_tries):
        t = _grow(rng, n_ops, max_depth, alphabet, root, arity, set_p)
        if t is not None and not infinitely_ambiguous(t):
            return t
    raise RuntimeError("no acceptable random RE for seed %d" % seed)


def _grow(rng, n_ops, max_depth, alphabet, root, arity, set_p=0.0):
    # mutable tree: nodes are lists [kind, payload]; leaves ['lit', b] or ['set', bytes]
    def new_leaf():
        if set_p > 0 and len(alphabet) > 2 and rng.random() < set_p:
            if rng.random() < 0.125:
                return ['set', WILDCARD]
            k = int(rng.integers(2, len(alphabet)))
            pick = rng.choice(len(alphabet), size=k, replace=False)
            return ['set', bytes(sorted(int(alphabet[i]) for i in pick))]
        return ['lit', int(alphabet[rng.integers(len(alphabet))])]

    def make_op(kind):
        if kind in ('cat', 'alt'):
            a = int(rng.integers(arity[0], arity[1] + 1))
            return [kind, [new_leaf() for _ in range(a)]]
        return [kind, new_leaf()]

    kind = root if root else _OP_KINDS[rng.choice(5, p=_OP_WEIGHTS)]
    tree = make_op(kind)
    ops = 1
    while ops < n_ops:
        # collect leaf slots (parent, index, depth)
        slots = []

        def walk(node, d):
            if node[0] in ('cat', 'alt'):
                for i, ch in enumerate(node[1]):
                    if ch[0] in ('lit', 'set'):
                        if d + 1 < max_depth:
                            slots.append((node[1], i))
                    else:
                        walk(ch, d + 1)
            else:
                ch = node[1]
                if ch[0] in ('lit', 'set'):
                    if d + 1 < max_depth:
                        slots.append((node, 1))
                else:
                    walk(ch, d + 1)
        walk(tree, 0)
        if not slots:
            return None
        parent, idx = slots[int(rng.integers(len(slots)))]
        kind = _OP_KINDS[rng.choice(5, p=_OP_WEIGHTS)]
        parent[idx] = make_op(kind)
        ops += 1

    def freeze(node):
        if node[0] in ('lit', 'set'):
            return (node[0], node[1])
        if node[0] in ('cat', 'alt'):
            return (node[0], [freeze(c) for c in node[1]])
        return (node[0], freeze(node[1]))
    return freeze(tree)


# ------------------------------------------------------------ fixed REs

def plain_small_re():
    """(a|ab|b)*(c|bc)+(a|b)* over {a, b, c}."""
    return cat(star(alt(lit('a'), cat(lit('a'), lit('b')), lit('b'))),
               plus(alt(lit('c'), cat(lit('b'), lit('c')))),
               star(alt(lit('a'), lit('b'))))


def motif_re():
    """Union-heavy ambiguous 4-letter motif RE (genomic-style)."""
    A, C, G, T = (lit(x) for x in "ACGT")
    return star(alt(A, C, G, T, cat(A, C), cat(G, T), cat(A, C, G),
                    cat(T, A, alt(A, T)), cat(C, G, plus(C))))


_DIGITS = b"0123456789"
# printable bytes other than '"' plus a few controls: with the digits and
# separators this gives a 128-symbol record alphabet
_QUOTED = bytes(b for b in range(32, 127) if b != 0x22) + bytes(range(1, 9)) + bytes(range(14, 32))


def csv_record_re(ts_digits=(4, 2, 2, 2, 2, 2), min_fields=3, max_fields=8,
                  quoted=_QUOTED, sets=False):
    """CSV-like traffic record RE, all under one star.

    record := timestamp ':' field (',' field){min-1..max-1} [',' '"' q+ '"'] '\\n'
    timestamp is groups of fixed-width digits joined by '-' (then ' ' and ':'
    for the time part); field := digit+; q ranges over ``quoted``.  Every
    digit position and the quoted byte are a union of single-byte terminals,
    or with ``sets`` one character-set terminal each (the same language and
    the same trees, with far fewer segments).
    """
    D = (lambda: cset(_DIGITS)) if sets else (lambda: lit_union(_DIGITS))  # noqa: E731
    Q = cset(quoted) if sets else lit_union(quoted)
    groups = []
    seps = [b'-', b'-', b' ', b':', b':']
    for gi, w in enumerate(ts_digits):
        groups.extend(D() for _ in range(w))
        if gi < len(seps) and gi < len(ts_digits) - 1:
            groups.append(lit(seps[gi][0]))
    field = lambda: plus(D())  # noqa: E731
    # (',' field) repeated: min-1 mandatory then nested optionals
    tail = None
    for _ in range(max_fields - min_fields):
        inner = [lit(','), field()] + ([tail] if tail is not None else [])
        tail = opt(cat(*inner))
    body = groups + [lit(':'), field()]
    for _ in range(min_fields - 1):
        body += [lit(','), field()]
    if tail is not None:
        body.append(tail)
    body.append(opt(cat(lit(','), lit('"'), plus(Q), lit('"'))))
    body.append(lit('\n'))
    return star(cat(*body))


# Field types of the multi-schema record: nested and overlapping byte sets
# (a digit string is an int, a hex string, an alnum string and a token).
RECORD_FIELD_SETS = {
    'int': _DIGITS,
    'word': b"abcdefghijklmnopqrstuvwxyz",
    'alnum': _DIGITS + b"abcdefghijklmnopqrstuvwxyz",
    'hex': _DIGITS + b"abcdef",
    'tok': bytes(b for b in range(33, 127) if b not in (0x2C, 0x22)),
}


def record_schemas(count=14, fields=8, seed=2, types=('int', 'word', 'alnum', 'hex', 'tok')):
    """``count`` distinct seeded schemas: tuples of ``fields`` field-type names."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        s = tuple(types[int(rng.integers(len(types)))] for _ in range(fields))
        if s not in out:
            out.append(s)
    return out


def record_re(schemas=None, quoted=_QUOTED):
    """Multi-schema log record RE, all under one star.

    record := timestamp ':' schema [',' '"' q+ '"'] '\\n'
    timestamp is YYYY-MM-DD HH:MM:SS (one digit set per position); a schema
    is one of ``schemas`` (default ``record_schemas()``): comma-separated
    fields, each a non-empty string over its type's byte set.  The types
    overlap, so which schemas a line can follow is known only field by field,
    and a line may follow several (several syntax trees).
    """
    schemas = record_schemas() if schemas is None else schemas
    D = lambda: cset(_DIGITS)  # noqa: E731
    ts = [D() for _ in range(4)] + [lit('-')] + [D(), D()] + [lit('-')] + [D(), D()] + [lit(' ')]
    ts += [D(), D(), lit(':'), D(), D(), lit(':'), D(), D()]
    alts = []
    for sch in schemas:
        parts = []
        for j, t in enumerate(sch):
            if j:
                parts.append(lit(','))
            parts.append(plus(cset(RECORD_FIELD_SETS[t])))
        alts.append(cat(*parts))
    body = ts + [lit(':'), alt(*alts)]
    body.append(opt(cat(lit(','), lit('"'), plus(cset(quoted)), lit('"'))))
    body.append(lit('\n'))
    return star(cat(*body))
