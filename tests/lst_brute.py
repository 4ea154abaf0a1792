"""Brute-force enumeration of linearized syntax trees (test helper).

Independent of the oracle and of the library: it reads the RE itself, numbers
it in left-to-right preorder (Sect. 2.2 of arXiv 2503.06763) and, for a given
string, enumerates every syntax tree as its LST (Sect. 2.1: a concatenation
takes all children, a union one, a star zero or more copies, a cross one or
more, an optional part zero or one).  Factoring an LST after each terminal and
after the end mark gives its segments (Sect. 2.3.2), so the clean SLPF column
r is the set of r-th segments over all LSTs, and the number of trees is the
number of LSTs.  Exponential; for tiny inputs only.
"""
from __future__ import annotations

META = set(b"()|*+?\\.[]")


class Node:
    __slots__ = ("kind", "byte", "kids", "num", "members", "form")

    def __init__(self, kind, byte=None, kids=None, members=None, form="byte"):
        self.kind, self.byte, self.kids, self.num = kind, byte, kids or [], 0
        # a terminal matches the bytes in members; form: "byte", "set" ("[...]") or "dot"
        self.members = members if members is not None else (frozenset([byte]) if byte is not None else None)
        self.form = form


def read_re(s: bytes) -> Node:
    pos = 0

    def peek():
        return s[pos] if pos < len(s) else None

    def alt():
        nonlocal pos
        items = [cat()]
        while peek() == ord('|'):
            pos += 1
            items.append(cat())
        return items[0] if len(items) == 1 else Node('alt', kids=items)

    def cat():
        items = []
        while peek() is not None and peek() not in (ord(')'), ord('|')):
            items.append(rep())
        if not items:
            return Node('eps')
        return items[0] if len(items) == 1 else Node('cat', kids=items)

    def rep():
        nonlocal pos
        x = atom()
        while peek() is not None and peek() in b"*+?":
            k = {ord('*'): 'star', ord('+'): 'plus', ord('?'): 'opt'}[peek()]
            pos += 1
            x = Node(k, kids=[x])
        return x

    def one_byte():
        nonlocal pos
        c = s[pos]
        pos += 1
        if c != ord('\\'):
            return c
        e = s[pos]
        pos += 1
        if e == ord('n'):
            return 10
        if e == ord('t'):
            return 9
        if e == ord('x'):
            v = int(s[pos:pos + 2], 16)
            pos += 2
            return v
        return e

    def bracket():
        nonlocal pos
        pos += 1
        neg = peek() == ord('^')
        if neg:
            pos += 1
        got = set()
        first = True
        while True:
            if peek() is None:
                raise SyntaxError(pos)
            if peek() == ord(']') and not first:
                pos += 1
                break
            first = False
            lo = one_byte()
            hi = lo
            if peek() == ord('-') and pos + 1 < len(s) and s[pos + 1] != ord(']'):
                pos += 1
                hi = one_byte()
            got.update(range(lo, hi + 1))
        if neg:
            got = set(range(256)) - got
        if not got:
            raise SyntaxError(pos)
        return Node('lit', members=frozenset(got), form="set")

    def atom():
        nonlocal pos
        c = peek()
        if c is None or c in b")|*+?":
            raise SyntaxError(pos)
        if c == ord('['):
            return bracket()
        if c == ord('.'):
            pos += 1
            return Node('lit', members=frozenset(set(range(256)) - {10}), form="dot")
        if c == ord('('):
            pos += 1
            if peek() == ord(')'):
                pos += 1
                return Node('eps')
            x = alt()
            if peek() != ord(')'):
                raise SyntaxError(pos)
            pos += 1
            return x
        pos += 1
        if c == ord('\\'):
            e = s[pos]
            pos += 1
            if e == ord('n'):
                c = 10
            elif e == ord('t'):
                c = 9
            elif e == ord('x'):
                c = int(s[pos:pos + 2], 16)
                pos += 2
            else:
                c = e
        return Node('lit', byte=c)

    root = alt()
    if pos != len(s):
        raise SyntaxError(pos)
    counter = [0]

    def number(x):
        counter[0] += 1
        x.num = counter[0]
        for k in x.kids:
            number(k)
    number(root)
    return root


def _set_text(members) -> str:
    """Maximal ranges of the set: one byte, two bytes, or lo-hi; letters and
    digits as themselves, other bytes as \\xHH."""
    def one(b):
        return chr(b) if (48 <= b <= 57) or (65 <= b <= 90) or (97 <= b <= 122) else "\\x%02x" % b
    out, bs, k = [], sorted(members), 0
    while k < len(bs):
        e = k
        while e + 1 < len(bs) and bs[e + 1] == bs[e] + 1:
            e += 1
        lo, hi = bs[k], bs[e]
        out.append(one(lo) if lo == hi else one(lo) + one(hi) if hi == lo + 1 else one(lo) + "-" + one(hi))
        k = e + 1
    return "[" + "".join(out) + "]"


def _tok_leaf(x: Node) -> str:
    if x.kind == 'eps':
        return "ε%d" % x.num
    if x.form == "dot":
        return ".%d" % x.num
    if x.form == "set":
        return "%s%d" % (_set_text(x.members), x.num)
    b = x.byte
    if (97 <= b <= 122) or (65 <= b <= 90):
        return "%s%d" % (chr(b), x.num)
    return "\\x%02x%d" % (b, x.num)


def _derive(x: Node, text: bytes, i: int):
    """All (j, lst) such that x derives text[i:j] with linearized tree lst."""
    if x.kind == 'lit':
        return [(i + 1, (_tok_leaf(x),))] if i < len(text) and text[i] in x.members else []
    if x.kind == 'eps':
        return [(i, (_tok_leaf(x),))]
    if x.kind == 'cat':
        parts = [(i, ())]
        for k in x.kids:
            parts = [(j2, l1 + l2) for (j1, l1) in parts for (j2, l2) in _derive(k, text, j1)]
        inner = parts
    elif x.kind == 'alt':
        inner = [r for k in x.kids for r in _derive(k, text, i)]
    elif x.kind in ('star', 'plus'):
        inner = []
        frontier = [(i, ())]
        first = True
        while frontier:
            if not first or x.kind == 'star':
                inner.extend(frontier)
            nxt = []
            for (j1, l1) in frontier:
                for (j2, l2) in _derive(x.kids[0], text, j1):
                    if j2 == j1:
                        raise ValueError("iterator over a nullable body")
                    nxt.append((j2, l1 + l2))
            frontier = nxt
            first = False
    elif x.kind == 'opt':
        inner = [(i, ())] + _derive(x.kids[0], text, i)
    else:
        raise ValueError(x.kind)
    o, c = "%d(" % x.num, ")%d" % x.num
    return [(j, (o,) + l + (c,)) for (j, l) in inner]


def lsts(re: bytes, text: bytes):
    """Every LST of ``text`` (list of symbol tuples, without the end mark)."""
    root = read_re(re)
    return [l for (j, l) in _derive(root, text, 0) if j == len(text)]


def is_end_letter(tok: str) -> bool:
    return not (tok.endswith("(") or tok.startswith(")") or tok.startswith("ε"))


def leaf_number(tok: str) -> int:
    """The node number printed at the end of a leaf token (a terminal or an
    epsilon, in the forms ``_tok_leaf`` writes)."""
    if tok.startswith("\\x"):
        return int(tok[4:])                  # "\\x" and two hex digits
    if tok.startswith("["):
        return int(tok[tok.rindex("]") + 1:])
    return int(tok[1:])                      # one letter, ".", or "ε"


def segments_of(lst) -> list:
    """Factor an LST followed by the end mark into its segments."""
    segs, cur = [], []
    for tok in list(lst) + ["⊣"]:
        cur.append(tok)
        if is_end_letter(tok):
            segs.append(" ".join(cur))
            cur = []
    assert not cur
    return segs


def clean_columns(re: bytes, text: bytes):
    """(columns as sets of segment strings, number of trees)."""
    trees = lsts(re, text)
    cols = [set() for _ in range(len(text) + 1)]
    for t in trees:
        segs = segments_of(t)
        assert len(segs) == len(text) + 1
        for r, s in enumerate(segs):
            cols[r].add(s)
    return cols, len(trees)
