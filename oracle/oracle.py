"""ORACLE -- test infrastructure only (Python side of the serial CPU oracle).

Loads ``slpf_oracle.c`` (built with gcc into ``liboracle.so`` next to it) and
adds, in plain Python on top of its set primitives, the quantities of the
paper's parallel algorithm (Sect. 3.2: Eq. reacher, joiner, builder, merger)
so that they can be checked against the worked example and against the GPU
library's intermediate results.  Only tests, the smoke check and the
benchmark's CPU-baseline leg import this module.
"""
from __future__ import annotations

import ctypes
import re
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slpf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle (plain gcc -O2, single-threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        vp, u64p, i32p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32)
        L.oracle_compile.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_int,
                                     ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]
        L.oracle_compile.restype = ctypes.c_int
        L.oracle_free.argtypes = [vp]
        for f in ("oracle_num_segments", "oracle_words", "oracle_num_nodes"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = ctypes.c_int
        for f in ("oracle_initial", "oracle_final"):
            getattr(L, f).argtypes = [vp, u64p]
        L.oracle_node_parent.argtypes = [vp, ctypes.c_int]
        L.oracle_node_parent.restype = ctypes.c_int
        L.oracle_folseg.argtypes = [vp, ctypes.c_int, u64p]
        L.oracle_label.argtypes = [vp, ctypes.c_int]
        L.oracle_label.restype = ctypes.c_int
        L.oracle_label_set.argtypes = [vp, ctypes.c_int, u64p]
        L.oracle_segment_text.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
        L.oracle_segment_text.restype = ctypes.c_size_t
        L.oracle_step_fwd.argtypes = [vp, u64p, ctypes.c_int, u64p]
        L.oracle_step_bwd.argtypes = [vp, u64p, ctypes.c_int, u64p]
        L.oracle_parse.argtypes = [vp, ctypes.c_char_p, ctypes.c_uint64, u64p, u64p]
        L.oracle_parse.restype = ctypes.c_int
        L.oracle_parse_dfa.argtypes = [vp, ctypes.c_char_p, ctypes.c_uint64, ctypes.c_int, u64p,
                                       ctypes.c_uint64, u64p, u64p, ctypes.c_int]
        L.oracle_parse_dfa.restype = ctypes.c_int
        L.oracle_powerset.argtypes = [vp, ctypes.c_int, u64p, ctypes.c_int, i32p, ctypes.c_int,
                                      ctypes.c_int, u64p, i32p]
        L.oracle_powerset.restype = ctypes.c_int
        _lib = L
    return _lib


def _leaf_number(tok: str) -> int:
    """Node number of a terminal token of a segment text ("a4", "\\x0a4",
    "[a-e]4", ".4"); -1 for other tokens (parentheses, epsilon, the end mark)."""
    if tok.endswith("(") or tok.startswith(")") or tok.startswith("ε") or tok == "⊣":
        return -1
    if tok.startswith("\\x"):
        return int(tok[4:])
    if tok.startswith("["):
        return int(tok[tok.rindex("]") + 1:])
    return int(tok[1:])


def _u64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


class OracleError(Exception):
    def __init__(self, status, offset=None):
        super().__init__("oracle compile failed: status %d offset %s" % (status, offset))
        self.status = status
        self.offset = offset


STATUS_SYNTAX, STATUS_INF_AMBIG, STATUS_TOO_LARGE = -2, -3, -4
P61 = (1 << 61) - 1          # the second modulus of the tree count


def _bytes(x):
    if isinstance(x, str):
        return x.encode("latin1")
    if isinstance(x, np.ndarray):
        return x.tobytes()
    return bytes(x)


class Oracle:
    """The parser automaton of one RE plus the serial parsers over it."""

    def __init__(self, re, max_segments: int = 1 << 16):
        L = _load()
        b = _bytes(re)
        h = ctypes.c_void_p()
        off = ctypes.c_size_t(0)
        st = L.oracle_compile(b, len(b), max_segments, ctypes.byref(h), ctypes.byref(off))
        if st != 0:
            raise OracleError(st, off.value if st == STATUS_SYNTAX else None)
        self._h = h
        self._L = L
        self.nseg = L.oracle_num_segments(h)
        self.W = L.oracle_words(h)
        self.num_nodes = L.oracle_num_nodes(h)        # RE nodes, numbered 1.. in preorder
        self.segments = [self._seg_text(i) for i in range(self.nseg)]
        # the byte of each end-letter (-2 for a character set, -1 for the end
        # mark) and the set of bytes it matches
        self.labels = [L.oracle_label(h, i) for i in range(self.nseg)]
        self.label_sets = []
        for i in range(self.nseg):
            w = np.zeros(4, np.uint64)
            L.oracle_label_set(h, i, _u64(w))
            self.label_sets.append(frozenset(b for b in range(256) if (int(w[b >> 6]) >> (b & 63)) & 1))
        self.I = self._words(L.oracle_initial)
        self.F = self._words(L.oracle_final)
        self.folseg = []
        for i in range(self.nseg):
            w = np.zeros(self.W, np.uint64)
            L.oracle_folseg(h, i, _u64(w))
            self.folseg.append(self.to_set(w))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.oracle_free(h)
            self._h = None

    def _seg_text(self, i):
        need = self._L.oracle_segment_text(self._h, i, None, 0)
        buf = ctypes.create_string_buffer(need + 1)
        self._L.oracle_segment_text(self._h, i, buf, need + 1)
        return buf.value.decode("utf-8")

    def _words(self, fn):
        w = np.zeros(self.W, np.uint64)
        fn(self._h, _u64(w))
        return self.to_set(w)

    # -- sets <-> words
    def to_words(self, s) -> np.ndarray:
        w = np.zeros(self.W, np.uint64)
        for i in s:
            w[i >> 6] |= np.uint64(1) << np.uint64(i & 63)
        return w

    def to_set(self, w) -> frozenset:
        out = []
        for k, v in enumerate(np.asarray(w, dtype=np.uint64).tolist()):
            while v:
                b = (v & -v).bit_length() - 1
                out.append(64 * k + b)
                v &= v - 1
        return frozenset(out)

    def seg_id(self, text: str) -> int:
        return self.segments.index(text)

    # -- NFA steps (Eq. matrixmul)
    def step_fwd(self, s, a: int) -> frozenset:
        w = self.to_words(s)
        o = np.zeros(self.W, np.uint64)
        self._L.oracle_step_fwd(self._h, _u64(w), a, _u64(o))
        return self.to_set(o)

    def step_bwd(self, s, a: int) -> frozenset:
        w = self.to_words(s)
        o = np.zeros(self.W, np.uint64)
        self._L.oracle_step_bwd(self._h, _u64(w), a, _u64(o))
        return self.to_set(o)

    # -- serial parsers
    def parse_full(self, text):
        """Serial NFA parser (Fig. serialparser): (cols[(n+1), W] uint64,
        accepted, tree count mod 2^64, tree count mod 2^61 - 1)."""
        x = _bytes(text)
        n = len(x)
        cols = np.zeros((n + 1, self.W), np.uint64)
        sc = np.zeros(3, np.uint64)
        self._L.oracle_parse(self._h, x, n, _u64(cols), _u64(sc))
        return cols, bool(sc[0]), int(sc[1]), int(sc[2])

    def parse(self, text):
        """Serial NFA parser (Fig. serialparser): (cols[(n+1), W] uint64, accepted, count mod 2^64)."""
        return self.parse_full(text)[:3]

    def parse_dfa(self, text, win_starts=(), win_len: int = 0):
        """DFA-lookup serial parser; returns (window columns [nwin, win_len, W], accepted, count mod 2^64)."""
        return self.parse_dfa_full(text, win_starts, win_len)[:3]

    def parse_dfa_full(self, text, win_starts=(), win_len: int = 0, count: bool = True):
        """DFA-lookup serial parser; returns (window columns [nwin, win_len, W],
        accepted, count mod 2^64, count mod 2^61 - 1).  count=False skips the
        tree count (both counts 0): the windows and the accept flag only."""
        x = _bytes(text) if not isinstance(text, np.ndarray) else text
        if isinstance(x, np.ndarray):
            n = x.size
            xp = x.ctypes.data_as(ctypes.c_char_p)
        else:
            n = len(x)
            xp = x
        ws = np.ascontiguousarray(np.asarray(win_starts, dtype=np.uint64))
        out = np.zeros((len(ws), max(win_len, 0), self.W), np.uint64)
        sc = np.zeros(3, np.uint64)
        st = self._L.oracle_parse_dfa(self._h, xp, n, len(ws), _u64(ws) if len(ws) else None,
                                      win_len, _u64(out) if out.size else None, _u64(sc), 1 if count else 0)
        if st != 0:
            raise MemoryError("oracle_parse_dfa failed")
        return out, bool(sc[0]), int(sc[1]), int(sc[2])

    def columns(self, text):
        cols, acc, cnt = self.parse(text)
        return [self.to_set(c) for c in cols], acc, cnt

    # -- automata by powerset (Sect. 3.1)
    def powerset(self, seeds, direction: int = 0, alphabet=None, max_states: int = 1 << 20):
        """States (as frozensets, BFS order from the seeds) and transitions
        {(state_index, byte): state_index or None}."""
        if alphabet is None:
            alphabet = sorted(frozenset().union(*self.label_sets)) if self.label_sets else []
        seeds = list(seeds)
        sw = np.stack([self.to_words(s) for s in seeds]) if seeds else np.zeros((0, self.W), np.uint64)
        sw = np.ascontiguousarray(sw)
        al = np.ascontiguousarray(np.asarray(alphabet, dtype=np.int32))
        i32p = ctypes.POINTER(ctypes.c_int32)
        ns = self._L.oracle_powerset(self._h, direction, _u64(sw), len(seeds), al.ctypes.data_as(i32p),
                                     len(alphabet), max_states, None, None)
        if ns < 0:
            raise OracleError(STATUS_TOO_LARGE)
        sets = np.zeros((ns, self.W), np.uint64)
        nxt = np.zeros((ns, len(alphabet)), np.int32)
        self._L.oracle_powerset(self._h, direction, _u64(sw), len(seeds), al.ctypes.data_as(i32p),
                                len(alphabet), max_states, _u64(sets), nxt.ctypes.data_as(i32p))
        states = [self.to_set(s) for s in sets]
        trans = {}
        for i in range(ns):
            for k, a in enumerate(alphabet):
                t = int(nxt[i, k])
                trans[(i, a)] = None if t < 0 else t
        return states, trans

    def dfa(self, alphabet=None):
        """The parser DFA: powerset from I (forward)."""
        return self.powerset([self.I], 0, alphabet)

    def medfa(self, alphabet=None):
        """The multi-entry DFA: powerset from every singleton {q_j} (forward)."""
        return self.powerset([frozenset([j]) for j in range(self.nseg)], 0, alphabet)

    # -- compact SLPF (App. SLPF optimization, SLPF encoding), plain Python
    def candidates(self, prev, nxt):
        """The segments that can sit in a column between byte ``prev`` (None
        at the text start) and byte ``nxt`` (None at the text end), ascending:
        end-letter ``nxt`` (final segments at the end) and a follower of some
        segment labelled ``prev`` (initial segments at the start).  Every
        segment of a clean column follows a segment of the previous column
        through that column's label, and has the next byte as end-letter."""
        if prev is None:
            pool = self.I
        else:
            pool = frozenset().union(*([self.folseg[r] for r in range(self.nseg) if prev in self.label_sets[r]] or
                                       [frozenset()]))
        keep = self.F if nxt is None else frozenset(s for s in range(self.nseg) if nxt in self.label_sets[s])
        return sorted(pool & keep)

    def compact(self, text, cols=None):
        """Column r as one word: bit k set iff the k-th candidate of
        (x_r, x_{r+1}) is in the clean column.  Raises ValueError if a clean
        segment is not a candidate or a candidate index reaches 64."""
        x = _bytes(text)
        n = len(x)
        if cols is None:
            cols = self.parse(x)[0]
        out = np.zeros(n + 1, np.uint64)
        ranks = {}
        for r in range(n + 1):
            key = (x[r - 1] if r > 0 else None, x[r] if r < n else None)
            if key not in ranks:
                ranks[key] = {s: k for k, s in enumerate(self.candidates(*key))}
            rk = ranks[key]
            word = 0
            for s in self.to_set(cols[r]):
                if s not in rk or rk[s] >= 64:
                    raise ValueError("column %d: segment %d outside its candidate list" % (r, s))
                word |= 1 << rk[s]
            out[r] = np.uint64(word)
        return out

    # -- match extraction (Sect. 4, Other functions of the tool: getMatches)
    def group_events(self, g):
        """Per segment, its symbols "g(" / ")g" in order (from the segment text)."""
        o, c = "%d(" % g, ")%d" % g
        return [[t for t in txt.split(" ") if t in (o, c)] for txt in self.segments]

    def matches(self, text, g, cols=None):
        """Sorted (start, end) pairs: some tree has "g(" at position start and
        its matching ")g" at position end.  From each segment of C_r whose
        last g-symbol is an open, follow arcs (followers present in the next
        column) through segments without g-symbols; a segment whose first
        g-symbol is a close ends a match.  "g( .. )g" inside one segment is
        the empty match (r, r)."""
        x = _bytes(text)
        n = len(x)
        if cols is None:
            cols = self.parse(x)[0]
        ev = self.group_events(g)
        opens = {s for s, e in enumerate(ev) if e and e[-1].endswith("(")}
        closes = {s for s, e in enumerate(ev) if e and e[0].startswith(")")}
        empty = {s for s, e in enumerate(ev) if any(e[k].endswith("(") and e[k + 1].startswith(")")
                                                     for k in range(len(e) - 1))}
        C = [self.to_set(c) for c in cols]
        out = []
        for r in range(n + 1):
            if C[r] & empty:
                out.append((r, r))
            f = C[r] & opens
            c = r
            while f and c < n:
                c += 1
                nf = frozenset().union(*[self.folseg[s] for s in f]) & C[c]
                if nf & closes:
                    out.append((r, c))
                f = nf - closes
        return sorted(out)

    def node_parent(self, k: int) -> int:
        """Preorder number of the parent of node k (0 for the root, -1 if none)."""
        return self._L.oracle_node_parent(self._h, k)

    def children(self, text, g, start, end, cols=None):
        """getChildren (Sect. 4.2, match extraction): the matches of the child
        strings of the match (start, end) of node g, as sorted (k, a, b)
        triples: some tree has g's occurrence over (start, end) and, directly
        inside it, the child node k (a node whose parent is g) over (a, b).
        An operator child spans "k(" at a to ")k" at b; a terminal child the
        one byte at a (b = a + 1); an epsilon child (a, a).

        The trees through that occurrence of g are the walks in the clean SLPF
        from a segment at column start whose last g-symbol opens g, through
        segments without g-symbols, to a segment at column end whose first
        g-symbol closes it: the sub-forest is cut from the columns by a
        forward pass and a backward pass.  Inside it, a segment's symbols
        count from its last "g(" at column start and up to its first ")g" at
        column end.  An operator child's matches are then the walks of
        ``matches`` restricted to the sub-forest."""
        x = _bytes(text)
        n = len(x)
        if cols is None:
            cols = self.parse(x)[0]
        C = {c: self.to_set(cols[c]) for c in range(start, end + 1)}
        toks = [t.split(" ") for t in self.segments]
        o, cl = "%d(" % g, ")%d" % g

        def gsyms(s):
            return [t for t in toks[s] if t in (o, cl)]
        i, j = start, end
        S = {}
        if i == j:
            S[i] = {s for s in C[i] if any(a == o and b == cl for a, b in zip(gsyms(s), gsyms(s)[1:]))}
        else:
            F = {i: {s for s in C[i] if gsyms(s) and gsyms(s)[-1] == o}}
            for c in range(i + 1, j + 1):
                nxt = set().union(*[self.folseg[s] for s in F[c - 1]]) & C[c] if F[c - 1] else set()
                closes = {s for s in nxt if gsyms(s) and gsyms(s)[0] == cl}
                F[c] = closes if c == j else nxt - closes
            S[j] = F[j]
            for c in range(j - 1, i - 1, -1):
                S[c] = {s for s in F[c] if self.folseg[s] & S[c + 1]}
        if not S[i]:
            return []

        def bounds(s, c):
            """[lo, hi): the symbols of segment s at column c that lie inside
            g's occurrence."""
            t = toks[s]
            lo, hi = 0, len(t)
            if c == i:
                lo = max(k for k, u in enumerate(t) if u == o) + 1
            if c == j:
                hi = min(k for k, u in enumerate(t) if u == cl and k >= lo)
            return lo, hi

        def portion(s, c):
            lo, hi = bounds(s, c)
            return toks[s][lo:hi]
        kids = [k for k in range(1, self.num_nodes + 1) if self.node_parent(k) == g]
        out = set()
        for k in kids:
            ko, kc = "%d(" % k, ")%d" % k
            for a in range(i, j + 1):
                for s in S[a]:
                    p = portion(s, a)
                    ks = [u for u in p if u in (ko, kc)]
                    if any(u == ko and v == kc for u, v in zip(ks, ks[1:])):
                        out.add((k, a, a))                      # "k( .. )k" inside one segment
                    if ("ε%d" % k) in p:
                        out.add((k, a, a))                      # an epsilon child
                    if bounds(s, a)[1] == len(toks[s]) and _leaf_number(toks[s][-1]) == k:
                        out.add((k, a, a + 1))                  # a terminal child: the end-letter
                f = {s for s in S[a] if [u for u in portion(s, a) if u in (ko, kc)][-1:] == [ko]}
                c = a
                while f and c < j:
                    c += 1
                    nf = set().union(*[self.folseg[s] for s in f]) & S[c]
                    closing = {s for s in nf if [u for u in portion(s, c) if u in (ko, kc)][:1] == [kc]}
                    if closing:
                        out.add((k, a, c))
                    f = nf - closing
        return sorted(out)

    # -- the parallel algorithm's quantities (Sect. 3.2), plain Python
    def run_fwd(self, s, y):
        for a in y:
            s = self.step_fwd(s, a)
        return s

    def run_bwd(self, s, y):
        for a in reversed(y):
            s = self.step_bwd(s, a)
        return s

    def parallel_trace(self, text, k: int):
        """R, R^, J, J^, B, B^, M and C of Eq. reacher/joiner/builder/merger for
        chunks of length k (the last chunk may be shorter).

        Chunks are 1-based as in the paper: y_1..y_c; J[0..c], Jh[1..c+1]
        (index 0 unused); B[r], Bh[r], M[r] indexed by text position r = 1..n.
        """
        x = _bytes(text)
        n = len(x)
        chunks = [x[i:i + k] for i in range(0, n, k)]
        c = len(chunks)
        Q = range(self.nseg)
        R = {(i + 1, j): self.run_fwd(frozenset([j]), y) for i, y in enumerate(chunks) for j in Q}
        Rh = {(i + 1, j): self.run_bwd(frozenset([j]), y) for i, y in enumerate(chunks) for j in Q}
        J = [self.I]
        for i in range(1, c + 1):
            J.append(frozenset().union(*[R[(i, j)] for j in J[i - 1]]))
        Jh = [None] * (c + 2)
        Jh[c + 1] = self.F
        for i in range(c, 0, -1):
            Jh[i] = frozenset().union(*[Rh[(i, j)] for j in Jh[i + 1]])
        B, Bh, M = {}, {}, {}
        for i, y in enumerate(chunks, start=1):
            base = (i - 1) * k
            s = J[i - 1]
            for t, a in enumerate(y, start=1):
                s = self.step_fwd(s, a)
                B[base + t] = s
            s = Jh[i + 1]
            Bh[base + len(y)] = s
            for t in range(len(y) - 1, 0, -1):
                s = self.step_bwd(s, y[t])
                Bh[base + t] = s
            for t in range(1, len(y) + 1):
                M[base + t] = B[base + t] & Bh[base + t]
        C = [J[0] & Jh[1]] + [M[r] for r in range(1, n + 1)]
        return dict(R=R, Rh=Rh, J=J, Jh=Jh, B=B, Bh=Bh, M=M, C=C)
